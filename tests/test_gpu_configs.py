"""The gradient workloads at their own sizes against stored FP64 oracle
values (tests/golden/make_config_gradients.py):

* the 20-qubit, 400-parameter ansatz with all 64 parameter sets in one
  adjoint call: energies of sets 0-3 and parameter-shift gradients of 20
  sampled parameters;
* the 512-circuit batch (10-22 qubits): its first 64 circuits in one
  persistent launch, the 21-22-qubit items against stored energies and
  sampled gradients, narrow items against the oracle run here.

Tolerance for an energy or gradient of a complex64 sweep: rounding of each
gate application adds a relative error of about u = 2^-24 to the state, and
these errors add like a random walk over the G gate applications of the
forward and backward sweeps, so ||psi_gpu - psi||_2 ~ sqrt(G) u; a value
<psi|A|psi> with ||A|| <= sum_k |c_k| then moves by at most
2 sum_k |c_k| ||delta||.  The bar is 2 sum_k |c_k| sqrt(G) 2^-23, twice
that model."""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.golden import load as golden

pytestmark = pytest.mark.gpu


def lib():
    import paper_2008_00216_amd as m
    return m


def tol_c64(coeff_l1: float, gates: int) -> float:
    return 2.0 * coeff_l1 * math.sqrt(2 * gates) * 2.0 ** -23


def test_ansatz20_64_sets_against_oracle():
    m = lib()
    c = W.ansatz_circuit(20, 10)
    h = W.ansatz_observable(20)
    th = W.uniform_params(64, c.n_params, 3003)
    sel, en, gr = golden.ansatz20_gradients()
    s = m.StateVector(20, torch.complex64, batch=64)
    s.init("zero_deferred")
    e, g = s.adjoint_grad(c, th, h)
    tol = tol_c64(float(np.abs(h.coeff).sum()), len(c))
    errs_e = [abs(e[b] - en[b]) for b in sorted(en)]
    errs_g = [float(np.max(np.abs(g[b][sel] - gr[b]))) for b in sorted(gr)]
    print(f"ansatz20: tol {tol:.2e}  energy err {max(errs_e):.2e}  grad err {max(errs_g):.2e}")
    assert max(errs_e) <= tol and max(errs_g) <= tol
    # every set's energy is a valid expectation and the sets differ
    assert np.all(np.abs(e) <= np.abs(h.coeff).sum()) and len(set(np.round(e, 6))) > 60


def test_batch_first64_against_oracle():
    m = lib()
    circs = W.batch_circuits(64, 10, 22, 20, 60, seed0=4000)
    params = [W.uniform_params(1, c.n_params, 4000 + i)[0] for i, c in enumerate(circs)]
    obs = [W.z_sum(c.n) for c in circs]
    states = [torch.empty(1 << c.n, dtype=torch.complex64, device="cuda") for c in circs]
    lams = [torch.empty_like(t) for t in states]
    e, g, st = m.apply_batch(circs, params, states, obs, lambdas=lams, grad=True, init_zero=True)
    wide = golden.batch_wide_gradients()
    worst = 0.0
    for i, d in wide.items():
        assert circs[i].n == d["n"] and len(circs[i]) == d["gates"]
        tol = tol_c64(float(circs[i].n), len(circs[i]))
        err = abs(e[i] - d["energy"])
        worst = max(worst, err / tol)
        assert err <= tol, (i, e[i], d["energy"], tol)
        if "grad" in d:
            gerr = float(np.max(np.abs(g[i][d["params"]] - d["grad"])))
            worst = max(worst, gerr / tol)
            print(f"batch item {i} (n={d['n']}): energy err {err:.2e}  grad err {gerr:.2e}  tol {tol:.2e}")
            assert gerr <= tol, (i, gerr, tol)
    # narrow items: the oracle here (energies of all of them, shift-rule
    # gradients of a few parameters of two)
    narrow = [i for i, c in enumerate(circs) if c.n <= 13]
    assert len(narrow) >= 8
    for k, i in enumerate(narrow):
        c = circs[i]
        tol = tol_c64(float(c.n), len(c))
        ref = oracle.energy(c, params[i], obs[i])
        assert abs(e[i] - ref) <= tol, (i, e[i], ref)
        worst = max(worst, abs(e[i] - ref) / tol)
        if k < 2:
            which = list(range(0, c.n_params, max(1, c.n_params // 5)))
            gref = oracle.grad_param_shift(c, params[i], obs[i], which=which)
            assert np.max(np.abs(g[i][which] - gref)) <= tol, i
    print(f"batch: worst error / tolerance {worst:.3f}")
