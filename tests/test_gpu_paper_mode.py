"""The paper's own plan as a GPU mode (opts.paper = 1: kind clusters with
one pass per diagonal cluster and per gate pair; 2: plus the recursive
transform's LDS chunks) against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_util import check_close, round_c64, to_dev, to_host

pytestmark = pytest.mark.gpu

DTYPES = [torch.complex64, torch.complex128]
FAMILY = ("H", "SQRTX", "SQRTY", "SQRTXDG", "SQRTYDG", "T", "TDG", "S", "SDG", "Z", "CZ")


def lib():
    import paper_2008_00216_amd as m
    return m


def run(c, psi0, dtype, paper, params=None, batch=1):
    m = lib()
    t = to_dev(psi0, dtype)
    s = m.StateVector(c.n, dtype, batch=batch, tensor=t, opts=m.make_opts(paper=paper))
    st = s.apply(c, params)
    return to_host(t), st


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("paper", [1, 2])
def test_grid_circuit_from_zero(dtype, paper):
    m = lib()
    c = W.grid_circuit(4, 4, 12, seed=41, family=("SQRTX", "SQRTY", "T"))
    s = m.StateVector(c.n, dtype, opts=m.make_opts(paper=paper))
    s.init("zero_deferred")
    st = s.apply(c)
    assert st["folded_init"] == c.n          # the initial H layer became the uniform state
    check_close(to_host(s.tensor)[0], oracle.simulate(c), dtype, f"grid paper={paper}")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("paper", [1, 2])
@pytest.mark.parametrize("n", [5, 9, 13])
def test_random_family_circuits(dtype, paper, n):
    c = W.random_circuit(n, 160, 1000 + n, ops=FAMILY + ("SQRTW", "RX", "RZ", "CNOT", "SWAP", "X"))
    params = W.uniform_params(2, c.n_params, n)
    psi0 = np.stack([round_c64(W.random_state(n, 60 + n + b)) for b in range(2)])
    got, st = run(c, psi0, dtype, paper, params, batch=2)
    for b in range(2):
        check_close(got[b], oracle.simulate(c, params[b], psi0[b]), dtype, f"random n={n} paper={paper} state {b}")


@pytest.mark.parametrize("paper", [1, 2])
def test_rescale_passes_keep_the_state_in_range(paper):
    # 70 layers of H, sqrt(X) and sqrt(Y) on 12 qubits: the scale counter
    # passes 100 many times over
    n = 12
    g = []
    fam = ("H", "SQRTX", "SQRTY")
    rng = np.random.default_rng(3)
    for layer in range(70):
        g += [W.Gate(fam[int(rng.integers(0, 3))], (q,)) for q in range(n)]
        g += [W.Gate("CZ", (q, q + 1)) for q in range(layer % 2, n - 1, 2)]
    c = W.Circuit(n, g, 0, "deep")
    psi0 = round_c64(W.random_state(n, 5))
    got, st = run(c, psi0, torch.complex64, paper)
    assert st["passes"] > 70
    check_close(got[0], oracle.simulate(c, None, psi0), torch.complex64, "deep family circuit")


@pytest.mark.parametrize("n", [6, 11, 16])
def test_sign_and_phase_clusters_exact(n):
    # Z, S, CZ only: +-1 and +-i, applied without rounding
    c = W.random_circuit(n, 120, 77 + n, ops=("Z", "S", "SDG", "CZ"))
    psi0 = round_c64(W.random_state(n, 8))
    got, _ = run(c, psi0, torch.complex64, 1)
    ref = oracle.simulate(c, None, psi0)
    assert np.array_equal(got[0], ref)
