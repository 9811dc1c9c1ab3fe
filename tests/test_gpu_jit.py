"""Plan-specialised (run-time compiled) tile passes against the oracle and
against the runtime-interpreted kernel."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_util import check_close, round_c64, to_dev, to_host

pytestmark = pytest.mark.gpu


def lib():
    import paper_2008_00216_amd as m
    return m


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_jit_grid_matches_oracle_and_interpreter(dtype):
    m = lib()
    c = W.grid_circuit(3, 6, 14, seed=21)        # 18 qubits
    ref = oracle.simulate(c)
    outs = []
    for jit in (1, -1):
        s = m.StateVector(c.n, dtype, opts=m.make_opts(jit=jit))
        s.init("zero")
        s.apply(c)
        got = to_host(s.tensor)[0]
        check_close(got, ref, dtype, f"jit={jit}")
        outs.append(got)
    # both paths run the same op sequence on the same tiles
    assert np.max(np.abs(outs[0] - outs[1])) < (2e-6 if dtype == torch.complex64 else 1e-13)


@pytest.mark.parametrize("dtype,T", [(torch.complex64, 12), (torch.complex128, 12), (torch.complex128, 11)])
def test_jit_idle_waves(dtype, T):
    """512-thread workgroups on tiles with fewer register groups than threads:
    the waves past the last group only move the tile (2^12 amplitudes: 256
    groups, 4 of 8 waves idle in the phases; 2^11: 6 of 8)."""
    m = lib()
    c = W.grid_circuit(3, 6, 14, seed=21)        # 18 qubits
    ref = oracle.simulate(c)
    outs = []
    for jit in (1, -1):
        s = m.StateVector(c.n, dtype, opts=m.make_opts(jit=jit, tile_bits=T, threads=512))
        s.init("zero")
        s.apply(c)
        got = to_host(s.tensor)[0]
        check_close(got, ref, dtype, f"jit={jit} T={T}")
        outs.append(got)
    assert np.max(np.abs(outs[0] - outs[1])) < (2e-6 if dtype == torch.complex64 else 1e-13)


def test_jit_random_circuit_all_ops():
    m = lib()
    n = 17
    ops = ("H", "X", "Y", "Z", "S", "SDG", "T", "TDG", "SQRTX", "SQRTY", "SQRTW", "RX", "RY", "RZ",
           "P", "CZ", "CNOT", "SWAP", "CP")
    c = W.random_circuit(n, 160, 77, ops=ops, mat_k=(2, 3, 4))
    params = W.uniform_params(1, c.n_params, 5)[0]
    psi0 = round_c64(W.random_state(n, 3))
    ref = oracle.simulate(c, params, psi0)
    t = to_dev(psi0, torch.complex64)
    s = m.StateVector(n, torch.complex64, tensor=t, opts=m.make_opts(jit=1))
    s.apply(c, params)
    check_close(to_host(t)[0], ref, torch.complex64, "jit random")


def test_jit_adjoint():
    m = lib()
    n = 16
    c = W.ansatz_circuit(n, 3)
    h = W.ansatz_observable(n)
    th = W.uniform_params(2, c.n_params, 9)
    s = m.StateVector(n, torch.complex64, batch=2, opts=m.make_opts(jit=1))
    s.init("zero")
    e, g = s.adjoint_grad(c, th, h)
    for b in range(2):
        assert abs(e[b] - oracle.energy(c, th[b], h)) < 2e-4
        ref = oracle.grad_param_shift(c, th[b], h, which=list(range(0, c.n_params, 9)))
        np.testing.assert_allclose(g[b][::9], ref, atol=2e-4)


@pytest.mark.parametrize("jit", [1, -1])
def test_permutation_circuits_exact_in_tile_passes(jit):
    """X, Y, CNOT, SWAP with Z, S, CZ: register permutations and sign flips
    only, so the fused sweep (specialised or interpreted) equals the oracle
    exactly (+0 and -0 compare equal)."""
    m = lib()
    n = 17
    c = W.random_circuit(n, 300, 31, ops=("X", "Y", "CNOT", "SWAP", "Z", "S", "SDG", "CZ"))
    psi0 = round_c64(W.random_state(n, 32))
    ref = oracle.simulate(c, None, psi0)
    for dtype in (torch.complex64, torch.complex128):
        t = to_dev(psi0, dtype)
        s = m.StateVector(n, dtype, tensor=t, opts=m.make_opts(jit=jit))
        st = s.apply(c)
        assert st["dense_ops"] == 0
        assert np.array_equal(to_host(t)[0], ref), (jit, dtype)


def test_permutations_in_the_batch_and_adjoint():
    m = lib()
    n = 12
    gates = []
    p = 0
    rng = np.random.default_rng(5)
    for layer in range(6):
        for q in range(n):
            gates.append(W.Gate("RY", (q,), param=p)); p += 1
        for q in range(layer % 2, n - 1, 2):
            gates.append(W.Gate(("CNOT", "SWAP", "CZ")[int(rng.integers(0, 3))], (q, q + 1)))
        gates.append(W.Gate("X", (int(rng.integers(0, n)),)))
        gates.append(W.Gate("Y", (int(rng.integers(0, n)),)))
    c = W.Circuit(n, gates, p, "perm-ansatz")
    h = W.ansatz_observable(n)
    th = W.uniform_params(2, c.n_params, 3)
    s = m.StateVector(n, torch.complex64, batch=2)
    s.init("zero_deferred")
    e, g = s.adjoint_grad(c, th, h)
    circs, params, states, lams = [c, c], [th[0], th[1]], [], []
    for b in range(2):
        states.append(torch.zeros(1 << n, dtype=torch.complex64, device="cuda"))
        lams.append(torch.zeros(1 << n, dtype=torch.complex64, device="cuda"))
    eb, gb, _ = m.apply_batch(circs, params, states, [h, h], lambdas=lams, grad=True)
    for b in range(2):
        ref = oracle.energy(c, th[b], h)
        assert abs(e[b] - ref) < 2e-5 and abs(eb[b] - ref) < 2e-5
        which = list(range(0, c.n_params, 7))
        gref = oracle.grad_param_shift(c, th[b], h, which=which)
        np.testing.assert_allclose(g[b][which], gref, atol=2e-5)
        np.testing.assert_allclose(gb[b][which], gref, atol=2e-5)
