"""The fused planner's algebra on the host: the plan trace evaluated from
its definitions equals the gate-by-gate FP64 oracle (Sec. 4.5 reordering,
Sec. 4.4 butterflies, Sec. 4.3 lazily applied phase forms)."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.trace_eval import apply_pauli_sum, evaluate


def lib():
    m = pytest.importorskip("paper_2008_00216_amd")
    return m


def _check(m, c, params=None, tile_bits=0, psi0=None, tol=1e-12, **kw):
    opts = m.make_opts(tile_bits=tile_bits, **kw)
    tr = m.plan_trace(c, params, opts=opts)
    if psi0 is None:
        psi0 = W.basis_state(c.n, 0)
    got, _ = evaluate(tr, c.n, psi0)
    ref = oracle.simulate(c, params, psi0=psi0)
    assert np.max(np.abs(got - ref)) < tol, tr[:2000]
    return tr


def test_line_circuit_single_pass():
    m = lib()
    c = W.line_circuit(12, 10, seed=1000)
    tr = _check(m, c)
    # every non-diagonal one-qubit gate is one butterfly; T and CZ phases are
    # absorbed into twiddles or applied once at the end
    nbf = sum(1 for g in c.gates if g.op in ("H", "SQRTX", "SQRTY", "SQRTW"))
    assert sum(1 for l in tr.splitlines() if l.startswith("BF ")) == nbf
    assert tr.count("FORM") == 1


@pytest.mark.parametrize("tile_bits", [6, 8, 10])
def test_grid_multi_pass_carried_phases(tile_bits):
    m = lib()
    c = W.grid_circuit(3, 4, 12, seed=77)
    tr = _check(m, c, tile_bits=tile_bits, low_bits=3)
    assert tr.count("PASS") > 1


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_random_mixed_gates(seed):
    m = lib()
    c = W.random_circuit(9, 120, seed=seed, mat_k=(2, 3))
    p = W.uniform_params(1, c.n_params, 50 + seed)[0]
    psi0 = W.random_state(9, seed)
    _check(m, c, p, tile_bits=7, low_bits=3, psi0=psi0)


@pytest.mark.parametrize("n", [4, 5])
def test_states_smaller_than_a_default_tile(n):
    # the tile shrinks to the whole state (one or two register groups)
    m = lib()
    c = W.random_circuit(n, 60, seed=100 + n, mat_k=(1, 2, 3))
    p = W.uniform_params(1, c.n_params, 7)[0]
    _check(m, c, p, psi0=W.random_state(n, 200 + n))


def test_empty_circuit_has_an_empty_plan():
    m = lib()
    info = m.plan_info(W.Circuit(7, []))
    assert info["passes"] == 0 and info["launches"] == 0 and info["gates_in"] == 0


def test_wide_gates_force_flush_before_plain_steps():
    m = lib()
    c = W.random_circuit(8, 80, seed=9, ops=("H", "SQRTX", "SQRTY", "SQRTW", "T", "CZ", "S"), mat_k=(5, 6))
    assert any(g.op == "MAT" and len(g.qubits) >= 5 for g in c.gates)
    _check(m, c, tile_bits=6, low_bits=3, psi0=W.random_state(8, 5))


def test_unstructured_mode_matches_too():
    m = lib()
    c = W.grid_circuit(3, 3, 8, seed=5)
    tr = _check(m, c, tile_bits=6, low_bits=3, structured=0)
    assert "BF" not in tr


def test_adjoint_plan_is_the_inverse_sweep_with_shift_rule_gradients():
    m = lib()
    c = W.random_circuit(8, 90, seed=11, ops=("H", "SQRTX", "SQRTY", "SQRTW", "T", "TDG", "S", "CZ", "RY", "RZ",
                                              "RX", "CP"), param_frac=1.0)
    p = W.uniform_params(1, c.n_params, 12)[0]
    h = W.pauli_sum([(1.0, {0: "Z", 1: "Z"}), (0.5, {2: "X"}), (-0.3, {1: "Y", 3: "Z"})])
    tr = m.plan_trace(c, p, adjoint=True, opts=m.make_opts(tile_bits=6, low_bits=3))
    psi0 = W.random_state(8, 3)
    fwd = oracle.simulate(c, p, psi0=psi0)
    (back, _), grads = evaluate(tr, 8, fwd, apply_pauli_sum(fwd, 8, h))
    # the backward sweep un-computes psi
    assert np.max(np.abs(back - psi0)) < 1e-12
    ref = oracle.grad_param_shift(c, p, h, psi0)
    got = np.array([grads[i] for i in range(c.n_params)])
    np.testing.assert_allclose(got, ref, atol=1e-11)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_dense_block_fusion(k):
    m = lib()
    c = W.random_circuit(9, 150, seed=20 + k, mat_k=(2,))
    p = W.uniform_params(1, c.n_params, 70 + k)[0]
    tr = _check(m, c, p, tile_bits=8, low_bits=3, psi0=W.random_state(9, k), structured=0, max_fuse_k=k)
    widths = [int(l.split()[1]) for l in tr.splitlines() if l.startswith(("DENSE ", "DIAG "))]
    assert max(widths) <= max(k, 2)
    if k >= 3:
        assert max(widths) >= 3


def test_dense_block_fusion_grid_adjoint():
    m = lib()
    c = W.random_circuit(8, 90, seed=33, ops=("H", "SQRTX", "T", "CZ", "RY", "RZ", "CNOT"), param_frac=1.0)
    p = W.uniform_params(1, c.n_params, 34)[0]
    h = W.pauli_sum([(1.0, {0: "Z", 1: "Z"}), (0.5, {2: "X"})])
    tr = m.plan_trace(c, p, adjoint=True, opts=m.make_opts(tile_bits=6, low_bits=3, structured=0, max_fuse_k=3))
    psi0 = W.random_state(8, 4)
    fwd = oracle.simulate(c, p, psi0=psi0)
    (back, _), grads = evaluate(tr, 8, fwd, apply_pauli_sum(fwd, 8, h))
    assert np.max(np.abs(back - psi0)) < 1e-12
    ref = oracle.grad_param_shift(c, p, h, psi0)
    np.testing.assert_allclose([grads[i] for i in range(c.n_params)], ref, atol=1e-11)


def _max_scale_exponent(tr):
    """Largest number of unscaled butterflies at any point of a trace."""
    run = worst = 0
    for line in tr.splitlines():
        if line.startswith("BF "):
            run += 1
            worst = max(worst, run)
        elif line.startswith("SCALE"):
            run = 0
    return worst


def test_scale_factor_applied_inside_long_passes():
    """A whole circuit in one tile pass with hundreds of butterflies: the
    1/sqrt(2) factors are applied whenever 120 (forward) or 60 (adjoint)
    have accumulated, not only at pass ends, and the plan stays exact."""
    m = lib()
    c = W.layered_param_circuit(10, 40, 4021)
    p = W.uniform_params(1, c.n_params, 4022)[0]
    opts = m.make_opts(tile_bits=10, low_bits=4)
    tr = m.plan_trace(c, p, opts=opts)
    assert tr.count("PASS") == 1 and tr.count("BF ") > 240
    assert _max_scale_exponent(tr) <= 120
    got, _ = evaluate(tr, c.n, W.basis_state(c.n, 0))
    assert np.max(np.abs(got - oracle.simulate(c, p))) < 1e-12
    tra = m.plan_trace(c, p, adjoint=True, opts=opts)
    assert _max_scale_exponent(tra) <= 60
    h = W.z_sum(c.n)
    psi0 = W.random_state(c.n, 5)
    fwd = oracle.simulate(c, p, psi0=psi0)
    (back, _), grads = evaluate(tra, c.n, fwd, apply_pauli_sum(fwd, c.n, h))
    assert np.max(np.abs(back - psi0)) < 1e-11
    sel = list(range(0, c.n_params, 37))
    ref = oracle.grad_param_shift(c, p, h, psi0)
    np.testing.assert_allclose([grads[i] for i in sel], ref[sel], atol=1e-10)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_permutation_gates_are_register_permutations(seed):
    """X, Y, CNOT and SWAP run as register permutations (PERM lines), never
    as dense matrices, and the plan still equals the oracle."""
    m = lib()
    ops = ("H", "T", "CZ", "SQRTX", "X", "Y", "CNOT", "SWAP", "S")
    c = W.random_circuit(9, 150, seed=300 + seed, ops=ops)
    psi0 = W.random_state(9, 40 + seed)
    tr = _check(m, c, None, tile_bits=7, low_bits=3, psi0=psi0)
    lines = tr.splitlines()
    nperm = sum(1 for g in c.gates if g.op in ("X", "Y", "CNOT", "SWAP"))
    assert sum(1 for l in lines if l.startswith("PERM ")) == nperm
    assert not any(l.startswith("DENSE ") for l in lines)
    # adjoint plans too (inverse gates in reverse order)
    tr_b = m.plan_trace(c, None, opts=m.make_opts(tile_bits=7, low_bits=3), adjoint=True)
    assert sum(1 for l in tr_b.splitlines() if l.startswith("PERM ")) == nperm


@pytest.mark.parametrize("beam", [1, 2, 8, 32])
def test_beam_searched_local_sets_keep_the_state(beam):
    # Sec. 4.5: any choice of local sets is a valid reordering; the beam
    # search only changes which gates share a pass
    m = lib()
    c = W.grid_circuit(3, 5, 16, seed=91)
    tr = _check(m, c, tile_bits=7, low_bits=3, plan_beam=beam)
    assert tr.count("PASS") > 1
    # 12 passes greedily, 10 with the beam search at width 8
    c2 = W.random_circuit(10, 150, seed=97, mat_k=(2, 3))
    p = W.uniform_params(1, c2.n_params, 93)[0]
    _check(m, c2, p, tile_bits=6, low_bits=2, psi0=W.random_state(10, 94), plan_beam=beam)


def test_beam_search_never_adds_passes():
    m = lib()
    import torch
    cases = [(W.grid_circuit(3, 5, 16, seed=91), 7, 3), (W.grid_circuit(4, 4, 20, seed=95), 8, 3),
             (W.random_circuit(12, 200, seed=96, mat_k=(2, 3)), 7, 3), (W.grid33(), 13, 4)]
    fewer = 0
    for c, tb, lb in cases:
        for dt in (torch.complex64, torch.complex128):
            greedy = m.plan_info(c, dt, opts=m.make_opts(tile_bits=tb, low_bits=lb, plan_beam=1))["passes"]
            for beam in (2, 8, 16):
                p = m.plan_info(c, dt, opts=m.make_opts(tile_bits=tb, low_bits=lb, plan_beam=beam))["passes"]
                assert p <= greedy, (c.n, tb, beam, p, greedy)
                fewer += p < greedy
    # the 3x11 grid of 33 qubits at 2^13-amplitude tiles: 22 greedy passes
    assert m.plan_info(W.grid33(), opts=m.make_opts(tile_bits=13, low_bits=4, plan_beam=8))["passes"] < 22
    assert fewer > 0


@pytest.mark.parametrize("beam", [2, 8])
def test_beam_searched_adjoint_plan_matches_the_oracle(beam):
    m = lib()
    # 6 passes greedily, 5 with the beam search at width 8
    c = W.random_circuit(10, 160, seed=97, ops=("H", "SQRTX", "SQRTY", "T", "S", "CZ", "RY", "RZ", "RX", "CP"),
                         param_frac=1.0)
    p = W.uniform_params(1, c.n_params, 98)[0]
    h = W.pauli_sum([(1.0, {0: "Z", 5: "Z"}), (0.5, {7: "X"}), (-0.3, {2: "Y", 9: "Z"})])
    opts = m.make_opts(tile_bits=6, low_bits=2, plan_beam=beam)
    tr = m.plan_trace(c, p, adjoint=True, opts=opts)
    assert tr.count("PASS") > 1
    if beam == 8:
        greedy = m.plan_info(c, adjoint=True, opts=m.make_opts(tile_bits=6, low_bits=2, plan_beam=1))["passes"]
        assert m.plan_info(c, adjoint=True, opts=opts)["passes"] < greedy
    psi0 = W.random_state(10, 99)
    fwd = oracle.simulate(c, p, psi0=psi0)
    (back, _), grads = evaluate(tr, 10, fwd, apply_pauli_sum(fwd, 10, h))
    assert np.max(np.abs(back - psi0)) < 1e-12
    ref = oracle.grad_param_shift(c, p, h, psi0)
    np.testing.assert_allclose(np.array([grads[i] for i in range(c.n_params)]), ref, atol=1e-11)
