"""Schroedinger-Feynman mode (sv_sf_*) against the FP64 oracle's full-width
sweep: the path sum over the gates across the cut must give the same
amplitudes as the circuit itself (to the dtype's tolerance), whether the path
bits are held in memory or enumerated from a checkpoint."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_util import check_close

pytestmark = pytest.mark.gpu

DTYPES = [torch.complex64, torch.complex128]


def lib():
    import paper_2008_00216_amd as m
    return m


def column_mask(rows, cols, left):
    return sum(1 << (r * cols + c) for r in range(rows) for c in range(left))


def all_amplitudes(m, circ, mask, dtype, params=None, work=None):
    sim = m.SchrodingerFeynman(circ, mask, dtype, work_bytes=work)
    got, st = sim.amplitudes(np.arange(1 << circ.n, dtype=np.uint64), params)
    info = sim.info
    sim.close()
    return got, st, info


@pytest.mark.parametrize("dtype", DTYPES)
def test_grid_column_cut_all_paths_in_memory(dtype):
    m = lib()
    c = W.grid_circuit(4, 5, 8, seed=31)
    mask = column_mask(4, 5, 2)
    ref = oracle.simulate(c)
    got, st, info = all_amplitudes(m, c, mask, dtype)
    assert info["n_cross"] >= 6 and info["n_outer"] == 0
    check_close(got, ref, dtype, f"S-F grid 4x5, {info['n_cross']} cross gates")


def test_doublings_are_read_by_the_next_pass():
    # every segment after a cross gate is planned with its path qubit local
    # in its first pass, which reads the doubled half from the half with that
    # qubit clear: no doubling copy is launched, and the amplitudes still
    # match the full sweep
    m = lib()
    c = W.grid_circuit(2, 9, 10, seed=33)
    mask = column_mask(2, 9, 4)
    ref = oracle.simulate(c)
    got, st, info = all_amplitudes(m, c, mask, torch.complex64)
    assert info["n_cross"] >= 4 and info["n_outer"] == 0
    extra = st["launches"] - st["passes"]
    print(f"S-F 2x9: {info['n_cross']} cross gates, {st['passes']} passes, {st['launches']} launches")
    assert extra <= 2, f"{extra} launches besides the passes (init and contraction expected)"
    check_close(got, ref, torch.complex64, "S-F 2x9 with fused doublings")


@pytest.mark.parametrize("dtype", DTYPES)
def test_enumerated_path_bits_match(dtype):
    m = lib()
    c = W.grid_circuit(4, 5, 8, seed=32)
    mask = column_mask(4, 5, 3)
    ref = oracle.simulate(c)
    info = m.sf_plan(c, mask, dtype)
    ab = 8 if dtype == torch.complex64 else 16
    for inner in (info["n_cross"] - 3, 1, 0):
        work = 2 * ((1 << (info["n_a"] + inner)) + (1 << (info["n_b"] + inner))) * ab
        got, st, inf = all_amplitudes(m, c, mask, dtype, work=work)
        assert inf["n_inner"] == inner and inf["n_outer"] == info["n_cross"] - inner
        check_close(got, ref, dtype, f"S-F with {inf['n_outer']} enumerated path bits")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("seed", [0, 1, 3])
def test_random_circuits_with_cz_cp_cnot_across(dtype, seed):
    m = lib()
    n = 11
    rng = np.random.default_rng(500 + seed)
    mask = int(sum(1 << int(q) for q in rng.permutation(n)[:5]))
    inside = W.random_circuit(n, 120, 600 + seed, ops=("H", "SQRTX", "SQRTY", "T", "RX", "RY", "RZ", "P", "S", "X",
                                                       "Y", "Z", "CZ", "CP", "CNOT", "SWAP"),
                              mat_k=(1, 2), diag_k=(1, 2))
    # keep SWAP and explicit matrices inside one half; CZ, CP and CNOT may cross
    def half(q):
        return (mask >> q) & 1
    gates = [g for g in inside.gates
             if g.op in ("CZ", "CP", "CNOT") or len({half(q) for q in g.qubits}) == 1]
    c = W.Circuit(n, gates, inside.n_params, "sf-random")
    params = W.uniform_params(1, c.n_params, 700 + seed)[0]
    ref = oracle.simulate(c, params)
    info = m.sf_plan(c, mask, dtype)
    assert info["n_cross"] >= 5
    ab = 8 if dtype == torch.complex64 else 16
    for inner in (info["n_cross"], info["n_cross"] // 2):
        work = (2 if inner < info["n_cross"] else 1) * ((1 << (info["n_a"] + inner)) + (1 << (info["n_b"] + inner))) * ab
        got, _, inf = all_amplitudes(m, c, mask, dtype, params=params, work=work)
        assert inf["n_inner"] == inner
        check_close(got, ref, dtype, f"S-F random seed {seed}, {inf['n_outer']} enumerated")


def test_no_gate_across_the_cut():
    m = lib()
    a = W.grid_circuit(2, 3, 5, seed=1)
    gates = list(a.gates) + [W.Gate(g.op, tuple(q + 6 for q in g.qubits)) for g in a.gates]
    c = W.Circuit(12, gates, 0, "two-blocks")
    got, _, info = all_amplitudes(m, c, (1 << 6) - 1, torch.complex64)
    assert info["n_cross"] == 0
    check_close(got, oracle.simulate(c), torch.complex64, "S-F without cross gates")


def test_sampled_amplitudes_22_qubits():
    m = lib()
    c = W.grid_circuit(2, 11, 12, seed=1006)
    mask = sum(1 << q for q in range(22) if q % 11 < 5 or q == 5)
    ref = oracle.simulate(c)
    idx = np.unique(np.random.default_rng(9).integers(0, 1 << 22, 4096).astype(np.uint64))
    sim = m.SchrodingerFeynman(c, mask, torch.complex64)
    got, st = sim.amplitudes(idx)
    got2, _ = sim.amplitudes(idx)              # second call: plans reused
    assert np.array_equal(got, got2)
    err = np.max(np.abs(got - ref[idx.astype(np.int64)]))
    assert err <= 1e-5, err
    assert st["passes"] > 0 and st["hbm_bytes"] > 0
