"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: complex64 max-abs 1e-5 and L2 1e-4, complex128 max-abs and L2
1e-12; sign/permutation-only circuits must agree exactly (numeric equality,
so +0 and -0 compare equal)."""
import math

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


DTYPES = [torch.complex64, torch.complex128]
ALL_OPS = ("H", "X", "Y", "Z", "S", "SDG", "T", "TDG", "SQRTX", "SQRTY", "SQRTW",
           "SQRTXDG", "SQRTYDG", "SQRTWDG", "RX", "RY", "RZ", "P", "CZ", "CNOT", "SWAP", "CP")
EXACT_OPS = ("X", "Y", "Z", "S", "SDG", "CZ", "CNOT", "SWAP")


def run(circ, psi0, dtype, params=None, **opts):
    m = lib()
    t = to_dev(psi0, dtype)
    s = m.StateVector(circ.n, dtype, batch=t.shape[0], tensor=t, opts=m.make_opts(**opts))
    st = s.apply(circ, params)
    out = to_host(t)
    s.close()
    return out, st


@pytest.mark.parametrize("dtype", DTYPES)
def test_init_kinds(dtype):
    m = lib()
    n = 9
    s = m.StateVector(n, dtype)
    s.init("zero")
    got = to_host(s.tensor)[0]
    assert got[0] == 1 and np.count_nonzero(got) == 1
    s.init("basis", 301)
    got = to_host(s.tensor)[0]
    assert got[301] == 1 and np.count_nonzero(got) == 1
    s.init("uniform")
    got = to_host(s.tensor)[0]
    np.testing.assert_allclose(got, np.full(1 << n, 2.0 ** (-n / 2)), rtol=1e-7 if dtype == torch.complex64 else 1e-15)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("op", ALL_OPS)
def test_single_gate_plain_and_fused(dtype, op):
    n = 10
    rng = np.random.default_rng(sum(map(ord, op)))
    k = W.ARITY[op]
    for trial in range(3):
        qs = tuple(int(x) for x in rng.permutation(n)[:k])
        if trial == 1:
            qs = tuple(range(n - k, n)) if k == 1 else (n - 1, 0)    # highest / straddling
        g = W.Gate(op, qs, theta=0.7317 if op in W.PARAMETRIC else 0.0)
        c = W.Circuit(n, [g])
        psi0 = round_c64(W.random_state(n, trial + 3))
        ref = oracle.simulate(c, psi0=psi0)
        for plain in (1, 0):
            got, _ = run(c, psi0, dtype, plain=plain)
            if op in EXACT_OPS:
                assert np.array_equal(got[0], ref), f"{op} {qs} plain={plain} not exact"
            else:
                check_close(got[0], ref, dtype, f"{op} {qs} plain={plain}")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("seed", range(4))
def test_random_circuits_fused(dtype, seed):
    n = [6, 9, 14, 16][seed]
    c = W.random_circuit(n, 150, seed, ops=ALL_OPS, mat_k=(1, 2, 3, 4), diag_k=(1, 2, 3))
    params = W.uniform_params(1, c.n_params, seed)[0]
    psi0 = round_c64(W.random_state(n, seed + 11))
    ref = oracle.simulate(c, params, psi0)
    for structured in (1, 0):
        got, st = run(c, psi0, dtype, params, structured=structured)
        check_close(got[0], ref, dtype, f"random n={n} structured={structured}")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_tiny_states(dtype, n):
    # states smaller than a register group (16 amplitudes) or a default tile:
    # n <= 3 runs gate by gate, n = 4, 5 as one tile holding the whole state
    c = W.random_circuit(n, 60, 100 + n, ops=ALL_OPS, mat_k=(1, 2, 3), diag_k=(1, 2))
    params = W.uniform_params(1, c.n_params, n)[0]
    psi0 = round_c64(W.random_state(n, 200 + n))
    ref = oracle.simulate(c, params, psi0)
    for plain in (1, 0):
        got, _ = run(c, psi0, dtype, params, plain=plain)
        check_close(got[0], ref, dtype, f"n={n} plain={plain}")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [1, 5, 14])
def test_empty_circuit(dtype, n):
    m = lib()
    c = W.Circuit(n, [])
    psi0 = round_c64(W.random_state(n, 300 + n))
    for plain in (1, 0):
        got, st = run(c, psi0, dtype, plain=plain)
        assert np.array_equal(got[0], psi0) and st["launches"] == 0
    # a deferred |0..0> is written by the (empty) sweep
    s = m.StateVector(n, dtype)
    s.tensor.fill_(1.0)
    s.init("zero_deferred")
    s.apply(c)
    got = to_host(s.tensor)[0]
    assert got[0] == 1 and np.count_nonzero(got) == 1


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [1, 14])
def test_copy_state(dtype, n):
    m = lib()
    B = 2
    psi0 = np.stack([round_c64(W.random_state(n, 400 + b)) for b in range(B)])
    a = m.StateVector(n, dtype, batch=B, tensor=to_dev(psi0, dtype))
    b = m.StateVector(n, dtype, batch=B)
    b.copy_from(a)
    assert np.array_equal(to_host(b.tensor), psi0)
    # a deferred |0..0> is passed on and written by the next sweep
    a.init("zero_deferred")
    b.tensor.fill_(3.0)
    b.copy_from(a)
    b.apply(W.Circuit(n, []))
    got = to_host(b.tensor)
    assert np.all(got[:, 0] == 1) and np.count_nonzero(got) == B
    with pytest.raises(m.SvError):
        b.copy_from(m.StateVector(n + 1, dtype, batch=B))
    with pytest.raises(m.SvError):
        b.copy_from(m.StateVector(n, dtype, batch=B + 1))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("case", ["tile_last", "plain_last", "plain_mode"])
def test_apply_with_norm(dtype, case):
    # the norm returned by the sweep equals the separate FP64 norm and the
    # oracle's: summed by the last tile pass, or by a reduction when the plan
    # ends with a per-gate step
    m = lib()
    n, B = 15, 2
    c = W.grid_circuit(3, 5, 6, seed=1007)
    if case == "plain_last":
        # a 6-qubit matrix at the end runs as a per-gate step after the tiles
        rng = np.random.default_rng(5)
        z = rng.standard_normal((64, 64)) + 1j * rng.standard_normal((64, 64))
        qm, r = np.linalg.qr(z)
        wide = W.Gate("MAT", (0, 3, 5, 8, 11, 14), mat=qm * (np.diag(r) / np.abs(np.diag(r))))
        c = W.Circuit(n, list(c.gates) + [wide], 0)
    psi0 = np.stack([round_c64(W.random_state(n, 500 + b)) * (1.0 + 0.5 * b) for b in range(B)])
    t = to_dev(psi0, dtype)
    s = m.StateVector(n, dtype, batch=B, tensor=t, opts=m.make_opts(plain=1 if case == "plain_mode" else 0))
    st, nrm = s.apply_norm(c)
    assert st["passes"] >= 1
    sep = s.norm()
    out = to_host(t)
    # against the oracle the complex64 state's own rounding dominates (about
    # 1e-6 after 300 gate-by-gate FP32 updates); against the separate FP64
    # norm of the same state only the summation order differs
    tol = 1e-5 if dtype == torch.complex64 else 1e-12
    for b in range(B):
        ref = oracle.norm2(oracle.simulate(c, psi0=psi0[b]))
        assert abs(nrm[b] - ref) < tol * ref, (b, nrm[b], ref)
        assert abs(nrm[b] - sep[b]) < 1e-13 * ref
        check_close(out[b], oracle.simulate(c, psi0=psi0[b]), dtype, f"{case} state {b}")


@pytest.mark.parametrize("dtype", DTYPES)
def test_wide_matrix_gates(dtype):
    n = 12
    c = W.random_circuit(n, 20, 5, ops=("H", "CZ", "T"), mat_k=(5, 6))
    psi0 = round_c64(W.random_state(n, 2))
    ref = oracle.simulate(c, psi0=psi0)
    got, _ = run(c, psi0, dtype)
    check_close(got[0], ref, dtype, "k=5,6 matrices")


@pytest.mark.parametrize("plain", [1, 0])
def test_exact_circuits_bit_exact(plain):
    for seed in range(3):
        n = 13
        c = W.random_circuit(n, 300, seed, ops=EXACT_OPS)
        psi0 = round_c64(W.random_state(n, seed))
        ref = oracle.simulate(c, psi0=psi0)
        got, _ = run(c, psi0, torch.complex64, plain=plain)
        assert np.array_equal(got[0], ref), f"seed {seed}: sign/perm circuit not exact"


@pytest.mark.parametrize("tile_bits,low_bits", [(13, 5), (12, 4), (14, 7), (10, 3)])
def test_tile_geometries(tile_bits, low_bits):
    c = W.grid_circuit(3, 6, 6, seed=9)
    n = c.n
    ref = oracle.simulate(c)
    for dtype in DTYPES:
        if dtype == torch.complex128 and tile_bits > 13:
            continue
        got, st = run(c, np.eye(1, 1 << n, 0)[0].astype(np.complex128), dtype, tile_bits=tile_bits,
                      low_bits=low_bits, product_init=0)
        check_close(got[0], ref, dtype, f"T={tile_bits} L={low_bits}")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("beam", [1, 2, 16])
def test_planner_beam_widths(dtype, beam):
    # different local-set sequences (15 passes greedily, 13 with a beam)
    # and the interpreted and plan-specialised kernels give the oracle's state
    c = W.random_circuit(16, 220, seed=97, mat_k=(2, 3))
    p = W.uniform_params(1, c.n_params, 93)[0]
    psi0 = W.random_state(16, 94)
    ref = oracle.simulate(c, p, psi0=psi0)
    for jit in (-1, 1):
        got, st = run(c, psi0, dtype, params=p, tile_bits=8, low_bits=3, plan_beam=beam, jit=jit)
        check_close(got[0], ref, dtype, f"beam={beam} jit={jit} passes={st['passes']}")


def test_line_circuit_gate_by_gate_c128():
    c = W.line_circuit()
    ref = oracle.simulate(c)
    m = lib()
    s = m.StateVector(c.n, torch.complex128, opts=m.make_opts(plain=1))
    s.init("zero")
    st = s.apply(c)
    got = to_host(s.tensor)[0]
    check_close(got, ref, torch.complex128, "line circuit plain")
    assert st["launches"] >= 170


@pytest.mark.parametrize("dtype", DTYPES)
def test_grid_product_init(dtype):
    c = W.grid_circuit(4, 5, 8, seed=3)
    ref = oracle.simulate(c)
    m = lib()
    s = m.StateVector(c.n, dtype)
    s.init("zero_deferred")
    st = s.apply(c)
    got = to_host(s.tensor)[0]
    check_close(got, ref, dtype, "grid 20q")
    assert st["folded_init"] >= c.n


@pytest.mark.parametrize("dtype", DTYPES)
def test_written_zero_is_read(dtype):
    """After a written |0..0> the buffer is the input: a caller's write
    through the tensor is honoured (no product-state folding)."""
    c = W.grid_circuit(2, 4, 3, seed=5)
    m = lib()
    s = m.StateVector(c.n, dtype)
    s.init("zero")
    psi0 = round_c64(W.random_state(c.n, 77))
    s.tensor.copy_(torch.from_numpy(psi0.astype(np.complex128)).to(s.tensor.dtype).reshape(1, -1).to(s.tensor.device))
    st = s.apply(c)
    assert st["folded_init"] == 0
    check_close(to_host(s.tensor)[0], oracle.simulate(c, None, psi0), dtype, "caller-written input")


@pytest.mark.parametrize("dtype", DTYPES)
def test_batch_of_states(dtype):
    n = 12
    c = W.ansatz_circuit(n, 3)
    B = 5
    params = W.uniform_params(B, c.n_params, 4)
    psi0 = np.stack([round_c64(W.random_state(n, 20 + b)) for b in range(B)])
    got, _ = run(c, psi0, dtype, params)
    for b in range(B):
        ref = oracle.simulate(c, params[b], psi0[b])
        check_close(got[b], ref, dtype, f"batch {b}")


@pytest.mark.parametrize("dtype", DTYPES)
def test_norm_and_expect(dtype):
    m = lib()
    n = 14
    B = 3
    psi0 = np.stack([round_c64(W.random_state(n, 40 + b)) for b in range(B)])
    t = to_dev(psi0, dtype)
    s = m.StateVector(n, dtype, batch=B, tensor=t)
    h = W.pauli_sum([(0.7, {0: "Z", 5: "Z"}), (-1.3, {3: "X"}), (0.25, {2: "Y", 9: "X", 13: "Z"}),
                     (0.5, {}), (1.1, {1: "Y"})])
    nrm = s.norm()
    e = s.expect(h)
    tol = 1e-6 if dtype == torch.complex64 else 1e-12
    for b in range(B):
        x = psi0[b] if dtype == torch.complex128 else psi0[b]
        assert abs(nrm[b] - oracle.norm2(x)) < tol
        assert abs(e[b] - oracle.expect(x, h)) < tol


def test_mirror_returns_to_zero():
    c = W.grid_circuit(3, 5, 12, seed=7)
    mirror = W.concat(c, W.inverse(c))
    m = lib()
    s = m.StateVector(c.n, torch.complex64)
    s.init("zero")
    s.apply(mirror)
    got = to_host(s.tensor)[0]
    assert abs(got[0] - 1) < 1e-5 and np.max(np.abs(got[1:])) < 1e-5


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("k", [2, 3, 4, 5, 6])
def test_dense_block_fusion(dtype, k):
    """Dense mode: gates fused into blocks of <= k qubits (FP64 products),
    k <= 4 inside tile passes, 5-6 as plain kernels."""
    m = lib()
    n = 12
    c = W.random_circuit(n, 200, seed=300 + k, mat_k=(2,))
    p = W.uniform_params(1, c.n_params, 310 + k)
    psi0 = round_c64(W.random_state(n, 320 + k))
    t = to_dev(psi0, dtype)
    for jit in ((-1, 1) if k == 4 else (-1,)):
        t.copy_(to_dev(psi0, dtype))
        s = m.StateVector(n, dtype, tensor=t, opts=m.make_opts(structured=0, max_fuse_k=k, jit=jit))
        s.apply(c, p)
        ref = oracle.simulate(c, p[0], psi0=psi0)
        check_close(to_host(t)[0], ref, dtype, f"dense k={k} jit={jit}")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("k", [5, 6])
@pytest.mark.parametrize("n", [11, 12, 17])
def test_mfma_dense_blocks(k, n, dtype):
    """5- and 6-qubit blocks on the matrix cores (FP32 tiles for complex64
    from 12 qubits, FP64 tiles for complex128 from 11): explicit matrices on
    spread targets, and per-state fused blocks of parametric gates for a
    batch of two states."""
    m = lib()
    rng = np.random.default_rng(900 + 10 * k + n)
    gates = []
    for rep in range(3):
        qs = tuple(int(x) for x in rng.permutation(n)[:k])
        z = rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))
        qm, r = np.linalg.qr(z)
        gates.append(W.Gate("MAT", qs, mat=(qm * (np.diag(r) / np.abs(np.diag(r)))).astype(np.complex128)))
        gates.append(W.Gate("H", (int(rng.integers(0, n)),)))
    c = W.Circuit(n, gates, 0)
    psi0 = round_c64(W.random_state(n, 7))
    got, _ = run(c, psi0, dtype)
    check_close(got[0], oracle.simulate(c, psi0=psi0), dtype, f"MAT k={k} n={n}")
    # per-state matrices: dense blocks fused from RY/RZ/CZ with two parameter sets
    c2 = W.random_circuit(n, 60, seed=950 + k, ops=("RY", "RZ", "CZ", "H"), param_frac=1.0)
    p = W.uniform_params(2, c2.n_params, 960 + k)
    psi = np.stack([round_c64(W.random_state(n, 11 + b)) for b in range(2)])
    t = to_dev(psi, dtype)
    s = m.StateVector(n, dtype, batch=2, tensor=t, opts=m.make_opts(structured=0, max_fuse_k=k))
    st = s.apply(c2, p)
    assert st["dense_ops"] > 0
    out = to_host(t)
    for b in range(2):
        check_close(out[b], oracle.simulate(c2, p[b], psi0=psi[b]), dtype, f"fused k={k} state {b}")


def test_tune_then_apply(tmp_path, monkeypatch):
    """sv_tune picks one of its candidate geometries, remembers it, and the
    tuned context still matches the oracle."""
    monkeypatch.setenv("SVMI_TUNE_CACHE", str(tmp_path / "tune.txt"))
    m = lib()
    c = W.grid_circuit(3, 6, 10, seed=21)
    s = m.StateVector(c.n, torch.complex64)
    chosen, ms = s.tune(c)
    assert chosen["tile_bits"] in (12, 13) and chosen["low_bits"] in (4, 5) and ms > 0
    again, ms2 = s.tune(c)
    assert ms2 == -1.0 and again["tile_bits"] == chosen["tile_bits"]
    s.init("zero")
    s.apply(c)
    check_close(to_host(s.tensor)[0], oracle.simulate(c), torch.complex64, f"tuned {chosen}")
