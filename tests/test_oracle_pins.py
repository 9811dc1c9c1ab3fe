"""Pins of the FP64 oracle against things other than itself: the paper's
printed matrices and examples (tests/golden), closed forms, identities,
brute-force operator products and exact summation."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import brute, gates as G
from tests.golden import load as golden

C = math.sqrt(0.5)
OMEGA = complex(C, C)


# ---------------------------------------------------------------- gate table

def test_printed_matrices_match_gate_table():
    m = golden.matrices()
    np.testing.assert_array_equal(m["NOT"], G.X)
    np.testing.assert_allclose(m["H_times_sqrt2"] * C, G.H, atol=1e-16)
    np.testing.assert_array_equal(m["Z"], G.Z)
    np.testing.assert_array_equal(m["CZ"], G.CZ)
    np.testing.assert_allclose(m["SQRTX_times_2"] / 2, G.SQRTX, atol=1e-16)
    arg = m["T_phase_arg_over_pi"][0]
    t = np.diag([np.exp(1j * math.pi * arg[0].real), np.exp(1j * math.pi * arg[1].real)])
    np.testing.assert_allclose(t, G.T, atol=1e-15)


def test_cnot_printed_bigendian_equals_littleendian_action():
    # Reorder the printed (big-endian) CNOT to the local index l = b0 + 2 b1
    # with the control on bit 0: swap the roles of the two index bits.
    m = golden.matrices()["CNOT_bigendian"]
    perm = [0, 2, 1, 3]
    np.testing.assert_array_equal(m[np.ix_(perm, perm)], G.CNOT)


def test_sqrty_reading():
    # The printed sqrt(Y) squares to -Y; the principal root used here squares
    # to Y.  Printed = e^{i pi/4} Z H ("HZ" in circuit order); principal =
    # e^{i pi/4} H Z as a matrix product.  Only the printed one makes
    # sqrt(Y) H diagonal (Sec. 4.5).
    yp = golden.matrices()["SQRTY_printed_times_2"] / 2
    np.testing.assert_allclose(yp @ yp, -G.Y, atol=1e-15)
    np.testing.assert_allclose(G.SQRTY @ G.SQRTY, G.Y, atol=1e-15)
    np.testing.assert_allclose(yp, OMEGA * G.Z @ G.H, atol=1e-15)
    np.testing.assert_allclose(G.SQRTY, OMEGA * G.H @ G.Z, atol=1e-15)
    d = yp @ G.H
    assert abs(d[0, 1]) < 1e-15 and abs(d[1, 0]) < 1e-15
    d2 = G.SQRTY @ G.H
    assert abs(d2[0, 1]) > 0.5


def test_factored_matrices_and_kronecker_products():
    m = golden.matrices()
    np.testing.assert_allclose(G.H / C, m["Hp"], atol=1e-15)
    np.testing.assert_allclose(2 * G.SQRTX, m["SQRTXp"], atol=1e-15)
    # The printed sqrt(Y)' is the paper's own sqrt(Y) times 2.
    np.testing.assert_allclose(m["SQRTYp"], m["SQRTY_printed_times_2"], atol=0)
    np.testing.assert_allclose(np.kron(m["Hp"], m["Hp"]), m["HpHp"], atol=0)
    # X'(x)X' and Y'(x)Y' are printed up to a factor 2 ((1+-i)^2 = +-2i).
    np.testing.assert_allclose(np.kron(m["SQRTXp"], m["SQRTXp"]), 2 * m["XpXp_printed"], atol=1e-14)
    np.testing.assert_allclose(np.kron(m["SQRTYp"], m["SQRTYp"]), 2j * m["YpYp_over_i"], atol=1e-14)


def test_gate_identities():
    # Eq. (1): (I (x) H) CNOT (I (x) H) = CZ, H on the target
    h_t = brute.full_operator(2, (1,), G.H)
    cn = brute.full_operator(2, (0, 1), G.CNOT)
    np.testing.assert_allclose(h_t @ cn @ h_t, G.CZ, atol=1e-15)
    # sqrt(X) = H P H (Sec. 2)
    np.testing.assert_allclose(G.H @ G.S @ G.H, G.SQRTX, atol=1e-15)
    # P = T^2, Z = T^4, T^8 = I (Sec. 4.3)
    np.testing.assert_allclose(G.T @ G.T, G.S, atol=1e-15)
    np.testing.assert_allclose(np.linalg.matrix_power(G.T, 4), G.Z, atol=1e-15)
    np.testing.assert_allclose(np.linalg.matrix_power(G.T, 8), np.eye(2), atol=1e-15)
    # principal roots square to their involutions
    for r, g in ((G.SQRTX, G.X), (G.SQRTY, G.Y), (G.SQRTW, G.W)):
        np.testing.assert_allclose(r @ r, g, atol=1e-15)
    np.testing.assert_allclose(G.W @ G.W, np.eye(2), atol=1e-15)
    # every fixed gate is unitary, and X Y = i Z fixes the sign convention of Y
    for name, u in G.FIXED.items():
        np.testing.assert_allclose(u.conj().T @ u, np.eye(u.shape[0]), atol=1e-15, err_msg=name)
    np.testing.assert_allclose(G.X @ G.Y, 1j * G.Z, atol=0)
    # rotations: R(pi) = -i P, RZ(t) = e^{-i t/2} P(t)
    for f, p in ((G.rx, G.X), (G.ry, G.Y), (G.rz, G.Z)):
        np.testing.assert_allclose(f(math.pi), -1j * p, atol=1e-15)
    t = 0.377
    np.testing.assert_allclose(G.rz(t), np.exp(-0.5j * t) * G.phase(t), atol=1e-15)


def test_t_phase_values():
    vals = golden.bitmasks()["t_phase_values"]
    want = set()
    for v in vals:
        a, b = (int(x) for x in v.split(","))
        s = 1.0 if (a == 0 or b == 0) else C
        want.add((round(a * s, 12), round(b * s, 12)))
    got = set()
    for e in range(8):
        z = G.T[1, 1] ** e
        got.add((round(z.real, 12) + 0.0, round(z.imag, 12) + 0.0))
    assert got == want


# ------------------------------------------------- generic kernel vs brute force

ALL_OPS = ("H", "X", "Y", "Z", "S", "SDG", "T", "TDG", "SQRTX", "SQRTY", "SQRTW",
           "SQRTXDG", "RX", "RY", "RZ", "P", "CZ", "CNOT", "SWAP", "CP")


@pytest.mark.parametrize("seed", range(6))
def test_oracle_matches_brute_force(seed):
    n = 3 + seed % 5
    c = W.random_circuit(n, 40, seed, ops=ALL_OPS, mat_k=(1, 2, 3) if n >= 3 else (1, 2), diag_k=(1, 2, 3))
    params = W.uniform_params(1, c.n_params, seed + 99)[0]
    psi0 = W.random_state(n, seed + 7)
    a = oracle.simulate(c, params, psi0)
    b = brute.simulate(c, params, psi0)
    assert np.max(np.abs(a - b)) <= 1e-13


def test_brute_constructions_agree():
    rng = np.random.default_rng(3)
    for n, q0, k in ((4, 0, 2), (5, 2, 3), (6, 3, 1), (6, 1, 4)):
        z = rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))
        qs = tuple(range(q0, q0 + k))
        np.testing.assert_allclose(brute.full_operator(n, qs, z), brute.kron_operator(n, qs, z), atol=0)


def test_reversed_and_nonadjacent_qubits():
    # A non-symmetric 2-qubit matrix on reversed, non-adjacent qubits: the
    # gate-by-gate kernel must agree with SWAP conjugation of the Kronecker
    # padding (an independent construction of the same operator).
    rng = np.random.default_rng(11)
    u = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    n = 5
    psi0 = W.random_state(n, 5)
    # gate on qubits (3, 1): local bit 0 <- qubit 3, local bit 1 <- qubit 1
    got = psi0.copy()
    oracle.apply_matrix(got, n, (3, 1), u)
    # move qubit 3 to position 1 and qubit 1 to position 2 with SWAPs, apply
    # U on (1, 2) by Kronecker padding, then undo the SWAPs
    sw12 = brute.kron_operator(n, (1, 2), G.SWAP)
    sw23 = brute.kron_operator(n, (2, 3), G.SWAP)
    # qubits (3,1): after sw23 (swap 2,3): q3->2 ; after sw12: q2->1, q1->2
    pre = sw12 @ sw23
    op = pre.T @ brute.kron_operator(n, (1, 2), u) @ pre
    np.testing.assert_allclose(got, op @ psi0, atol=1e-14)


# ----------------------------------------------------------------- closed forms

def test_hadamard_layer_uniform():
    n = 9
    c = W.Circuit(n, [W.Gate("H", (q,)) for q in range(n)])
    psi = oracle.simulate(c)
    np.testing.assert_allclose(psi, np.full(1 << n, 2.0 ** (-n / 2)), atol=1e-15)


def test_ghz():
    n = 8
    g = [W.Gate("H", (0,))] + [W.Gate("CNOT", (i, i + 1)) for i in range(n - 1)]
    psi = oracle.simulate(W.Circuit(n, g))
    want = np.zeros(1 << n, complex)
    want[0] = want[-1] = C
    np.testing.assert_allclose(psi, want, atol=1e-15)


def qft_gates(n):
    g = []
    for i in reversed(range(n)):          # most significant qubit first
        g.append(W.Gate("H", (i,)))
        for j in reversed(range(i)):
            g.append(W.Gate("CP", (j, i), theta=math.pi / (1 << (i - j))))
    for q in range(n // 2):
        g.append(W.Gate("SWAP", (q, n - 1 - q)))
    return g


@pytest.mark.parametrize("x", [0, 1, 5, 22, 63])
def test_qft_of_basis_state(x):
    n = 6
    psi = oracle.simulate(W.Circuit(n, qft_gates(n)), psi0=W.basis_state(n, x))
    y = np.arange(1 << n)
    want = np.exp(2j * math.pi * x * y / (1 << n)) / math.sqrt(1 << n)
    np.testing.assert_allclose(psi, want, atol=1e-14)


def test_x_mask_basis():
    n = 7
    mask = 0b1011010
    g = [W.Gate("X", (q,)) for q in range(n) if (mask >> q) & 1]
    psi = oracle.simulate(W.Circuit(n, g))
    assert psi[mask] == 1 and np.count_nonzero(psi) == 1


def test_t_layer_phase_formula():
    # Sec. 4.3: a T layer with bitmask m gives amplitude j the phase
    # e^{i pi popcount(m & j) / 4}; on the uniform state every amplitude
    # has modulus 2^{-n/2}.
    n = 6
    m = int(golden.bitmasks()["reorder_t_mask"][0], 2) | 0b110000
    g = [W.Gate("H", (q,)) for q in range(n)] + [W.Gate("T", (q,)) for q in range(n) if (m >> q) & 1]
    psi = oracle.simulate(W.Circuit(n, g))
    for j in range(1 << n):
        e = bin(m & j).count("1") % 8
        want = 2.0 ** (-n / 2) * complex(math.cos(math.pi * e / 4), math.sin(math.pi * e / 4))
        assert abs(psi[j] - want) < 1e-15


def test_cz_cluster_bitmask_formula():
    # Sec. 4.3 all-pairs example: masks m0..m3 (one per qubit, symmetric);
    # twelve set bits; the sign of amplitude j is (-1)^{#pairs inside j}, and
    # summing popcount(m_k & j) over k in j counts every pair twice.
    bm = golden.bitmasks()
    masks = [int(x, 2) for x in bm["cz_all_pairs_masks"]]
    # printed left to right as m0, m1, m2, m3 with bit 3 on the left
    assert sum(bin(x).count("1") for x in masks) == int(bm["cz_all_pairs_bitcount"][0])
    n = 4
    pairs = [(a, b) for a in range(n) for b in range(a + 1, n)]
    for k in range(n):
        want = sum(1 << l for l in range(n) if l != k)
        assert masks[n - 1 - k] == want or masks[k] == want
    g = [W.Gate("H", (q,)) for q in range(n)] + [W.Gate("CZ", p) for p in pairs]
    psi = oracle.simulate(W.Circuit(n, g))
    for j in range(1 << n):
        cnt = sum(bin(masks[k] & j).count("1") for k in range(n) if (j >> k) & 1)
        assert cnt % 2 == 0
        sign = -1.0 if (cnt // 2) % 2 else 1.0
        assert abs(psi[j] - sign * 0.25) < 1e-15


def test_pair_example_and_gray_code():
    bm = golden.bitmasks()
    a, b = (int(x) for x in bm["pair_example"])
    assert bin(a ^ b).count("1") == 1 and (a ^ b) == 8       # differ in bit 3
    gray = [k ^ (k >> 1) for k in range(8)]
    assert gray == [int(x) for x in bm["gray3"]]


def test_norm_preserved_random_circuits():
    for seed in range(3):
        c = W.random_circuit(10, 200, seed, mat_k=(1, 2, 3, 4))
        params = W.uniform_params(1, c.n_params, seed)[0]
        psi = oracle.simulate(c, params, W.random_state(10, seed))
        assert abs(oracle.norm2(psi) - 1.0) < 1e-13


def test_mirror_returns_to_zero():
    c = W.line_circuit(10, 6, seed=5)
    m = W.concat(c, W.inverse(c))
    psi = oracle.simulate(m)
    assert abs(psi[0] - 1) < 1e-13 and np.max(np.abs(psi[1:])) < 1e-13


# ------------------------------------------------------------ reductions

def test_norm2_compensated_is_exact():
    # values spanning 30 orders of magnitude: Sum2 matches an exactly rounded
    # sum (math.fsum) where plain left-to-right summation does not.
    rng = np.random.default_rng(0)
    n = 14
    re = rng.standard_normal(1 << n) * np.exp(rng.uniform(-35, 0, 1 << n))
    re[0] = 1.0
    psi = re.astype(np.complex128)
    sq = (re * re).tolist()
    exact = math.fsum(sq)
    naive = 0.0
    for v in sq:
        naive += v
    got = oracle.norm2(psi, nthreads=1)
    assert got == exact
    assert oracle.norm2(psi) == pytest.approx(exact, rel=1e-16, abs=0)


def test_inner_compensated_is_exact():
    # <a|b> = sum_j conj(a_j) b_j.  Per amplitude the four components share a
    # power of two and have 12-bit integer mantissas, so p r + q s and
    # p s - q r are exact in FP64 (with or without contraction); the
    # exponents span 2^-70 .. 2^0, where the order of a plain sum matters.
    # The compensated sum must equal the exactly rounded sum (math.fsum).
    rng = np.random.default_rng(1)
    n = 13
    N = 1 << n
    e = rng.integers(-35, 1, N).astype(np.float64)
    m = rng.integers(-2048, 2049, (4, N)).astype(np.float64)
    sc = np.exp2(e)
    p, q, r, s = (m[i] * sc for i in range(4))
    a = p + 1j * q
    b = r + 1j * s
    want_re = math.fsum((p * r + q * s).tolist())
    want_im = math.fsum((p * s - q * r).tolist())
    got = oracle.inner(a, b, nthreads=1)
    assert got.real == want_re and got.imag == want_im
    got8 = oracle.inner(a, b)
    assert got8.real == pytest.approx(want_re, rel=1e-16, abs=0)
    assert got8.imag == pytest.approx(want_im, rel=1e-16, abs=0)
    # conjugate-linear in the first argument, as np.vdot
    x = W.random_state(6, 3)
    y = W.random_state(6, 4)
    assert abs(oracle.inner(x, y) - np.vdot(x, y)) < 1e-15
    assert abs(oracle.inner(1j * x, y) - (-1j) * np.vdot(x, y)) < 1e-15


@pytest.mark.parametrize("seed", range(4))
def test_expectation_matches_explicit_pauli(seed):
    n = 5
    rng = np.random.default_rng(seed)
    psi = W.random_state(n, seed)
    for _ in range(6):
        x = int(rng.integers(0, 1 << n))
        z = int(rng.integers(0, 1 << n))
        P = brute.pauli_matrix(n, x, z)
        want = np.vdot(psi, P @ psi)
        got = oracle.pauli_term(psi, x, z)
        assert abs(got - want) < 1e-14
        assert abs(want.imag) < 1e-14     # Hermitian


def test_expectation_known_states():
    plus = np.array([C, C], complex)
    plus_i = np.array([C, 1j * C], complex)
    assert oracle.pauli_term(plus, 1, 0) == pytest.approx(1.0)
    assert oracle.pauli_term(plus_i, 1, 1) == pytest.approx(1.0)          # Y
    assert oracle.pauli_term(np.array([1, 0], complex), 0, 1) == pytest.approx(1.0)
    n = 6
    g = [W.Gate("H", (0,))] + [W.Gate("CNOT", (i, i + 1)) for i in range(n - 1)]
    ghz = oracle.simulate(W.Circuit(n, g))
    assert oracle.pauli_term(ghz, 0, 0b11).real == pytest.approx(1.0)
    assert oracle.pauli_term(ghz, (1 << n) - 1, 0).real == pytest.approx(1.0)


# ------------------------------------------------------------ gradients

def test_gradient_closed_form_one_qubit():
    # RY(t) then RZ(p) on |0>, H = X/2: E = sin t cos p / 2
    c = W.Circuit(1, [W.Gate("RY", (0,), param=0), W.Gate("RZ", (0,), param=1)], 2)
    h = W.pauli_sum([(0.5, {0: "X"})])
    for t, p in ((0.3, 1.1), (2.0, -0.7), (4.4, 3.0)):
        th = np.array([t, p])
        assert oracle.energy(c, th, h) == pytest.approx(0.5 * math.sin(t) * math.cos(p), abs=1e-15)
        g = oracle.grad_param_shift(c, th, h)
        np.testing.assert_allclose(g, [0.5 * math.cos(t) * math.cos(p), -0.5 * math.sin(t) * math.sin(p)],
                                   atol=1e-14)
        np.testing.assert_allclose(oracle.grad_fd(c, th, h, h=1e-5), g, atol=1e-9)


def test_gradient_closed_form_two_qubit():
    c = W.Circuit(2, [W.Gate("RY", (0,), param=0), W.Gate("RY", (1,), param=1)], 2)
    h = W.pauli_sum([(1.0, {0: "Z", 1: "Z"})])
    th = np.array([0.9, 2.3])
    assert oracle.energy(c, th, h) == pytest.approx(math.cos(0.9) * math.cos(2.3), abs=1e-15)
    np.testing.assert_allclose(oracle.grad_param_shift(c, th, h),
                               [-math.sin(0.9) * math.cos(2.3), -math.cos(0.9) * math.sin(2.3)], atol=1e-14)


def test_last_layer_rz_gradient_zero_for_z_observable():
    c = W.ansatz_circuit(4, 2)
    th = W.uniform_params(1, c.n_params, 3)[0]
    g = oracle.grad_param_shift(c, th, W.z_sum(4))
    last_rz = [c.gates[i].param for i in range(len(c.gates)) if c.gates[i].op == "RZ"][-4:]
    assert np.max(np.abs(g[last_rz])) < 1e-14


def test_generators_deterministic():
    a = W.grid33()
    b = W.grid33()
    assert [(g.op, g.qubits) for g in a.gates] == [(g.op, g.qubits) for g in b.gates]
    assert len(a.gates) == 1873 and len(W.grid30().gates) == 875
    assert len(W.line_circuit().gates) == 175
    c = W.ansatz_circuit()
    assert len(c.gates) == 590 and c.n_params == 400
    assert len(W.ansatz_observable()) == 39
    u = W.sample_uniforms(1000, seed=3, batch=2)
    assert u.shape == (2, 1000) and np.array_equal(u, W.sample_uniforms(1000, seed=3, batch=2))
    assert float(u.min()) >= 0.0 and float(u.max()) < 1.0
    assert len(W.grid_circuit(4, 8, 26, seed=1004).gates) == 1208


# ------------------------------------------------------- measurement sampling

def test_sample_example_circuit_is_deterministic_on_basis_inputs():
    # Sec. 2 example: H on one qubit, CNOT, H again equals CZ, so a basis input
    # is measured as itself with certainty
    u = np.concatenate([[0.0], W.sample_uniforms(200, seed=7)])
    for x in range(4):
        c = W.Circuit(2, [W.Gate("H", (0,)), W.Gate("CNOT", (1, 0)), W.Gate("H", (0,))])
        psi = oracle.simulate(c, psi0=W.basis_state(2, x))
        assert np.all(oracle.sample(psi, u) == x)


def test_sample_uniform_state_closed_form():
    # after a Hadamard layer every outcome has probability 2^-n: the outcome
    # of u is floor(u 2^n); random numbers at the middle of each cell keep the
    # comparison away from rounding at the cell edges
    for n in (1, 5, 9):
        psi = oracle.simulate(W.Circuit(n, [W.Gate("H", (q,)) for q in range(n)]))
        k = np.arange(1 << n)
        assert np.array_equal(oracle.sample(psi, (k + 0.5) / (1 << n)), k)


def test_sample_ghz_halves():
    n = 6
    g = [W.Gate("H", (0,))] + [W.Gate("CNOT", (i, i + 1)) for i in range(n - 1)]
    psi = oracle.simulate(W.Circuit(n, g))
    u = W.sample_uniforms(500, seed=8)
    got = oracle.sample(psi, u)
    assert np.array_equal(got, np.where(u < 0.5, 0, (1 << n) - 1))


def test_sample_stratified_frequencies_equal_probabilities():
    # a grid of M random numbers gives each outcome j a share of the grid
    # within 1/M of |alpha_j|^2 (outcome j owns an interval of that length)
    n, M = 4, 1 << 16
    psi = W.random_state(n, seed=9)
    got = oracle.sample(psi, (np.arange(M) + 0.5) / M)
    freq = np.bincount(got.astype(np.int64), minlength=1 << n) / M
    assert np.max(np.abs(freq - np.abs(psi) ** 2)) <= 1.0 / M + 1e-15
    assert np.all(np.diff(got.astype(np.int64)) >= 0)


def test_sample_zero_probability_outcomes_never_drawn():
    # only qubit 0 is in superposition: outcomes 0 and 1, also for u just
    # below 1; scaling the state does not change the outcomes
    psi = oracle.simulate(W.Circuit(3, [W.Gate("H", (0,))]))
    u = np.array([0.0, 0.25, 0.5 - 1e-12, 0.5 + 1e-12, np.nextafter(1.0, 0.0)])
    assert list(oracle.sample(psi, u)) == [0, 0, 0, 1, 1]
    assert list(oracle.sample(3.0 * psi, u)) == [0, 0, 0, 1, 1]
    with pytest.raises(ValueError):
        oracle.sample(psi, np.array([1.0]))


def test_grid33_cut28_fixture_is_a_unit_state_sample():
    # the stored oracle amplitudes of the 28-qubit cut: the circuit is unitary
    # (norm 1), and a uniform sample of its Porter-Thomas amplitudes has mean
    # 2^n |alpha|^2 near 1
    idx, amp, nrm = golden.grid33_cut28()
    assert abs(nrm - 1.0) < 1e-12
    assert idx.size > 2000 and np.all(np.diff(idx.astype(np.int64)) > 0)
    x = np.abs(amp) ** 2 * float(1 << 28)
    assert 0.85 < float(np.mean(x)) < 1.15
