"""Adjoint gradients on the GPU against the oracle's shift-rule gradients and
closed forms."""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_util import round_c64, to_dev, to_host

pytestmark = pytest.mark.gpu


def lib():
    import paper_2008_00216_amd as m
    return m


TOL = {torch.complex64: 2e-4, torch.complex128: 1e-10}


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_closed_form_one_qubit(dtype):
    m = lib()
    c = W.Circuit(1, [W.Gate("RY", (0,), param=0), W.Gate("RZ", (0,), param=1)], 2)
    h = W.pauli_sum([(0.5, {0: "X"})])
    th = np.array([[0.3, 1.1], [2.0, -0.7]])
    s = m.StateVector(1, dtype, batch=2)
    s.init("zero")
    e, g = s.adjoint_grad(c, th, h)
    for b in range(2):
        t, p = th[b]
        assert abs(e[b] - 0.5 * math.sin(t) * math.cos(p)) < TOL[dtype]
        np.testing.assert_allclose(g[b], [0.5 * math.cos(t) * math.cos(p), -0.5 * math.sin(t) * math.sin(p)],
                                   atol=TOL[dtype])


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("plain", [0, 1])
@pytest.mark.parametrize("seed", range(3))
def test_random_param_circuits(dtype, plain, seed):
    m = lib()
    n = [5, 9, 14][seed]
    ops = ("H", "SQRTX", "T", "CZ", "CNOT", "RX", "RY", "RZ", "P", "CP", "S", "SQRTW")
    c = W.random_circuit(n, 80, 100 + seed, ops=ops, param_frac=1.0)
    B = 3
    th = W.uniform_params(B, c.n_params, seed)
    h = W.pauli_sum([(1.0, {0: "Z", 1: "Z"}), (0.5, {2 % n: "X"}), (-0.3, {1: "Y", (3 % n): "Z"})])
    psi0 = np.stack([round_c64(W.random_state(n, 7 + b)) for b in range(B)])
    t = to_dev(psi0, dtype)
    s = m.StateVector(n, dtype, batch=B, tensor=t, opts=m.make_opts(plain=plain))
    e, g = s.adjoint_grad(c, th, h)
    back = to_host(t)
    for b in range(B):
        e_ref = oracle.energy(c, th[b], h, psi0[b])
        g_ref = oracle.grad_param_shift(c, th[b], h, psi0[b])
        assert abs(e[b] - e_ref) < TOL[dtype], (e[b], e_ref)
        np.testing.assert_allclose(g[b], g_ref, atol=TOL[dtype])
        # the backward sweep un-computes psi back to the input
        assert np.max(np.abs(back[b] - psi0[b])) < (1e-4 if dtype == torch.complex64 else 1e-11)


def test_ansatz_against_fd_and_shift():
    m = lib()
    c = W.ansatz_circuit(10, 4)
    h = W.ansatz_observable(10)
    th = W.uniform_params(2, c.n_params, 5)
    s = m.StateVector(10, torch.complex64, batch=2)
    s.init("zero")
    e, g = s.adjoint_grad(c, th, h)
    for b in range(2):
        g_ref = oracle.grad_param_shift(c, th[b], h)
        np.testing.assert_allclose(g[b], g_ref, atol=2e-4)
        fd = oracle.grad_fd(c, th[b], h, which=list(range(0, c.n_params, 7)))
        np.testing.assert_allclose(g[b][::7], fd, atol=2e-4)


def test_autograd_function():
    m = lib()
    c = W.ansatz_circuit(6, 2)
    h = W.ansatz_observable(6)
    th = torch.tensor(W.uniform_params(2, c.n_params, 8), dtype=torch.float64, requires_grad=True)
    s = m.StateVector(6, torch.complex128, batch=2)
    e = m.Energy.apply(th, s, c, h)
    e.sum().backward()
    for b in range(2):
        g_ref = oracle.grad_param_shift(c, th.detach().numpy()[b], h)
        np.testing.assert_allclose(th.grad.numpy()[b], g_ref, atol=1e-10)
    # without a gradient request the forward runs one sweep and the expectation
    e2 = m.Energy.apply(th.detach(), s, c, h)
    for b in range(2):
        assert abs(float(e2[b]) - oracle.energy(c, th.detach().numpy()[b], h)) < 1e-10
        assert abs(float(e2[b]) - float(e.detach()[b])) < 1e-10


@pytest.mark.parametrize("jit", [-1, 1])
def test_long_single_pass_adjoint(jit):
    """Hundreds of butterflies inside one tile pass: the accumulated
    1/sqrt(2) factors must be applied within the pass so that psi, lambda
    and their products stay in the FP32 range (they overflowed to inf/NaN
    when the factor was only applied at pass ends)."""
    m = lib()
    n = 11
    c = W.layered_param_circuit(n, 40, 7011)
    p = W.uniform_params(1, c.n_params, 7012)
    h = W.z_sum(n)
    s = m.StateVector(n, torch.complex64, opts=m.make_opts(jit=jit))
    s.init("zero")
    e, g = s.adjoint_grad(c, p, h)
    assert np.all(np.isfinite(g)) and np.isfinite(e[0])
    ref = oracle.grad_param_shift(c, p[0], h)
    sel = list(range(0, c.n_params, 23))
    np.testing.assert_allclose(g[0][sel], ref[sel], atol=2e-4)
    assert abs(e[0] - oracle.expect(oracle.simulate(c, p[0]), h)) < 2e-4


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("n", [10, 11, 13, 16])
def test_lambda_tiles_rich_observable(dtype, n):
    # lambda = H psi runs by tiles of 2^11 amplitudes from n = 11 on: X masks
    # below, across and above the tile, several terms per X mask with even
    # and odd phase exponents (X, Y), Z on lane, tile and block bits, and an
    # identity term; n = 10 keeps the untiled kernel
    m = lib()
    hi = n - 1
    terms = [(0.7, {}), (1.0, {0: "Z", 9: "Z"}), (-0.4, {8: "Z", hi: "Z"}), (0.25, {3: "X"}), (0.6, {3: "Y"}),
             (-0.35, {3: "Y", 10 % n: "Z"}), (0.45, {9: "X", 5: "Z"}), (0.3, {hi: "X"}), (-0.2, {hi: "Y", 2: "Z"}),
             (0.15, {0: "X", hi: "X"}), (0.5, {1: "Y", (hi + 1) // 2: "Y"}), (-0.55, {7: "X", 8: "Y", hi: "Z"})]
    h = W.pauli_sum(terms)
    ops = ("H", "SQRTX", "T", "CZ", "RX", "RY", "RZ", "CP")
    c = W.random_circuit(n, 60, 300 + n, ops=ops, param_frac=1.0)
    B = 2
    th = W.uniform_params(B, c.n_params, 301 + n)
    psi0 = np.stack([round_c64(W.random_state(n, 302 + n + b)) for b in range(B)])
    t = to_dev(psi0, dtype)
    s = m.StateVector(n, dtype, batch=B, tensor=t)
    e, g = s.adjoint_grad(c, th, h)
    for b in range(B):
        e_ref = oracle.energy(c, th[b], h, psi0[b])
        assert abs(e[b] - e_ref) < TOL[dtype], (b, e[b], e_ref)
        if b == 0:
            g_ref = oracle.grad_param_shift(c, th[b], h, psi0[b])
            np.testing.assert_allclose(g[b], g_ref, atol=TOL[dtype])
