"""Measurement sampling and amplitude readout on the GPU against the oracle.

Sampling is exact where every probability and prefix sum is a dyadic number
(uniform states with amplitude 2^-n/2, basis states, two-outcome states):
there the GPU outcome must equal the oracle's bit for bit.  For random states
the two sides add the same FP64 probabilities in different orders, so an
outcome may differ only where u * total lies within rounding of a cumulative
probability; the test checks that every difference is of that kind."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_util import round_c64, to_dev, to_host

pytestmark = pytest.mark.gpu

DTYPES = [torch.complex64, torch.complex128]


def lib():
    import paper_2008_00216_amd as m
    return m


def _uniform_tensor(n, dtype, batch=1):
    return torch.full((batch, 1 << n), 2.0 ** (-n / 2), dtype=dtype, device="cuda")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [2, 4, 12, 14, 18])
def test_uniform_state_exact(n, dtype):
    m = lib()
    s = m.StateVector(n, dtype, tensor=_uniform_tensor(n, dtype))
    u = np.concatenate([[0.0, np.nextafter(1.0, 0.0)], W.sample_uniforms(3000, seed=11 + n)])
    got = s.sample(u)
    want = np.floor(u * (1 << n)).astype(np.uint64)
    assert np.array_equal(got, want)
    psi = to_host(s.tensor)[0]
    assert np.array_equal(got, oracle.sample(psi, u))


@pytest.mark.parametrize("dtype", DTYPES)
def test_basis_and_two_outcome_states(dtype):
    m = lib()
    n = 16
    u = np.concatenate([[0.0, 0.5, np.nextafter(0.5, 0.0), np.nextafter(1.0, 0.0)],
                        W.sample_uniforms(500, seed=12)])
    s = m.StateVector(n, dtype)
    for x in (0, 1, 4095, 4096, 40000, (1 << n) - 1):
        s.init("basis", x)
        assert np.all(s.sample(u) == x)
    # equal superposition of two outcomes in distant chunks
    t = torch.zeros((1, 1 << n), dtype=dtype, device="cuda")
    i, j = 77, 61234
    t[0, i] = 2.0 ** -0.5
    t[0, j] = -1j * 2.0 ** -0.5
    s2 = m.StateVector(n, dtype, tensor=t)
    got = s2.sample(u)
    want = oracle.sample(to_host(t)[0], u)
    assert np.array_equal(got, want)
    assert set(np.unique(got)) <= {i, j}


def _check_against_oracle(psi, u, got):
    want = oracle.sample(psi, u)
    diff = np.flatnonzero(got != want)
    if diff.size:
        cdf = np.cumsum(np.abs(psi) ** 2)
        tgt = u[diff] * cdf[-1]
        lo = np.minimum(got[diff], want[diff]).astype(np.int64)
        gap = np.abs(cdf[lo] - tgt)
        assert np.all(gap < 1e-13), (diff[:5], gap[:5])
    assert diff.size <= max(2, u.size // 1000)
    return diff.size


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [3, 11, 13, 15])
def test_random_state_batch_against_oracle(n, dtype):
    m = lib()
    B = 3
    psi0 = np.stack([W.random_state(n, 60 + b + n) for b in range(B)])
    if dtype == torch.complex64:
        psi0 = round_c64(psi0)
    s = m.StateVector(n, dtype, batch=B, tensor=to_dev(psi0, dtype))
    u = W.sample_uniforms(4000, seed=70 + n, batch=B)
    got = s.sample(u)
    assert got.shape == u.shape
    for b in range(B):
        _check_against_oracle(psi0[b], u[b], got[b])


def test_sample_after_circuit_unnormalised():
    # sampling scales u by the state's own norm: a circuit applied to 3|0>
    m = lib()
    c = W.grid_circuit(3, 5, 8, seed=1003)
    s = m.StateVector(c.n, torch.complex64)
    s.init("zero")
    s.apply(c)
    s.tensor.mul_(3.0)
    psi = to_host(s.tensor)[0]
    u = W.sample_uniforms(5000, seed=13)
    _check_against_oracle(psi, u, s.sample(u))


def test_sample_errors_and_empty():
    m = lib()
    s = m.StateVector(6, torch.complex64)
    s.init("zero")
    assert s.sample(np.zeros(0)).size == 0
    for bad in ([1.0], [-0.1], [np.nan]):
        with pytest.raises(m.SvError):
            s.sample(np.array(bad))
    # more than 2^32 samples in one call is refused before any array is read
    u1, o1 = np.zeros(1), np.zeros(1, np.uint64)
    st = m._lib.sv_sample(s._h, 1 << 33, u1.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          o1.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    assert st != 0 and b"2^32" in m._lib.sv_last_error()
    s.tensor.zero_()
    with pytest.raises(m.SvError):
        s.sample(np.array([0.3]))


@pytest.mark.parametrize("dtype", DTYPES)
def test_amplitudes_readout(dtype):
    m = lib()
    n, B = 13, 2
    psi0 = np.stack([W.random_state(n, 80 + b) for b in range(B)])
    if dtype == torch.complex64:
        psi0 = round_c64(psi0)
    s = m.StateVector(n, dtype, batch=B, tensor=to_dev(psi0, dtype))
    idx = np.array([0, 1, 17, 4095, 4096, (1 << n) - 1, 5, 5], np.uint64)
    got = s.amplitudes(idx)
    assert got.shape == (B, idx.size)
    assert np.array_equal(got, psi0[:, idx.astype(np.int64)])
    with pytest.raises(m.SvError):
        s.amplitudes(np.array([1 << n], np.uint64))


def test_uniform_32_qubits_exact():
    # full-size chunk layout (2^20 chunks) with exact probabilities 2^-32
    m = lib()
    n = 32
    s = m.StateVector(n, torch.complex64)
    s.init("uniform")
    u = W.sample_uniforms(20000, seed=14)
    got = s.sample(u)
    assert np.array_equal(got, np.floor(u * float(1 << n)).astype(np.uint64))


def test_grid33_samples_follow_output_distribution():
    # 33-qubit random grid circuit: the sampled outcomes j carry probabilities
    # with mean 2^n <p_j> = 2 when the output follows the Porter-Thomas law
    # (a sampler that ignored the probabilities would give 1); the sampled
    # amplitudes are read back from the state
    m = lib()
    c = W.grid33()
    s = m.StateVector(33, torch.complex64)
    s.init("zero_deferred")
    s.apply(c)
    u = W.sample_uniforms(8192, seed=15)
    got = s.sample(u)
    amp = s.amplitudes(got)[0]
    x = np.abs(amp) ** 2 * float(1 << 33)
    assert np.all(x > 0.0)
    assert abs(float(np.mean(x)) - 2.0) < 0.15, float(np.mean(x))
