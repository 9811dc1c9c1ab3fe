"""Full-size checks in the launch configuration bench.py times (complex64,
default options: plan-specialised tile passes of 2^13 amplitudes, 2^4-
amplitude segments, 512 threads).  The 33-qubit state has no independent
FP64 reference on the host, so it is checked through a 24-qubit cut of the
same circuit against the oracle, the norm, and the mirror circuit."""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_util import check_close, to_host

pytestmark = pytest.mark.gpu


def lib():
    import paper_2008_00216_amd as m
    return m


def test_grid33_cut24_against_oracle():
    m = lib()
    c = W.grid33().cut(24)
    s = m.StateVector(24, torch.complex64)
    s.init("zero")
    st = s.apply(c)
    assert st["passes"] > 1
    ref = oracle.simulate(c)
    check_close(to_host(s.tensor)[0], ref, torch.complex64, "grid33 cut 24")


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_grid33_cut28_against_stored_oracle_amplitudes(dtype):
    # the 28-qubit cut of the headline circuit in the launch configuration
    # the benchmark uses (tuned geometry, plan-specialised passes, product-
    # state input), against FP64 oracle amplitudes stored by
    # tests/golden/make_grid33_cut28.py
    from tests.golden import load as golden
    m = lib()
    idx, want, nrm_want = golden.grid33_cut28()
    c = W.grid33().cut(28)
    opts = m.make_opts(tile_bits=13, low_bits=4, threads=512) if dtype == torch.complex64 else m.make_opts()
    s = m.StateVector(28, dtype, opts=opts)
    s.init("zero_deferred")
    st = s.apply(c)
    assert st["passes"] > 1
    got = s.amplitudes(idx)[0]
    tol = 1e-5 if dtype == torch.complex64 else 1e-12
    err = float(np.max(np.abs(got - want)))
    assert err <= tol, err
    # Relative to the typical amplitude 2^{-n/2} (the absolute bar is loose
    # here): rounding errors of the G gate applications add like a random
    # walk, ||delta||_2 ~ sqrt(G) u, and the largest of the sampled
    # amplitude errors stays within a few times ||delta||_2 2^{-n/2}; the
    # bar is 16 sqrt(G) u, u = 2^-24 (c64) or 2^-53 (c128).
    u = 2.0 ** -24 if dtype == torch.complex64 else 2.0 ** -53
    rel = err * 2.0 ** (c.n / 2)
    print(f"cut28 {dtype}: max-abs {err:.3e}, max-abs * 2^(n/2) {rel:.3e}, bar {16 * math.sqrt(len(c)) * u:.3e}")
    assert rel <= 16 * math.sqrt(len(c)) * u, rel
    assert abs(float(s.norm()[0]) - nrm_want) < (1e-5 if dtype == torch.complex64 else 1e-12)
    del s
    torch.cuda.empty_cache()


def test_grid30_cut22_c128_against_oracle():
    m = lib()
    c = W.grid30().cut(22)
    s = m.StateVector(22, torch.complex128)
    s.init("zero")
    s.apply(c)
    check_close(to_host(s.tensor)[0], oracle.simulate(c), torch.complex128, "grid30 cut 22 c128")


def test_grid33_norm_and_mirror():
    m = lib()
    c = W.grid33()
    s = m.StateVector(33, torch.complex64)
    s.init("zero_deferred")
    s.apply(c)
    nrm = float(s.norm()[0])
    assert abs(nrm - 1.0) < 1e-5, nrm
    # the sweep spreads the state: no amplitude keeps a large share
    head = to_host(s.tensor[0, :1 << 16])
    assert np.max(np.abs(head)) < 1e-3
    s.apply(W.inverse(c))
    psi0 = complex(s.tensor[0, 0].item())
    nrm2 = float(s.norm()[0])
    dist = math.sqrt(max(0.0, nrm2 - 2.0 * psi0.real + 1.0))   # || psi - |0...0> ||_2
    assert abs(nrm2 - 1.0) < 2e-5 and dist < 1e-3, (psi0, nrm2, dist)
    tail = to_host(s.tensor[0, 1:1 << 16])
    assert np.max(np.abs(tail)) < 1e-4
    del s
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype,n", [(torch.complex64, 34), (torch.complex128, 33)])
def test_maximum_width_norm_and_mirror(dtype, n):
    # the widest states the library accepts (128 GiB): a shallow grid circuit
    # and its inverse return |0..0>
    m = lib()
    torch.cuda.empty_cache()
    c = W.grid_circuit(2, 17, 3, seed=1010) if n == 34 else W.grid_circuit(3, 11, 3, seed=1011)
    assert c.n == n
    s = m.StateVector(n, dtype)
    s.init("zero_deferred")
    st = s.apply(c)
    assert st["passes"] >= 1
    tol = 1e-5 if dtype == torch.complex64 else 1e-12
    assert abs(float(s.norm()[0]) - 1.0) < tol
    s.apply(W.inverse(c))
    a = s.amplitudes(np.array([0, 1, (1 << n) - 1], np.uint64))[0]
    assert abs(a[0] - 1.0) < 10 * tol and abs(a[1]) < tol and abs(a[2]) < tol, a
    del s
    torch.cuda.empty_cache()
