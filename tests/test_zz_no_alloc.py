"""sv_expect_noalloc (the entry point that allocates nothing) against
sv_expect through the C ABI: the same kernels over a fixed device work
area, so the values must agree bit for bit, on two calls in a row (the
second on a smaller input), and with the FP64 oracle within tolerance."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_util import round_c64, to_dev

pytestmark = pytest.mark.gpu


def lib():
    import paper_2008_00216_amd as m
    return m


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_noalloc_matches_expect(dtype):
    m = lib()
    cases = [(16, 3, W.ansatz_observable(16)), (9, 1, W.z_sum(9))]   # second call: smaller input
    for n, batch, obs in cases:
        psi = np.stack([W.random_state(n, 40 + n + b) for b in range(batch)])
        if dtype == torch.complex64:
            psi = round_c64(psi)
        s = m.StateVector(n, dtype, batch=batch, tensor=to_dev(psi, dtype))
        got = s.expect_noalloc(obs)
        want = s.expect(obs)
        assert np.array_equal(got, want), (n, got, want)
        again = s.expect_noalloc(obs)
        assert np.array_equal(again, want)
        for b in range(batch):
            ref = oracle.expect(psi[b], obs)
            assert abs(got[b] - ref) < (1e-12 if dtype == torch.complex128 else 1e-10), (n, b, got[b], ref)
        s.close()


def test_noalloc_rejects_what_does_not_fit():
    m = lib()
    n, batch = 23, 130          # 130 states x 4096 FP64 partials: above the 4 MiB area
    t = torch.empty((batch, 1 << n), dtype=torch.complex64, device="cuda")
    s = m.StateVector(n, torch.complex64, batch=batch, tensor=t)
    with pytest.raises(m.SvError) as e:
        s.expect_noalloc(W.z_sum(n))
    assert e.value.status == m.SV_EINVAL and "work area" in str(e.value)
    s.close()
    del t
    torch.cuda.empty_cache()
