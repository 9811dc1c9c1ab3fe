"""Error paths that need a live context: the device work-area cap
(sv_opts.max_work_mib) turns an allocation into SV_ENOMEM without touching
the state, and the context stays usable afterwards."""
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


def test_work_cap_gives_enomem_and_leaves_state():
    m = lib()
    n = 22
    psi0 = round_c64(W.random_state(n, 5))
    t = to_dev(psi0)
    # the sampling tree needs 2^22 / 64 doubles = 512 KiB, within a 1 MiB cap
    s = m.StateVector(n, torch.complex64, tensor=t, opts=m.make_opts(max_work_mib=1))
    u = W.sample_uniforms(300000, 1)        # 2.4 MB of uniforms: above the 1 MiB cap
    with pytest.raises(m.SvError) as e:
        s.sample(u)
    assert e.value.status == m.SV_ENOMEM
    assert np.array_equal(to_host(t)[0], psi0)
    # within the cap the same context still works
    nrm = s.norm()[0]
    assert abs(nrm - oracle.norm2(psi0)) < 1e-6
    out = s.sample(u[:1000])
    assert out.shape == (1000,)
    # a circuit whose plan fits runs; a cap of 1 MiB is enough for it
    c = W.grid_circuit(2, 11, 4, seed=9)
    s.apply(c)
    ref = oracle.simulate(c, None, psi0)
    assert np.max(np.abs(to_host(t)[0] - ref)) < 1e-5
