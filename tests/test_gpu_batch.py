"""Heterogeneous batches in one persistent launch (sv_apply_batch) against
the oracle and against the one-circuit-at-a-time path."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.gpu_util import to_host

pytestmark = pytest.mark.gpu


def lib():
    import paper_2008_00216_amd as m
    return m


def small_batch(count, seed0):
    return W.batch_circuits(count, n_lo=5, n_hi=15, l_lo=2, l_hi=6, seed0=seed0)


def test_batch_forward_energies_and_states():
    m = lib()
    circs = small_batch(20, 500)
    params = [W.uniform_params(1, c.n_params, 600 + i)[0] for i, c in enumerate(circs)]
    obs = [W.z_sum(c.n) for c in circs]
    states = [torch.empty(1 << c.n, dtype=torch.complex64, device="cuda") for c in circs]
    e, _, st = m.apply_batch(circs, params, states, obs, grad=False, init_zero=True)
    assert st["launches"] == 2
    for i, c in enumerate(circs):
        ref = oracle.simulate(c, params[i])
        got = to_host(states[i])
        assert np.max(np.abs(got - ref)) < 1e-5
        assert abs(e[i] - oracle.expect(ref, obs[i])) < 1e-5
        # same kernels and plan shape one circuit at a time: identical amplitudes
        s = m.StateVector(c.n, torch.complex64,
                          opts=m.make_opts(tile_bits=12, threads=256, jit=-1, product_init=0))
        s.init("zero")
        s.apply(c, params[i])
        assert np.array_equal(to_host(s.tensor)[0], got)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_batch_adjoint_gradients(dtype):
    m = lib()
    circs = small_batch(16, 700)
    params = [W.uniform_params(1, c.n_params, 800 + i)[0] for i, c in enumerate(circs)]
    obs = [W.z_sum(c.n) if i % 2 else W.ansatz_observable(c.n) for i, c in enumerate(circs)]
    states = [torch.empty(1 << c.n, dtype=dtype, device="cuda") for c in circs]
    lams = [torch.empty_like(s) for s in states]
    e, g, st = m.apply_batch(circs, params, states, obs, lambdas=lams, grad=True, init_zero=True)
    tol = 2e-4 if dtype == torch.complex64 else 1e-10
    for i, c in enumerate(circs):
        assert abs(e[i] - oracle.energy(c, params[i], obs[i])) < tol
        which = list(range(0, c.n_params, max(1, c.n_params // 6)))
        ref = oracle.grad_param_shift(c, params[i], obs[i], which=which)
        np.testing.assert_allclose(g[i][which], ref, atol=tol)
        # the one-at-a-time adjoint with the same plan shape gives the same gradients
        s = m.StateVector(c.n, dtype, opts=m.make_opts(tile_bits=12 if dtype == torch.complex64 else 11,
                                                       threads=256, jit=-1, product_init=0))
        s.init("zero")
        e1, g1 = s.adjoint_grad(c, params[i][None, :], obs[i])
        np.testing.assert_allclose(g1[0], g[i], atol=tol)


@pytest.mark.parametrize("beam", [1, 8])
def test_batch_plan_beam_widths(beam):
    # items wider than the 2^12-amplitude tile take several passes, whose
    # local sets differ with the planner's beam width (68 forward passes in
    # all greedily, 64 at width 8); every width gives the oracle's energies
    # and gradients
    m = lib()
    circs = W.batch_circuits(10, n_lo=15, n_hi=18, l_lo=20, l_hi=30, seed0=910)
    params = [W.uniform_params(1, c.n_params, 950 + i)[0] for i, c in enumerate(circs)]
    obs = [W.z_sum(c.n) if i % 2 else W.ansatz_observable(c.n) for i, c in enumerate(circs)]
    states = [torch.empty(1 << c.n, dtype=torch.complex64, device="cuda") for c in circs]
    lams = [torch.empty_like(s) for s in states]
    e, g, _ = m.apply_batch(circs, params, states, obs, lambdas=lams, grad=True, init_zero=True,
                            opts=m.make_opts(plan_beam=beam))
    for i, c in enumerate(circs):
        assert abs(e[i] - oracle.energy(c, params[i], obs[i])) < 2e-4, (beam, i)
        which = list(range(0, c.n_params, max(1, c.n_params // 3)))
        ref = oracle.grad_param_shift(c, params[i], obs[i], which=which)
        np.testing.assert_allclose(g[i][which], ref, atol=2e-4)


def test_batch_planned_up_front_matches_overlapped():
    """With max_work_mib set, both directions are planned before the first
    launch; otherwise the backward plans are built while the forward launch
    runs.  Both give the same energies, gradients and states, bit for bit,
    and an empty batch is a no-op."""
    m = lib()
    circs = small_batch(24, 910)
    params = [W.uniform_params(1, c.n_params, 920 + i)[0] for i, c in enumerate(circs)]
    obs = [W.z_sum(c.n) for c in circs]
    out = []
    for o in (None, m.make_opts(max_work_mib=1 << 16)):
        states = [torch.empty(1 << c.n, dtype=torch.complex64, device="cuda") for c in circs]
        lams = [torch.empty_like(t) for t in states]
        e, g, st = m.apply_batch(circs, params, states, obs, lambdas=lams, grad=True, init_zero=True, opts=o)
        assert st["launches"] == 3
        out.append((e, g, [to_host(t) for t in states]))
    (e0, g0, s0), (e1, g1, s1) = out
    assert np.array_equal(e0, e1)
    for i in range(len(circs)):
        assert np.array_equal(g0[i], g1[i])
        assert np.array_equal(s0[i], s1[i])
    e, g, st = m.apply_batch([], [], [], [], grad=False, init_zero=True)
    assert len(e) == 0


def test_async_batch_matches_sync_and_pipelines():
    """sv_apply_batch_async + sv_batch_finish give what sv_apply_batch gives,
    bit for bit (forward with energies, and gradients); two jobs on the same
    states can be in flight at once (the stream orders them), a third is
    refused until one is finished."""
    m = lib()
    circs = small_batch(18, 950)
    params = [W.uniform_params(1, c.n_params, 960 + i)[0] for i, c in enumerate(circs)]
    obs = [W.z_sum(c.n) for c in circs]
    states = [torch.empty(1 << c.n, dtype=torch.complex64, device="cuda") for c in circs]
    lams = [torch.empty_like(t) for t in states]
    e0, g0, _ = m.apply_batch(circs, params, states, obs, lambdas=lams, grad=True, init_zero=True)
    ef, _, _ = m.apply_batch(circs, params, states, obs, grad=False, init_zero=True)
    j1 = m.apply_batch_async(circs, params, states, obs, lambdas=lams, grad=True, init_zero=True)
    j2 = m.apply_batch_async(circs, params, states, obs, lambdas=lams, grad=True, init_zero=True)
    with pytest.raises(m.SvError) as ex:
        m.apply_batch_async(circs, params, states, obs, lambdas=lams, grad=True, init_zero=True)
    assert "in flight" in str(ex.value)
    e1, g1, st1 = j1.finish()
    j3 = m.apply_batch_async(circs, params, states, obs, grad=False, init_zero=True, energies=True)
    e2, g2, _ = j2.finish()
    e3, _, _ = j3.finish()
    assert st1["launches"] == 3
    assert np.array_equal(e0, e1) and np.array_equal(e0, e2)
    for i in range(len(circs)):
        assert np.array_equal(g0[i], g1[i]) and np.array_equal(g0[i], g2[i])
    # the last job on these states was the forward batch
    assert np.array_equal(ef, e3)
    for i, c in enumerate(circs):
        ref = oracle.simulate(c, params[i])
        assert np.max(np.abs(to_host(states[i]) - ref)) < 1e-5
    with pytest.raises(RuntimeError):
        j1.finish()


def test_batch_long_circuits_gradients():
    """Long circuits (30-40 layers, one or two tile passes each) in one
    persistent launch: gradients finite and equal to the shift rule."""
    m = lib()
    circs = W.batch_circuits(4, n_lo=10, n_hi=13, l_lo=30, l_hi=40, seed0=7100)
    params = [W.uniform_params(1, c.n_params, 7200 + i)[0] for i, c in enumerate(circs)]
    obs = [W.z_sum(c.n) for c in circs]
    states = [torch.empty(1 << c.n, dtype=torch.complex64, device="cuda") for c in circs]
    lams = [torch.empty_like(t) for t in states]
    e, g, _ = m.apply_batch(circs, params, states, obs, lambdas=lams, grad=True, init_zero=True)
    for i, c in enumerate(circs):
        assert np.all(np.isfinite(g[i])), i
        ref = oracle.grad_param_shift(c, params[i], obs[i])
        sel = list(range(0, c.n_params, 29))
        np.testing.assert_allclose(g[i][sel], ref[sel], atol=2e-4)


def test_tuned_batch_matches_oracle(tmp_path, monkeypatch):
    """sv_tune_batch picks a fusion mode and tile geometry per width by
    timing; the batch run with those choices gives the oracle's energies and
    gradients."""
    import oracle
    import paper_2008_00216_amd as m
    monkeypatch.setenv("SVMI_BATCH_TUNE_CACHE", str(tmp_path / "bt.txt"))
    widths = [8, 12, 13, 15, 15, 16]
    circs = [W.layered_param_circuit(n, 6, 90 + i) for i, n in enumerate(widths)]
    params = [W.uniform_params(1, c.n_params, 190 + i)[0] for i, c in enumerate(circs)]
    obs = [W.z_sum(c.n) for c in circs]
    states = [torch.zeros((1, 1 << c.n), dtype=torch.complex64, device="cuda") for c in circs]
    lams = [torch.zeros_like(t) for t in states]
    tuned = m.tune_batch(circs, params, states, obs, lambdas=lams, grad=True)
    assert tuned == len(set(widths))
    for n in set(widths):
        g = m.batch_tuning(n, grad=True)
        assert g["structured"] in (0, 1) and 2 <= g["max_fuse_k"] <= 4
    e, gr, st = m.apply_batch(circs, params, states, obs, lambdas=lams, grad=True,
                              opts=m.make_opts(batch_tuned=1))
    for i, c in enumerate(circs):
        assert abs(e[i] - oracle.energy(c, params[i], obs[i])) < 2e-5
        which = list(range(0, c.n_params, 9))
        ref = oracle.grad_param_shift(c, params[i], obs[i], which=which)
        assert np.max(np.abs(gr[i][which] - ref)) < 2e-5, i
