"""Argument validation at the C ABI (include/sv.h, "Errors"): every bad
argument is rejected with SV_EINVAL and a message before any device call, so
these run on a host without a GPU.  Device pointers here are never
dereferenced: validation fails first."""
import ctypes

import numpy as np
import pytest

m = pytest.importorskip("paper_2008_00216_amd")
import workloads as W  # noqa: E402

lib = m._lib
EINVAL = 1
FAKE = 0x7f0000000000          # 256-byte aligned stand-in for a device pointer


def create(n=10, dtype=m.SV_C64, batch=1, ptr=FAKE, nbytes=None, opts=None):
    h = ctypes.c_void_p()
    ab = 8 if dtype == m.SV_C64 else 16
    if nbytes is None:
        nbytes = batch * (1 << n) * ab
    st = lib.sv_create(ctypes.byref(h), n, dtype, batch, ctypes.c_void_p(ptr), nbytes, None,
                       ctypes.byref(opts) if opts is not None else None)
    return st, lib.sv_last_error().decode()


@pytest.mark.parametrize("kw, msg", [
    (dict(nbytes=(1 << 10) * 8 - 8), "state_bytes"),
    (dict(nbytes=(1 << 10) * 16), "state_bytes"),
    (dict(dtype=m.SV_C128, nbytes=(1 << 10) * 8), "state_bytes"),
    (dict(batch=2, nbytes=(1 << 10) * 8), "state_bytes"),
    (dict(ptr=FAKE + 8), "aligned"),
    (dict(ptr=FAKE + 4), "aligned"),
    (dict(ptr=0), "NULL"),
    (dict(n=0, nbytes=8), "out of range"),
    (dict(n=35, nbytes=8), "out of range"),
    (dict(n=34, dtype=m.SV_C128, nbytes=16), "out of range"),
    (dict(batch=0, nbytes=0), "batch"),
    (dict(batch=70000, nbytes=8), "batch"),
    (dict(dtype=3), "dtype"),
])
def test_create_rejects(kw, msg):
    st, err = create(**kw)
    assert st == EINVAL and msg in err, (st, err)


@pytest.mark.parametrize("field, value, msg", [
    ("max_fuse_k", 7, "max_fuse_k"), ("max_fuse_k", -1, "max_fuse_k"),
    ("tile_bits", 15, "tile_bits"), ("max_work_mib", -1, "max_work_mib"),
    ("plan_beam", 65, "plan_beam"), ("plan_beam", -1, "plan_beam"),
])
def test_create_rejects_options(field, value, msg):
    st, err = create(opts=m.make_opts(**{field: value}))
    assert st == EINVAL and msg in err, (st, err)


def _raw_circuit(n, recs, n_params=0, mats=None):
    """An sv_circuit built field by field (bypasses the binding's checks)."""
    gates = (m.SvGate * max(1, len(recs)))()
    for i, (op, qs, param, mat) in enumerate(recs):
        gates[i].op = op
        gates[i].nq = len(qs)
        for t, q in enumerate(qs):
            gates[i].q[t] = q
        gates[i].param = param
        gates[i].mat = mat
    mv = np.zeros(1, np.float64) if mats is None else np.ascontiguousarray(mats, np.float64)
    c = m.SvCircuit(n, len(recs), gates, int(mv.size if mats is not None else 0),
                    mv.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n_params)
    return c, (gates, mv)


def plan_status(c):
    st = m.SvStats()
    o = m.make_opts()
    r = lib.sv_plan_info(ctypes.byref(c), m.SV_C64, 0, ctypes.byref(o), ctypes.byref(st))
    return r, lib.sv_last_error().decode()


OP = m.OPS


@pytest.mark.parametrize("recs, n_params, mats, msg", [
    ([(OP["H"], (10,), -1, -1)], 0, None, "out of range"),
    ([(OP["H"], (-1,), -1, -1)], 0, None, "out of range"),
    ([(OP["CZ"], (3, 3), -1, -1)], 0, None, "duplicate"),
    ([(OP["CZ"], (1,), -1, -1)], 0, None, "nq"),
    ([(OP["H"], (0, 1), -1, -1)], 0, None, "nq"),
    ([(99, (0,), -1, -1)], 0, None, "unknown op"),
    ([(-1, (0,), -1, -1)], 0, None, "unknown op"),
    ([(OP["RX"], (0,), 2, -1)], 2, None, "param"),
    ([(OP["H"], (0,), 0, -1)], 1, None, "takes no parameter"),
    ([(OP["MAT"], (0,), -1, 2)], 0, np.zeros(8), "mat"),
    ([(OP["MAT"], (0,), -1, -1)], 0, np.zeros(8), "mat"),
    ([(OP["MAT"], (0, 1), -1, 0)], 0, np.zeros(8), "mat"),
])
def test_gate_validation(recs, n_params, mats, msg):
    c, keep = _raw_circuit(10, recs, n_params, mats)
    st, err = plan_status(c)
    assert st == EINVAL and msg in err, (st, err)


def test_seven_qubit_gate_struct_cannot_be_built():
    # sv_gate has room for 6 qubits: nq = 7 is rejected on its count alone
    c, keep = _raw_circuit(10, [(OP["MAT"], (0, 1, 2, 3, 4, 5), -1, 0)], 0, np.zeros(2 * 64 * 64))
    keep[0][0].nq = 7
    st, err = plan_status(c)
    assert st == EINVAL and "nq" in err


def test_batch_item_validation():
    circ = m.CircuitABI(W.layered_param_circuit(6, 2, 1))
    obs = m.PauliABI(W.z_sum(6))
    pr = np.zeros(circ.n_params)
    items = (m.SvBatchItem * 1)()
    items[0].circuit = ctypes.pointer(circ.c)
    items[0].params = pr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    items[0].d_state = FAKE + 8
    items[0].observable = ctypes.pointer(obs.p)
    e = np.zeros(1)
    g = np.zeros(circ.n_params)
    dp = ctypes.POINTER(ctypes.c_double)

    def call(count=1, its=items, flags=m.BATCH_FORWARD, dtype=m.SV_C64):
        r = lib.sv_apply_batch(count, its, dtype, None, flags, e.ctypes.data_as(dp), g.ctypes.data_as(dp), None, None)
        return r, lib.sv_last_error().decode()

    assert call()[0] == EINVAL and "aligned" in call()[1]
    items[0].d_state = FAKE
    r, err = call(flags=m.BATCH_GRAD)           # no lambda buffer
    assert r == EINVAL and "d_lambda" in err
    r, err = call(count=-1)
    assert r == EINVAL and "count" in err
    r, err = call(dtype=7)
    assert r == EINVAL and "dtype" in err
    items[0].params = None
    r, err = call()
    assert r == EINVAL and "params" in err
    r, err = call(its=None)
    assert r == EINVAL and "NULL" in err


def test_async_batch_validation():
    """sv_apply_batch_async validates like sv_apply_batch before anything is
    queued, and returns no job on error; sv_batch_finish rejects a NULL job."""
    circ = m.CircuitABI(W.layered_param_circuit(6, 2, 1))
    pr = np.zeros(circ.n_params)
    items = (m.SvBatchItem * 1)()
    items[0].circuit = ctypes.pointer(circ.c)
    items[0].params = pr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    items[0].d_state = FAKE
    items[0].observable = None
    job = ctypes.c_void_p(123)
    # energies of a forward batch need observables
    r = lib.sv_apply_batch_async(1, items, m.SV_C64, None, m.BATCH_FORWARD | m.BATCH_ENERGY, None, ctypes.byref(job))
    assert r == EINVAL and "observable" in lib.sv_last_error().decode()
    assert job.value is None
    items[0].d_state = FAKE + 8
    r = lib.sv_apply_batch_async(1, items, m.SV_C64, None, m.BATCH_FORWARD, None, ctypes.byref(job))
    assert r == EINVAL and "aligned" in lib.sv_last_error().decode()
    r = lib.sv_apply_batch_async(1, items, m.SV_C64, None, m.BATCH_FORWARD, None, None)
    assert r == EINVAL and "job" in lib.sv_last_error().decode()
    r = lib.sv_batch_finish(None, None, None, None)
    assert r == EINVAL and "job" in lib.sv_last_error().decode()


def test_entry_points_reject_null_context():
    d = ctypes.c_double()
    for f, args in (("sv_init", (None, 0, 0)), ("sv_expect", (None, None, ctypes.byref(d))),
                    ("sv_sync", (None,)), ("sv_destroy", (None,)), ("sv_set_opts", (None, None)),
                    ("sv_adjoint_grad", (None, None, None, None, None, 0, None, None, None)),
                    ("sv_tune", (None, None, None, None, None))):
        assert getattr(lib, f)(*args) == EINVAL, f
        assert lib.sv_last_error().decode(), f


def test_sf_plan_host_only():
    c = W.grid_circuit(2, 17, 20, seed=1007)
    mask = sum(1 << q for q in range(34) if q % 17 < 8 or q == 8)
    info = m.sf_plan(c, mask, work_bytes=80 << 30)
    # a 2 x 17 grid cut after column 8 of row 0 and column 7 of row 1: three
    # edges cross, one of them active in each of three of every four cycles
    assert (info["n_a"], info["n_b"], info["n_cross"]) == (17, 17, 15)
    assert info["n_inner"] == 15 and info["n_outer"] == 0 and info["paths"] == 2.0 ** 15
    assert info["work_bytes_all_inner"] == 2 * (1 << 32) * 8
    small = m.sf_plan(c, mask, work_bytes=info["work_bytes_all_inner"] // 8)
    assert small["n_inner"] + small["n_outer"] == 15 and small["n_outer"] > 0
    # SWAP across the cut has no two-term split: unsupported
    bad = W.Circuit(4, [W.Gate("SWAP", (0, 3))], 0)
    with pytest.raises(m.SvError) as e:
        m.sf_plan(bad, 0b0011)
    assert e.value.status == 4 and "crosses the cut" in str(e.value)
    with pytest.raises(m.SvError) as e:
        m.sf_plan(W.grid_circuit(2, 2, 1, seed=1), 0b1111)
    assert e.value.status == 4
