"""The C-ABI library loads on a machine without a GPU and exports every
entry point declared in include/sv.h; host-only calls work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sv.h")
LIB = os.path.join(ROOT, "paper_2008_00216_amd", "libsvmi.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sv_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("sv_create", "sv_destroy", "sv_init", "sv_apply_circuit", "sv_expect", "sv_norm",
              "sv_adjoint_grad", "sv_apply_batch", "sv_plan_info", "sv_plan_trace", "sv_last_error"):
        assert f in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libsvmi.so not built")
    lib = ctypes.CDLL(LIB)
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_binding_lists_the_same_symbols():
    m = pytest.importorskip("paper_2008_00216_amd")
    assert sorted(m.EXPORTED) == declared_functions()


def test_host_only_calls_and_errors():
    m = pytest.importorskip("paper_2008_00216_amd")
    import workloads as W
    st = m.plan_info(W.grid_circuit(3, 4, 6, seed=1))
    assert st["passes"] >= 1 and st["gates_in"] > 0 and st["alu_ops"] > 0
    bad = W.Circuit(3, [W.Gate("CZ", (0, 0))], 0)
    with pytest.raises(m.SvError) as e:
        m.plan_info(bad)
    assert e.value.status == 1
    assert m._lib.sv_version().decode()


def test_null_arguments_are_rejected_without_a_device():
    # argument validation happens before any device call, so these run on a
    # host without a GPU
    m = pytest.importorskip("paper_2008_00216_amd")
    lib = m._lib
    EINVAL = 1
    d = ctypes.c_double()
    u = ctypes.c_uint64()
    assert lib.sv_sample(None, 1, ctypes.byref(d), ctypes.byref(u)) == EINVAL
    assert b"ctx" in lib.sv_last_error()
    assert lib.sv_amplitudes(None, 1, ctypes.byref(u), ctypes.byref(d)) == EINVAL
    assert lib.sv_copy_state(None, None) == EINVAL
    assert lib.sv_norm(None, ctypes.byref(d)) == EINVAL
    assert lib.sv_apply_circuit_norm(None, None, None, ctypes.byref(d), None) == EINVAL
    assert lib.sv_apply_circuit(None, None, None, None) == EINVAL
