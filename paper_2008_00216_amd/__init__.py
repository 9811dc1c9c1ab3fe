"""Python binding of libsvmi, the MI355X state-vector sweep library.

Argument marshalling only: every step of the simulation runs in the HIP
kernels behind the C ABI declared in include/sv.h.  PyTorch supplies device
memory (the state tensors) and the HIP stream.  If the shared library has not
been built, importing this package raises ImportError; there is no CPU
fallback.

Circuits are passed duck-typed: any object with ``n``, ``gates`` (items with
``op``, ``qubits``, ``param``, ``theta``, ``mat``) and ``n_params``; Pauli sums
with ``coeff``, ``x_mask``, ``z_mask`` arrays.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime before libsvmi)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsvmi.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2008_00216_amd/build.py "
                      "(or __graft_entry__.build()) first")

_lib = ctypes.CDLL(LIB_PATH)

SV_OK, SV_EINVAL, SV_ENOMEM, SV_EDEVICE, SV_EUNSUPPORTED = 0, 1, 2, 3, 4
SV_C64, SV_C128 = 1, 2
INIT_ZERO, INIT_BASIS, INIT_UNIFORM, INIT_ZERO_DEFERRED = 0, 1, 2, 3
BATCH_FORWARD, BATCH_GRAD, BATCH_INIT_ZERO, BATCH_ENERGY = 1, 2, 4, 8

OPS = {
    "I": 0, "H": 1, "X": 2, "Y": 3, "Z": 4, "S": 5, "SDG": 6, "T": 7, "TDG": 8,
    "SQRTX": 9, "SQRTY": 10, "SQRTW": 11, "SQRTXDG": 12, "SQRTYDG": 13, "SQRTWDG": 14,
    "RX": 15, "RY": 16, "RZ": 17, "P": 18, "CZ": 19, "CNOT": 20, "SWAP": 21, "CP": 22, "MAT": 23, "DIAG": 24,
}


class SvGate(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("nq", ctypes.c_int32), ("q", ctypes.c_int32 * 6),
                ("param", ctypes.c_int32), ("mat", ctypes.c_int32), ("theta", ctypes.c_double)]


# numpy view of sv_gate (same layout as SvGate: 48 bytes, theta at offset 40)
_GATE_DTYPE = np.dtype({"names": ["op", "nq", "q", "param", "mat", "theta"],
                        "formats": [np.int32, np.int32, (np.int32, 6), np.int32, np.int32, np.float64],
                        "offsets": [0, 4, 8, 32, 36, 40], "itemsize": 48})
assert ctypes.sizeof(SvGate) == _GATE_DTYPE.itemsize


class SvCircuit(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_gates", ctypes.c_int32),
                ("gates", ctypes.POINTER(SvGate)), ("n_mat_doubles", ctypes.c_int64),
                ("mats", ctypes.POINTER(ctypes.c_double)), ("n_params", ctypes.c_int32)]


class SvPauliSum(ctypes.Structure):
    _fields_ = [("n_terms", ctypes.c_int32), ("coeff", ctypes.POINTER(ctypes.c_double)),
                ("x_mask", ctypes.POINTER(ctypes.c_uint64)), ("z_mask", ctypes.POINTER(ctypes.c_uint64))]


class SvOpts(ctypes.Structure):
    _fields_ = [("max_fuse_k", ctypes.c_int32), ("tile_bits", ctypes.c_int32),
                ("low_bits", ctypes.c_int32), ("plain", ctypes.c_int32), ("threads", ctypes.c_int32),
                ("product_init", ctypes.c_int32), ("structured", ctypes.c_int32),
                ("timing", ctypes.c_int32), ("jit", ctypes.c_int32), ("max_work_mib", ctypes.c_int32),
                ("batch_tuned", ctypes.c_int32), ("paper", ctypes.c_int32),
                ("plan_beam", ctypes.c_int32)]


class SvStats(ctypes.Structure):
    _fields_ = [("gates_in", ctypes.c_int32), ("passes", ctypes.c_int32), ("phases", ctypes.c_int32),
                ("dense_ops", ctypes.c_int32), ("diag_ops", ctypes.c_int32), ("launches", ctypes.c_int32),
                ("folded_init", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("plan_ms", ctypes.c_double), ("hbm_bytes", ctypes.c_double), ("flops", ctypes.c_double),
                ("alu_ops", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class SvSfInfo(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_a", ctypes.c_int32), ("n_b", ctypes.c_int32),
                ("n_cross", ctypes.c_int32), ("n_inner", ctypes.c_int32), ("n_outer", ctypes.c_int32),
                ("paths", ctypes.c_double), ("work_bytes_all_inner", ctypes.c_size_t),
                ("work_bytes_min", ctypes.c_size_t)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SvBatchItem(ctypes.Structure):
    _fields_ = [("circuit", ctypes.POINTER(SvCircuit)), ("params", ctypes.POINTER(ctypes.c_double)),
                ("d_state", ctypes.c_void_p), ("d_lambda", ctypes.c_void_p),
                ("observable", ctypes.POINTER(SvPauliSum))]


_vp, _dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
_lib.sv_opts_default.argtypes = [ctypes.POINTER(SvOpts)]
_lib.sv_opts_default.restype = None
_lib.sv_last_error.restype = ctypes.c_char_p
_lib.sv_version.restype = ctypes.c_char_p
_lib.sv_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp,
                           ctypes.c_size_t, _vp, ctypes.POINTER(SvOpts)]
_lib.sv_destroy.argtypes = [_vp]
_lib.sv_set_stream.argtypes = [_vp, _vp]
_lib.sv_set_opts.argtypes = [_vp, ctypes.POINTER(SvOpts)]
_lib.sv_init.argtypes = [_vp, ctypes.c_int32, ctypes.c_uint64]
_lib.sv_apply_circuit.argtypes = [_vp, ctypes.POINTER(SvCircuit), _dp, ctypes.POINTER(SvStats)]
_lib.sv_expect.argtypes = [_vp, ctypes.POINTER(SvPauliSum), _dp]
_lib.sv_expect_noalloc.argtypes = [_vp, ctypes.POINTER(SvPauliSum), _dp]
_lib.sv_norm.argtypes = [_vp, _dp]
_lib.sv_apply_circuit_norm.argtypes = [_vp, ctypes.POINTER(SvCircuit), _dp, _dp, ctypes.POINTER(SvStats)]
_lib.sv_copy_state.argtypes = [_vp, _vp]
_lib.sv_sample.argtypes = [_vp, ctypes.c_int64, _dp, ctypes.POINTER(ctypes.c_uint64)]
_lib.sv_amplitudes.argtypes = [_vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_uint64), _dp]
_lib.sv_adjoint_grad.argtypes = [_vp, ctypes.POINTER(SvCircuit), _dp, ctypes.POINTER(SvPauliSum), _vp,
                                 ctypes.c_size_t, _dp, _dp, ctypes.POINTER(SvStats)]
_lib.sv_apply_batch.argtypes = [ctypes.c_int32, ctypes.POINTER(SvBatchItem), ctypes.c_int32, _vp, ctypes.c_int32,
                                _dp, _dp, ctypes.POINTER(SvOpts), ctypes.POINTER(SvStats)]
_lib.sv_sf_plan.argtypes = [ctypes.POINTER(SvCircuit), ctypes.c_uint64, ctypes.c_int32, ctypes.c_size_t,
                            ctypes.POINTER(SvSfInfo)]
_lib.sv_sf_create.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(SvCircuit), ctypes.c_uint64, ctypes.c_int32, _vp,
                              ctypes.c_size_t, _vp, ctypes.POINTER(SvOpts)]
_lib.sv_sf_destroy.argtypes = [_vp]
_lib.sv_sf_amplitudes.argtypes = [_vp, _dp, ctypes.c_int64, ctypes.POINTER(ctypes.c_uint64), _dp,
                                  ctypes.POINTER(SvStats)]
_lib.sv_tune_batch.argtypes = [ctypes.c_int32, ctypes.POINTER(SvBatchItem), ctypes.c_int32, _vp, ctypes.c_int32,
                               ctypes.POINTER(SvOpts), ctypes.POINTER(ctypes.c_int32)]
_lib.sv_batch_tuning.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(SvOpts)]
_lib.sv_apply_batch_async.argtypes = [ctypes.c_int32, ctypes.POINTER(SvBatchItem), ctypes.c_int32, _vp,
                                      ctypes.c_int32, ctypes.POINTER(SvOpts), ctypes.POINTER(_vp)]
_lib.sv_batch_finish.argtypes = [_vp, _dp, _dp, ctypes.POINTER(SvStats)]
_lib.sv_sync.argtypes = [_vp]
_lib.sv_timing.argtypes = [_vp, _dp, ctypes.POINTER(ctypes.c_int64), _dp]
_lib.sv_plan_info.argtypes = [ctypes.POINTER(SvCircuit), ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(SvOpts),
                              ctypes.POINTER(SvStats)]
_lib.sv_tune.argtypes = [_vp, ctypes.POINTER(SvCircuit), _dp, ctypes.POINTER(SvOpts), _dp]
_lib.sv_plan_trace.argtypes = [ctypes.POINTER(SvCircuit), _dp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(SvOpts),
                               ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
for _f in ("sv_create", "sv_destroy", "sv_set_stream", "sv_set_opts", "sv_init", "sv_apply_circuit",
           "sv_apply_circuit_norm", "sv_expect", "sv_expect_noalloc", "sv_norm", "sv_copy_state", "sv_sample", "sv_amplitudes",
           "sv_adjoint_grad", "sv_apply_batch", "sv_sync", "sv_timing", "sv_plan_info", "sv_plan_trace",
           "sv_tune", "sv_sf_plan", "sv_sf_create", "sv_sf_destroy", "sv_sf_amplitudes", "sv_tune_batch",
           "sv_batch_tuning", "sv_apply_batch_async", "sv_batch_finish"):
    getattr(_lib, _f).restype = ctypes.c_int32

EXPORTED = ("sv_opts_default", "sv_create", "sv_destroy", "sv_set_stream", "sv_set_opts", "sv_init",
            "sv_apply_circuit", "sv_apply_circuit_norm", "sv_expect", "sv_expect_noalloc", "sv_norm", "sv_copy_state", "sv_sample",
            "sv_amplitudes", "sv_adjoint_grad", "sv_apply_batch", "sv_sync", "sv_timing", "sv_plan_info",
            "sv_plan_trace", "sv_tune", "sv_sf_plan", "sv_sf_create", "sv_sf_destroy", "sv_sf_amplitudes",
            "sv_tune_batch", "sv_batch_tuning", "sv_apply_batch_async", "sv_batch_finish", "sv_last_error",
            "sv_version")


class SvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"status {status}: {msg}")
        self.status = status


def _check(st: int):
    if st != SV_OK:
        raise SvError(st, _lib.sv_last_error().decode())


def version() -> str:
    return _lib.sv_version().decode()


def make_opts(**kw) -> SvOpts:
    o = SvOpts()
    _lib.sv_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, int(v))
    return o


class CircuitABI:
    """ctypes view of a circuit (keeps its arrays alive)."""

    def __init__(self, circ):
        gates = list(circ.gates)
        self.n = int(circ.n)
        self.n_params = int(circ.n_params)
        ng = max(1, len(gates))
        rec = np.zeros(ng, _GATE_DTYPE)
        mats = []
        moff = 0
        if gates:
            try:
                rec["op"][:len(gates)] = [OPS[g.op] for g in gates]
            except KeyError as e:
                raise KeyError(f"unknown gate {e.args[0]}") from None
            rec["nq"][:len(gates)] = [len(g.qubits) for g in gates]
            q = rec["q"]
            for t in range(6):
                sel = [i for i, g in enumerate(gates) if len(g.qubits) > t]
                if sel:
                    q[sel, t] = [gates[i].qubits[t] for i in sel]
            rec["param"][:len(gates)] = [g.param for g in gates]
            rec["theta"][:len(gates)] = [g.theta for g in gates]
            rec["mat"][:len(gates)] = -1
            for i, g in enumerate(gates):
                if g.op in ("MAT", "DIAG"):
                    m = np.ascontiguousarray(g.mat, np.complex128).view(np.float64).ravel()
                    rec["mat"][i] = moff
                    mats.append(m)
                    moff += m.size
        self._rec = rec
        arr = ctypes.cast(rec.ctypes.data, ctypes.POINTER(SvGate))
        self._gates = arr
        self._mats = np.concatenate(mats) if mats else np.zeros(1, np.float64)
        self.c = SvCircuit(self.n, len(gates), arr, int(moff),
                           self._mats.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), self.n_params)


class PauliABI:
    def __init__(self, pauli):
        self._c = np.ascontiguousarray(pauli.coeff, np.float64)
        self._x = np.ascontiguousarray(pauli.x_mask, np.uint64)
        self._z = np.ascontiguousarray(pauli.z_mask, np.uint64)
        self.p = SvPauliSum(int(self._c.size), self._c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            self._x.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                            self._z.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))


def _as_circuit(circ):
    return circ if isinstance(circ, CircuitABI) else CircuitABI(circ)


def _as_pauli(p):
    return p if isinstance(p, PauliABI) else PauliABI(p)


def _params_ptr(params, batch, n_params):
    if params is None or n_params == 0:
        return None, None
    p = np.ascontiguousarray(np.asarray(params, np.float64).reshape(batch, n_params))
    return p, p.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class StateVector:
    """A batch of 2^n-amplitude states in a torch tensor, driven through libsvmi."""

    def __init__(self, n: int, dtype=torch.complex64, batch: int = 1, device="cuda",
                 opts: Optional[SvOpts] = None, tensor: Optional[torch.Tensor] = None):
        if dtype not in (torch.complex64, torch.complex128):
            raise TypeError("dtype must be complex64 or complex128")
        self.n, self.batch, self.dtype = int(n), int(batch), dtype
        if tensor is None:
            tensor = torch.empty((batch, 1 << n), dtype=dtype, device=device)
        if tensor.dtype != dtype or not tensor.is_cuda or not tensor.is_contiguous():
            raise ValueError("state tensor must be a contiguous CUDA tensor of the given dtype")
        self.tensor = tensor
        self.opts = opts if opts is not None else make_opts()
        h = ctypes.c_void_p()
        _check(_lib.sv_create(ctypes.byref(h), self.n, SV_C64 if dtype == torch.complex64 else SV_C128,
                              self.batch, ctypes.c_void_p(tensor.data_ptr()),
                              tensor.numel() * tensor.element_size(), _stream_handle(),
                              ctypes.byref(self.opts)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.sv_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        _check(_lib.sv_set_stream(self._h, _stream_handle()))

    def set_opts(self, opts: SvOpts):
        self.opts = opts
        _check(_lib.sv_set_opts(self._h, ctypes.byref(opts)))

    def init(self, kind: str = "zero", index: int = 0):
        self._stream()
        k = {"zero": INIT_ZERO, "basis": INIT_BASIS, "uniform": INIT_UNIFORM,
             "zero_deferred": INIT_ZERO_DEFERRED}[kind]
        _check(_lib.sv_init(self._h, k, int(index)))
        return self

    def apply(self, circ, params=None) -> dict:
        self._stream()
        c = _as_circuit(circ)
        _, pp = _params_ptr(params, self.batch, c.n_params)
        st = SvStats()
        _check(_lib.sv_apply_circuit(self._h, ctypes.byref(c.c), pp, ctypes.byref(st)))
        return st.as_dict()

    def apply_norm(self, circ, params=None):
        """apply() and the FP64 norms ||psi_b||^2 from the same sweep:
        returns (stats, norms)."""
        self._stream()
        c = _as_circuit(circ)
        _, pp = _params_ptr(params, self.batch, c.n_params)
        st = SvStats()
        out = np.zeros(self.batch, np.float64)
        _check(_lib.sv_apply_circuit_norm(self._h, ctypes.byref(c.c), pp,
                                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(st)))
        return st.as_dict(), out

    def expect(self, pauli) -> np.ndarray:
        self._stream()
        p = _as_pauli(pauli)
        out = np.zeros(self.batch, np.float64)
        _check(_lib.sv_expect(self._h, ctypes.byref(p.p), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def expect_noalloc(self, pauli) -> np.ndarray:
        """expect() through sv_expect_noalloc: the library allocates nothing
        (its work area is a fixed per-device array)."""
        self._stream()
        p = _as_pauli(pauli)
        out = np.zeros(self.batch, np.float64)
        _check(_lib.sv_expect_noalloc(self._h, ctypes.byref(p.p),
                                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def norm(self) -> np.ndarray:
        self._stream()
        out = np.zeros(self.batch, np.float64)
        _check(_lib.sv_norm(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def copy_from(self, other: "StateVector"):
        """This context's states = other's (same width, dtype and batch)."""
        self._stream()
        _check(_lib.sv_copy_state(self._h, other._h))
        return self

    def sample(self, uniforms) -> np.ndarray:
        """Bit strings measured from every state, one per random number in
        [0, 1): uniforms of shape (count,) for one state or (batch, count);
        returns uint64 indices of the same shape (bit q = qubit q)."""
        self._stream()
        u = np.ascontiguousarray(uniforms, dtype=np.float64)
        shape = u.shape
        if u.ndim == 1:
            if self.batch != 1:
                raise ValueError("uniforms must have shape (batch, count) for a batched context")
            u = u.reshape(1, -1)
        if u.ndim != 2 or u.shape[0] != self.batch:
            raise ValueError("uniforms must have shape (count,) or (batch, count)")
        out = np.zeros(u.shape, np.uint64)
        _check(_lib.sv_sample(self._h, u.shape[1], u.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
        return out.reshape(shape)

    def amplitudes(self, indices) -> np.ndarray:
        """Complex128 amplitudes psi_b[indices] of shape (batch, len(indices))."""
        self._stream()
        idx = np.ascontiguousarray(indices, dtype=np.uint64).reshape(-1)
        out = np.zeros((self.batch, idx.size, 2), np.float64)
        _check(_lib.sv_amplitudes(self._h, idx.size, idx.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out[..., 0] + 1j * out[..., 1]

    def adjoint_grad(self, circ, params, pauli, scratch: Optional[torch.Tensor] = None):
        """Returns (energy[batch], grad[batch, n_params]); see sv_adjoint_grad."""
        self._stream()
        c = _as_circuit(circ)
        p = _as_pauli(pauli)
        _, pp = _params_ptr(params, self.batch, c.n_params)
        if scratch is None:
            scratch = torch.empty_like(self.tensor)
        e = np.zeros(self.batch, np.float64)
        g = np.zeros((self.batch, max(1, c.n_params)), np.float64)
        st = SvStats()
        _check(_lib.sv_adjoint_grad(self._h, ctypes.byref(c.c), pp, ctypes.byref(p.p),
                                    ctypes.c_void_p(scratch.data_ptr()), scratch.numel() * scratch.element_size(),
                                    e.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(st)))
        self.last_stats = st.as_dict()
        return e, g[:, :c.n_params]

    def tune(self, circ, params=None):
        """Pick the fastest tile geometry for circ (sv_tune; destroys the state).
        Returns (chosen options, best ms or -1 when remembered)."""
        self._stream()
        c = _as_circuit(circ)
        _, pp = _params_ptr(params, self.batch, c.n_params)
        o = SvOpts()
        ms = ctypes.c_double()
        _check(_lib.sv_tune(self._h, ctypes.byref(c.c), pp, ctypes.byref(o), ctypes.byref(ms)))
        self.opts = o
        return {k: getattr(o, k) for k, _ in o._fields_ if k != "reserved"}, ms.value

    def sync(self):
        _check(_lib.sv_sync(self._h))

    def timing(self):
        """(tile-pass ms, launches, algorithmic bytes) since the last call."""
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        by = ctypes.c_double()
        _check(_lib.sv_timing(self._h, ctypes.byref(ms), ctypes.byref(cnt), ctypes.byref(by)))
        return ms.value, cnt.value, by.value


def plan_info(circ, dtype=torch.complex64, adjoint=False, opts: Optional[SvOpts] = None) -> dict:
    """Host-only planning statistics (no GPU needed)."""
    c = _as_circuit(circ)
    st = SvStats()
    o = opts if opts is not None else make_opts()
    _check(_lib.sv_plan_info(ctypes.byref(c.c), SV_C64 if dtype == torch.complex64 else SV_C128,
                             1 if adjoint else 0, ctypes.byref(o), ctypes.byref(st)))
    return st.as_dict()


def plan_trace(circ, params=None, dtype=torch.complex64, adjoint=False, opts: Optional[SvOpts] = None) -> str:
    """Host-only trace of the fused plan (sv_plan_trace); no GPU needed."""
    c = _as_circuit(circ)
    pr = None
    if c.n_params:
        pr = np.ascontiguousarray(np.asarray(params, np.float64).reshape(-1))
    o = opts if opts is not None else make_opts()
    n = ctypes.c_size_t(0)
    args = (ctypes.byref(c.c), pr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if pr is not None else None,
            SV_C64 if dtype == torch.complex64 else SV_C128, 1 if adjoint else 0, ctypes.byref(o))
    _check(_lib.sv_plan_trace(*args, None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value + 1)
    _check(_lib.sv_plan_trace(*args, buf, n.value + 1, ctypes.byref(n)))
    return buf.value.decode()


def _batch_items(circuits, params, states, observables, lambdas):
    count = len(circuits)
    cabi = [_as_circuit(c) for c in circuits]
    pabi = [_as_pauli(p) for p in observables]
    items = (SvBatchItem * max(1, count))()
    keep = [cabi, pabi]
    for i in range(count):
        pr = None
        if cabi[i].n_params:
            pr = np.ascontiguousarray(np.asarray(params[i], np.float64))
            keep.append(pr)
        items[i].circuit = ctypes.pointer(cabi[i].c)
        items[i].params = pr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if pr is not None else None
        items[i].d_state = states[i].data_ptr()
        items[i].d_lambda = lambdas[i].data_ptr() if lambdas is not None else None
        items[i].observable = ctypes.pointer(pabi[i].p)
    return items, keep


def tune_batch(circuits: Sequence, params: Sequence, states: Sequence[torch.Tensor], observables: Sequence,
               lambdas: Optional[Sequence[torch.Tensor]] = None, grad: bool = False,
               opts: Optional[SvOpts] = None) -> int:
    """sv_tune_batch: per-width fusion mode and tile geometry by measurement
    (overwrites the states).  Returns the number of widths tuned; apply with
    make_opts(batch_tuned=1)."""
    items, keep = _batch_items(circuits, params, states, observables, lambdas)
    n = ctypes.c_int32()
    o = opts if opts is not None else make_opts()
    _check(_lib.sv_tune_batch(len(circuits), items, SV_C64 if states[0].dtype == torch.complex64 else SV_C128,
                              _stream_handle(), BATCH_GRAD if grad else BATCH_FORWARD, ctypes.byref(o),
                              ctypes.byref(n)))
    return n.value


def batch_tuning(n_qubits: int, dtype=torch.complex64, grad: bool = False) -> dict:
    """The remembered sv_tune_batch choice for one width."""
    o = SvOpts()
    _check(_lib.sv_batch_tuning(SV_C64 if dtype == torch.complex64 else SV_C128, 1 if grad else 0, int(n_qubits),
                                ctypes.byref(o)))
    return {"structured": o.structured, "max_fuse_k": o.max_fuse_k, "tile_bits": o.tile_bits,
            "low_bits": o.low_bits}


def apply_batch(circuits: Sequence, params: Sequence, states: Sequence[torch.Tensor],
                observables: Sequence, lambdas: Optional[Sequence[torch.Tensor]] = None,
                grad: bool = False, init_zero: bool = True, opts: Optional[SvOpts] = None):
    """Heterogeneous batch through sv_apply_batch.  Returns (energies, grads list, stats)."""
    count = len(circuits)
    cabi = [_as_circuit(c) for c in circuits]
    pabi = [_as_pauli(p) for p in observables]
    dtype = states[0].dtype if count else torch.complex64
    items = (SvBatchItem * max(1, count))()
    keep = []
    for i in range(count):
        pr = None
        if cabi[i].n_params:
            pr = np.ascontiguousarray(np.asarray(params[i], np.float64))
            keep.append(pr)
        items[i].circuit = ctypes.pointer(cabi[i].c)
        items[i].params = pr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if pr is not None else None
        items[i].d_state = states[i].data_ptr()
        items[i].d_lambda = lambdas[i].data_ptr() if lambdas is not None else None
        items[i].observable = ctypes.pointer(pabi[i].p)
    ntot = sum(c.n_params for c in cabi)
    energies = np.zeros(max(1, count), np.float64)
    grads = np.zeros(max(1, ntot), np.float64)
    flags = (BATCH_GRAD if grad else BATCH_FORWARD) | (BATCH_INIT_ZERO if init_zero else 0)
    st = SvStats()
    o = opts if opts is not None else make_opts()
    _check(_lib.sv_apply_batch(count, items, SV_C64 if dtype == torch.complex64 else SV_C128,
                               _stream_handle(), flags,
                               energies.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               grads.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               ctypes.byref(o), ctypes.byref(st)))
    out, off = [], 0
    for c in cabi:
        out.append(grads[off:off + c.n_params].copy())
        off += c.n_params
    return energies[:count], out, st.as_dict()


class BatchJob:
    """A batch queued by apply_batch_async; finish() waits and returns
    (energies, grads list, stats) like apply_batch."""

    def __init__(self, handle, count, nparams, grad, energies, keep):
        self._h = handle
        self._count = count
        self._nparams = nparams
        self._grad = grad
        self._energies = energies
        self._keep = keep      # device buffers the job still uses

    def finish(self):
        if self._h is None:
            raise RuntimeError("batch job already finished")
        h, self._h = self._h, None
        energies = np.zeros(max(1, self._count), np.float64)
        grads = np.zeros(max(1, sum(self._nparams)), np.float64)
        st = SvStats()
        _check(_lib.sv_batch_finish(h, energies.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
                                    if self._energies else None,
                                    grads.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if self._grad else None,
                                    ctypes.byref(st)))
        self._keep = None
        out, off = [], 0
        for n in self._nparams:
            out.append(grads[off:off + n].copy())
            off += n
        return energies[:self._count], out, st.as_dict()

    def __del__(self):
        # a job that is dropped unfinished is still waited for, so its slot is freed
        if getattr(self, "_h", None) is not None:
            try:
                self.finish()
            except Exception:
                pass


def apply_batch_async(circuits: Sequence, params: Sequence, states: Sequence[torch.Tensor],
                      observables: Sequence, lambdas: Optional[Sequence[torch.Tensor]] = None,
                      grad: bool = False, init_zero: bool = True, energies: bool = True,
                      opts: Optional[SvOpts] = None) -> BatchJob:
    """sv_apply_batch_async: queue the batch and return at once; the host can
    prepare the next batch while this one runs.  BatchJob.finish() gives the
    results.  At most two jobs may be unfinished per device."""
    count = len(circuits)
    items, keep = _batch_items(circuits, params, states, observables, lambdas)
    cabi = keep[0]
    flags = (BATCH_GRAD if grad else BATCH_FORWARD) | (BATCH_INIT_ZERO if init_zero else 0) | \
            (BATCH_ENERGY if (energies and not grad) else 0)
    h = _vp()
    o = opts if opts is not None else make_opts()
    _check(_lib.sv_apply_batch_async(count, items, SV_C64 if (not count or states[0].dtype == torch.complex64)
                                     else SV_C128, _stream_handle(), flags, ctypes.byref(o), ctypes.byref(h)))
    return BatchJob(h, count, [c.n_params for c in cabi], grad, energies or grad,
                    (list(states), list(lambdas) if lambdas is not None else None))


def sf_plan(circ, half_mask: int, dtype=torch.complex64, work_bytes: int = 0) -> dict:
    """Host-only statistics of a Schroedinger-Feynman split (sv_sf_plan)."""
    c = _as_circuit(circ)
    info = SvSfInfo()
    _check(_lib.sv_sf_plan(ctypes.byref(c.c), int(half_mask), SV_C64 if dtype == torch.complex64 else SV_C128,
                           int(work_bytes), ctypes.byref(info)))
    return info.as_dict()


class SchrodingerFeynman:
    """Amplitudes of a circuit cut into two halves (sv_sf_*): half A holds the
    qubits set in half_mask.  The device work area is a torch tensor owned by
    this object (by default large enough to hold every path bit)."""

    def __init__(self, circ, half_mask: int, dtype=torch.complex64, work_bytes: Optional[int] = None,
                 opts: Optional[SvOpts] = None, device="cuda"):
        self._c = _as_circuit(circ)
        self.dtype = dtype
        dt = SV_C64 if dtype == torch.complex64 else SV_C128
        info = sf_plan(self._c, half_mask, dtype, 0)
        if work_bytes is None:
            work_bytes = info["work_bytes_all_inner"]
        self.work = torch.empty(int(work_bytes), dtype=torch.uint8, device=device)
        self.opts = opts if opts is not None else make_opts()
        h = ctypes.c_void_p()
        _check(_lib.sv_sf_create(ctypes.byref(h), ctypes.byref(self._c.c), int(half_mask), dt,
                                 ctypes.c_void_p(self.work.data_ptr()), int(work_bytes), _stream_handle(),
                                 ctypes.byref(self.opts)))
        self._h = h
        self.info = sf_plan(self._c, half_mask, dtype, int(work_bytes))

    def amplitudes(self, indices, params=None):
        """(complex128 amplitudes of the given indices, stats dict)."""
        idx = np.ascontiguousarray(indices, dtype=np.uint64).reshape(-1)
        out = np.zeros((idx.size, 2), np.float64)
        _, pp = _params_ptr(params, 1, self._c.n_params)
        st = SvStats()
        _check(_lib.sv_sf_amplitudes(self._h, pp, idx.size, idx.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(st)))
        return out[:, 0] + 1j * out[:, 1], st.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            _lib.sv_sf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Energy(torch.autograd.Function):
    """E(theta) = <psi(theta)|H|psi(theta)>, psi(theta) = U(theta)|0...0>, with the
    gradient from the adjoint sweep (sv_adjoint_grad).  theta: [batch, n_params]
    FP64 CPU tensor; returns [batch] FP64."""

    @staticmethod
    def forward(ctx, theta, sv: StateVector, circ, pauli):
        th = theta.detach().cpu().numpy().astype(np.float64)
        if not ctx.needs_input_grad[0]:
            # forward only: one sweep and the FP64 expectation, no adjoint
            sv.init("zero_deferred")
            sv.apply(circ, th)
            return torch.from_numpy(sv.expect(pauli))
        sv.init("zero_deferred")
        e, g = sv.adjoint_grad(circ, th, pauli)
        ctx.save_for_backward(torch.from_numpy(g))
        return torch.from_numpy(e)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out.reshape(-1, 1).to(g.dtype) * g, None, None, None
