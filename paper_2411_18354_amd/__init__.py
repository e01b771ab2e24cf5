"""Python binding of libsv.so, the MI355X state-vector library.

Argument marshalling only: every function here converts Python/torch
arguments into the C ABI declared in include/sv.h and calls the function of
the same name.  All arithmetic runs in the library's HIP kernels; torch only
provides device memory (tensors) and streams.  If libsv.so is missing the
import fails: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsv.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libsv.so not built at %s; run `python paper_2411_18354_amd/build.py`" % LIB_PATH)

_L = ctypes.CDLL(LIB_PATH)

SV_OK, SV_EINVAL, SV_ENOMEM, SV_EHIP, SV_ENOTSUP = 0, -1, -2, -3, -4
SV_C128, SV_C64, SV_CQ16, SV_CQ32 = 0, 1, 2, 3
SV_MODE_AUTO, SV_MODE_MASKED, SV_MODE_PAIR, SV_MODE_WAVE, SV_MODE_TILE = 0, 1, 2, 3, 4
MODES = {"auto": SV_MODE_AUTO, "masked": SV_MODE_MASKED, "pair": SV_MODE_PAIR,
         "wave": SV_MODE_WAVE, "tile": SV_MODE_TILE}


class SvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("sv error %d: %s" % (code, msg))
        self.code = code


class sv_state_t(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("n", ctypes.c_int32), ("dtype", ctypes.c_int32)]


_vp, _i32, _u64, _i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)
_sp = ctypes.POINTER(sv_state_t)


def _sig(name, args, res=ctypes.c_int):
    f = getattr(_L, name)
    f.argtypes = args
    f.restype = res
    return f


_L_last_error = _sig("sv_last_error", [], ctypes.c_char_p)
_sig("sv_version", [])
_sig("sv_alloc", [_sp, ctypes.c_int, ctypes.c_int])
_sig("sv_free", [_sp])
_sig("sv_init", [_sp, _u64, _vp])
_sig("sv_apply_gate", [_sp, ctypes.c_int, ctypes.POINTER(_i32), ctypes.c_int, _u64, _dp, ctypes.c_int, _vp])
_sig("sv_apply_gate_masks", [_sp, ctypes.c_int, _u64, _u64, _dp, ctypes.c_int, _vp])
_sig("sv_debug_pair_indices", [ctypes.c_int, ctypes.c_int, ctypes.POINTER(_i32), ctypes.c_int, _u64, _vp,
                               _i64, _vp])


def lib():
    return _L


def sv_last_error() -> str:
    return _L_last_error().decode()


def sv_version() -> int:
    return int(_L.sv_version())


def _check(rc: int):
    if rc != SV_OK:
        raise SvError(rc, sv_last_error())


# ---------------------------------------------------------------- marshalling

def _torch():
    import torch
    return torch


def stream_ptr(stream=None):
    """hipStream_t of a torch stream (default: the current stream)."""
    if isinstance(stream, (int, ctypes.c_void_p)):
        return ctypes.c_void_p(stream if isinstance(stream, int) else stream.value)
    torch = _torch()
    if stream is None:
        if not torch.cuda.is_available():
            return ctypes.c_void_p(0)  # host-only use: argument checks, no launch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.complex128:
        return SV_C128
    if t.dtype == torch.complex64:
        return SV_C64
    if t.dtype == torch.uint8:
        return SV_CQ16
    raise TypeError("state tensor must be complex128, complex64 or uint8 (SV_CQ16), got %s" % t.dtype)


def q16_nbytes(n: int) -> int:
    """Bytes of an n-qubit SV_CQ16 state: 4 per amplitude, then 1 per 64."""
    return (4 << n) + max(1, (1 << n) // 64)


def fixed_nbytes(n: int, dtype: int = SV_CQ16) -> int:
    """Bytes of an n-qubit fixed-point state (SV_CQ16: 4 per amplitude,
    SV_CQ32: 8), then one scale byte per 64 amplitudes."""
    per = {SV_CQ16: 4, SV_CQ32: 8}[dtype]
    return (per << n) + max(1, (1 << n) // 64)


class FixedState:
    """A fixed-point state: its bytes (a contiguous uint8 CUDA tensor), n and
    dtype (SV_CQ16 or SV_CQ32).  Accepted wherever a state is."""

    def __init__(self, n: int, dtype: int = SV_CQ16, data=None, device="cuda"):
        nbytes = fixed_nbytes(n, dtype)
        if data is None:
            data = _torch().empty(nbytes, dtype=_torch().uint8, device=device)
        if data.dtype != _torch().uint8 or data.numel() != nbytes:
            raise ValueError("fixed-point state of %d qubits needs %d uint8 bytes" % (n, nbytes))
        self.data, self.n, self.dtype = data, int(n), int(dtype)

    @property
    def device(self):
        return self.data.device


def _q16_qubits(nbytes: int) -> int:
    for n in range(1, 37):
        if q16_nbytes(n) == nbytes:
            return n
    raise ValueError("%d bytes is not the size of a fixed-point state" % nbytes)


def fixed_state(n: int, device="cuda"):
    """Uninitialised uint8 tensor holding an n-qubit SV_CQ16 state."""
    return _torch().empty(q16_nbytes(n), dtype=_torch().uint8, device=device)


def state_view(t, n: Optional[int] = None) -> sv_state_t:
    """sv_state_t view of a contiguous CUDA tensor: complex of 2^n elements,
    or uint8 of q16_nbytes(n) bytes for a fixed-point state."""
    if isinstance(t, sv_state_t):
        return t
    if isinstance(t, FixedState):
        if not t.data.is_cuda or not t.data.is_contiguous():
            raise ValueError("state must be a contiguous CUDA tensor")
        return sv_state_t(t.data.data_ptr(), t.n, t.dtype)
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("state must be a contiguous CUDA tensor")
    numel = t.numel()
    code = _dtype_code(t)
    if code == SV_CQ16:
        if n is None:
            n = _q16_qubits(numel)
        if numel != q16_nbytes(n):
            raise ValueError("fixed-point state has %d bytes, expected %d" % (numel, q16_nbytes(n)))
        return sv_state_t(t.data_ptr(), n, code)
    if n is None:
        n = numel.bit_length() - 1
    if numel != (1 << n):
        raise ValueError("state has %d elements, expected 2^%d" % (numel, n))
    return sv_state_t(t.data_ptr(), n, code)


def _u8(U) -> ctypes.Array:
    """8 doubles (a, b, c, d as re, im) from a 2x2 complex array or 8 floats."""
    import numpy as np
    a = np.asarray(U)
    if np.iscomplexobj(a) or a.shape == (2, 2):
        a = np.asarray(a, dtype=np.complex128).reshape(4)
        vals = [v for c in a for v in (float(c.real), float(c.imag))]
    else:
        vals = [float(v) for v in a.reshape(-1)]
    if len(vals) != 8:
        raise ValueError("U must be 2x2 complex or 8 doubles")
    return (ctypes.c_double * 8)(*vals)


def _ctrl_array(controls: Sequence[int]):
    arr = (_i32 * max(1, len(controls)))(*[int(c) for c in controls])
    return arr


def ctrl_vals_mask(controls: Sequence[int], values: Sequence[int] = ()) -> int:
    vals = list(values) if len(values) else [1] * len(controls)
    if len(vals) != len(controls):
        raise ValueError("values must align with controls")
    m = 0
    for q, v in zip(controls, vals):
        if v:
            m |= 1 << int(q)
    return m


# ---------------------------------------------------------------- C ABI

def sv_alloc(n: int, dtype: int = SV_C128) -> sv_state_t:
    s = sv_state_t()
    _check(_L.sv_alloc(ctypes.byref(s), int(n), int(dtype)))
    return s


def sv_free(s: sv_state_t) -> None:
    _check(_L.sv_free(ctypes.byref(s)))


def sv_init(state, basis_index: int = 0, stream=None) -> None:
    s = state_view(state)
    _check(_L.sv_init(ctypes.byref(s), int(basis_index), stream_ptr(stream)))


def sv_apply_gate(state, target: int, controls: Sequence[int] = (), ctrl_vals: Optional[int] = None,
                  U=None, mode="auto", stream=None) -> None:
    """Apply U (2x2) on target with controls; ctrl_vals is the qubit-indexed
    mask of required control values (default: all controls require 1)."""
    s = state_view(state)
    if ctrl_vals is None:
        ctrl_vals = ctrl_vals_mask(controls)
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    _check(_L.sv_apply_gate(ctypes.byref(s), int(target), _ctrl_array(controls), len(controls),
                            int(ctrl_vals), _u8(U), m, stream_ptr(stream)))


def sv_apply_gate_masks(state, target: int, ctrl_mask: int, ctrl_vals: int, U, mode="auto", stream=None) -> None:
    s = state_view(state)
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    _check(_L.sv_apply_gate_masks(ctypes.byref(s), int(target), int(ctrl_mask), int(ctrl_vals), _u8(U), m,
                                  stream_ptr(stream)))


def sv_debug_pair_indices(n: int, target: int, controls: Sequence[int] = (), ctrl_vals: Optional[int] = None,
                          out=None, stream=None):
    """Device uint64 tensor of the first pair element for every reduced
    iteration index, from the kernels' own index function."""
    torch = _torch()
    if ctrl_vals is None:
        ctrl_vals = ctrl_vals_mask(controls)
    count = 1 << (n - 1 - len(controls))
    if out is None:
        out = torch.empty(count, dtype=torch.uint64 if hasattr(torch, "uint64") else torch.int64, device="cuda")
    _check(_L.sv_debug_pair_indices(int(n), int(target), _ctrl_array(controls), len(controls), int(ctrl_vals),
                                    ctypes.c_void_p(out.data_ptr()), out.numel(), stream_ptr(stream)))
    return out


_sig("sv_gate_plan", [ctypes.c_int, ctypes.c_int, ctypes.c_int, _u64, _u64, ctypes.c_int, ctypes.c_char_p,
                      ctypes.c_int, ctypes.POINTER(_u64)])


_sig("sv_hbm_probe", [_sp, _u64, _u64, ctypes.c_int, _vp])

PROBE_OPS = {"rmw": 0, "read": 1, "write": 2}


def sv_hbm_probe(state, fixed_mask: int = 0, fixed_vals: int = 0, op="rmw", stream=None) -> None:
    """Measurement helper: stream over the amplitudes matching fixed_vals on
    fixed_mask ("rmw" keeps the values, "read" reads only, "write" zeroes)."""
    s = state_view(state)
    o = PROBE_OPS[op] if isinstance(op, str) else int(op)
    _check(_L.sv_hbm_probe(ctypes.byref(s), int(fixed_mask), int(fixed_vals), o, stream_ptr(stream)))


def sv_gate_plan(n: int, dtype: int, target: int, ctrl_mask: int = 0, ctrl_vals: int = 0, mode="auto"):
    """(kernel name, work items) that sv_apply_gate would launch."""
    buf = ctypes.create_string_buffer(256)
    it = _u64(0)
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    _check(_L.sv_gate_plan(int(n), int(dtype), int(target), int(ctrl_mask), int(ctrl_vals), m, buf, 256,
                           ctypes.byref(it)))
    return buf.value.decode(), int(it.value)


_sig("sv_tune_set", [ctypes.c_char_p, _i64])
_sig("sv_tune_get", [ctypes.c_char_p, ctypes.POINTER(_i64)])


# every knob sv_tune_set accepts (include/sv.h lists their ranges)
TUNE_KEYS = ("granule_bits_c128", "granule_bits_c64", "low_policy", "wave_auto", "tile_log2_c128",
             "tile_log2_c64", "tile_low_bits_c128", "tile_low_bits_c64", "fuse_min_gates", "dense_qubits",
             "dense_min_gates", "pair_unroll", "masked_unroll", "masked_block", "fuse_group", "fuse_pairs",
             "plan_lookahead", "fuse_perm", "batch_split", "phase_sweep_min_c128", "phase_sweep_min_c64")


def sv_tune_set(key: str, value: int) -> None:
    _check(_L.sv_tune_set(key.encode(), int(value)))


_sig("sv_autotune", [ctypes.c_int, ctypes.c_int, ctypes.c_char_p, ctypes.c_char_p, ctypes.c_int, _vp])
_sig("sv_tune_load", [ctypes.c_char_p])


def sv_autotune(n: int = 24, dtype: int = SV_C128, cache_path: Optional[str] = None, stream=None) -> str:
    """Measure and apply the fastest launch choices; returns the timing report."""
    buf = ctypes.create_string_buffer(8192)
    _check(_L.sv_autotune(int(n), int(dtype), cache_path.encode() if cache_path else None, buf, 8192,
                          stream_ptr(stream)))
    return buf.value.decode()


def sv_tune_load(path: str) -> None:
    _check(_L.sv_tune_load(path.encode()))


def sv_tune_get(key: str) -> int:
    v = _i64(0)
    _check(_L.sv_tune_get(key.encode(), ctypes.byref(v)))
    return int(v.value)


_sig("sv_copy_state", [_sp, _sp, _vp])
_sig("sv_convert", [_sp, _sp, _vp])
_sig("sv_state_bytes", [ctypes.c_int, ctypes.c_int, ctypes.POINTER(_u64)])


def sv_copy_state(dst, src, stream=None) -> None:
    a, b = state_view(dst), state_view(src)
    _check(_L.sv_copy_state(ctypes.byref(a), ctypes.byref(b), stream_ptr(stream)))


def sv_convert(dst, src, stream=None) -> None:
    """Convert src into dst (same n, any dtypes; SV_CQ16 encode/decode)."""
    a, b = state_view(dst), state_view(src)
    _check(_L.sv_convert(ctypes.byref(a), ctypes.byref(b), stream_ptr(stream)))


def sv_state_bytes(n: int, dtype: int) -> int:
    out = _u64(0)
    _check(_L.sv_state_bytes(int(n), int(dtype), ctypes.byref(out)))
    return int(out.value)


# ---------------------------------------------------------------- circuits

SV_G_MATRIX, SV_G_X, SV_G_Y, SV_G_Z, SV_G_H, SV_G_RX, SV_G_RY, SV_G_RZ, SV_G_P = range(9)
SV_G_ADJOINT = 0x100
SV_FUSE, SV_GRAPH, SV_MASKED, SV_DENSE, SV_REMAP = 1, 2, 4, 8, 16
KIND_CODES = {"U": SV_G_MATRIX, "X": SV_G_X, "Y": SV_G_Y, "Z": SV_G_Z, "H": SV_G_H,
              "RX": SV_G_RX, "RY": SV_G_RY, "RZ": SV_G_RZ, "P": SV_G_P}


class sv_gate_t(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("target", ctypes.c_int32), ("ctrl_mask", ctypes.c_uint64),
                ("ctrl_vals", ctypes.c_uint64), ("param", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("theta", ctypes.c_double), ("U", ctypes.c_double * 8)]


def _gate_dtype():
    import numpy as np
    dt = np.dtype([("kind", "<i4"), ("target", "<i4"), ("ctrl_mask", "<u8"), ("ctrl_vals", "<u8"),
                   ("param", "<i4"), ("reserved", "<i4"), ("theta", "<f8"), ("U", "<f8", (8,))])
    assert dt.itemsize == ctypes.sizeof(sv_gate_t)
    return dt


_GATE_DTYPE = _gate_dtype()


def kind_code(kind: str) -> int:
    adj = kind.startswith("~")
    return KIND_CODES[kind[1:] if adj else kind] | (SV_G_ADJOINT if adj else 0)


def circuit_gates(circ_or_gates):
    """ctypes array of sv_gate_t from a workloads.Circuit (or a gate list)."""
    import numpy as np
    gates = getattr(circ_or_gates, "gates", circ_or_gates)
    n = len(gates)
    K, T, CM, CV, P, TH, mats = [], [], [], [], [], [], []
    codes = {}
    for i, g in enumerate(gates):
        code = codes.get(g.kind)
        if code is None:
            code = codes[g.kind] = kind_code(g.kind)
        cm = cv = 0
        if g.controls:
            vals = g.values
            for j, q in enumerate(g.controls):
                b = 1 << int(q)
                cm |= b
                if not len(vals) or vals[j]:
                    cv |= b
        p = g.param
        K.append(code)
        T.append(int(g.target))
        CM.append(cm)
        CV.append(cv)
        P.append(-1 if p is None or p < 0 else int(p))
        TH.append(float(g.theta))
        if g.matrix is not None:
            mats.append((i, g.matrix))
    rec = np.zeros(max(1, n), dtype=_GATE_DTYPE)
    if n:
        rec["kind"][:n] = K
        rec["target"][:n] = T
        rec["ctrl_mask"][:n] = np.array(CM, dtype=np.uint64)
        rec["ctrl_vals"][:n] = np.array(CV, dtype=np.uint64)
        rec["param"][:n] = P
        rec["theta"][:n] = TH
        for i, m in mats:
            rec["U"][i] = [float(x) for x in m]
    arr = (sv_gate_t * max(1, n)).from_buffer_copy(rec.tobytes())
    arr._sv_count = len(gates)
    return arr


_sig("sv_gate_matrix", [ctypes.c_int, ctypes.c_double, _dp, _dp])
_sig("sv_circuit_create", [ctypes.c_int, ctypes.c_int, ctypes.POINTER(sv_gate_t), ctypes.c_int, ctypes.c_int,
                           ctypes.c_int, ctypes.POINTER(_vp)])
_sig("sv_circuit_run", [_vp, _sp, _vp, _vp])
_sig("sv_circuit_info", [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64)])
_sig("sv_circuit_destroy", [_vp])
_sig("sv_apply_circuit", [_sp, ctypes.POINTER(sv_gate_t), ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp])


def sv_gate_matrix(kind, theta: float = 0.0, U=None):
    """The library's 2x2 matrix for a gate kind (code or name), as 8 doubles."""
    k = kind_code(kind) if isinstance(kind, str) else int(kind)
    out = (ctypes.c_double * 8)()
    u = _u8(U) if U is not None else None
    _check(_L.sv_gate_matrix(k, float(theta), u, out))
    return list(out)


def _params_ptr(params):
    if params is None:
        return ctypes.c_void_p(0), 0
    return ctypes.c_void_p(params.data_ptr()), int(params.numel())


class Circuit:
    """Owns an sv_circuit_t plan (sv_circuit_create / run / destroy)."""

    def __init__(self, n: int, gates, dtype: int = SV_C128, nparams: int = 0, flags: int = SV_FUSE):
        arr = gates if isinstance(gates, ctypes.Array) else circuit_gates(gates)
        count = getattr(arr, "_sv_count", len(arr))
        h = _vp()
        _check(_L.sv_circuit_create(int(n), int(dtype), arr, count, int(nparams), int(flags), ctypes.byref(h)))
        self._h = h
        self.n, self.dtype, self.nparams, self.flags = n, dtype, nparams, flags

    def run(self, state, params=None, stream=None) -> None:
        s = state_view(state)
        p, _ = _params_ptr(params)
        _check(_L.sv_circuit_run(self._h, ctypes.byref(s), p, stream_ptr(stream)))

    def info(self):
        a, b, c = _i64(0), _i64(0), _i64(0)
        _check(_L.sv_circuit_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"passes": a.value, "fused_gates": b.value, "fused_runs": c.value}

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _L.sv_circuit_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sv_apply_circuit(state, gates, params=None, nparams: Optional[int] = None, flags: int = SV_FUSE,
                     stream=None) -> None:
    s = state_view(state)
    arr = gates if isinstance(gates, ctypes.Array) else circuit_gates(gates)
    count = getattr(arr, "_sv_count", len(arr))
    p, np_ = _params_ptr(params)
    if nparams is None:
        nparams = np_
    _check(_L.sv_apply_circuit(ctypes.byref(s), arr, count, p, int(nparams), int(flags), stream_ptr(stream)))


_sig("sv_circuit_plan", [ctypes.c_int, ctypes.c_int, ctypes.POINTER(sv_gate_t), ctypes.c_int, ctypes.c_int,
                         ctypes.c_int, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i64)])


def sv_circuit_plan(n: int, gates, dtype: int = SV_C128, nparams: int = 0, flags: int = SV_FUSE):
    """Host-only planner dry run: (order, pass_of, npasses)."""
    arr = gates if isinstance(gates, ctypes.Array) else circuit_gates(gates)
    count = getattr(arr, "_sv_count", len(arr))
    order = (_i32 * max(1, count))()
    pas = (_i32 * max(1, count))()
    npas = _i64(0)
    _check(_L.sv_circuit_plan(int(n), int(dtype), arr, count, int(nparams), int(flags), order, pas,
                              ctypes.byref(npas)))
    return list(order)[:count], list(pas)[:count], int(npas.value)


_sig("sv_swap_qubits", [_sp, ctypes.POINTER(ctypes.c_int32), ctypes.c_int, _vp])


def sv_swap_qubits(state, pairs, stream=None) -> None:
    """Exchange the qubits of each (a, b) in pairs (disjoint pairs)."""
    s = state_view(state)
    flat = [int(q) for p in pairs for q in p]
    arr = (ctypes.c_int32 * max(1, len(flat)))(*flat)
    _check(_L.sv_swap_qubits(ctypes.byref(s), arr, len(pairs), stream_ptr(stream)))


_sig("sv_apply_dense_low", [_sp, ctypes.c_int, _dp, _vp])


def sv_apply_dense_low(state, k: int, M, stream=None) -> None:
    """Apply the 2^k x 2^k complex matrix M to the k lowest qubits (MFMA)."""
    import numpy as np
    s = state_view(state)
    m = np.ascontiguousarray(np.asarray(M, dtype=np.complex128).reshape(1 << k, 1 << k))
    buf = np.ascontiguousarray(np.stack([m.real, m.imag], axis=-1).reshape(-1))
    _check(_L.sv_apply_dense_low(ctypes.byref(s), int(k), buf.ctypes.data_as(_dp), stream_ptr(stream)))


from .observables import (sv_pauli_t, pauli_terms, sv_expect, sv_expect_noalloc, sv_expect_terms,  # noqa: E402
                          sv_apply_pauli_sum, sv_adjoint_grad, AdjointPlan, SvExpectation, ExpectationModel)
from .batched import sv_apply_circuits_batched, sv_adjoint_grad_batched, Batch  # noqa: E402
