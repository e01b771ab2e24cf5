"""CPU oracle for the state-vector simulator (test infrastructure only).

Plain, slow, obviously correct reference for what the GPU library computes.
Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package; the GPU library never does, and the two
share no code.  Inner loops are the C functions in ``sv_oracle.c`` (double
precision, fixed evaluation order); this module adds gate matrices, circuits,
expectation values and reference gradients, each citing the passage of the
paper (arXiv:2411.18354) or the textbook definition it follows.

Pins against things other than the oracle itself live in
``tests/test_oracle_pins.py``.  Parity-unpinned functions: none.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Iterable, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sv_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-fopenmp"]


def build(force: bool = True) -> str:
    """Compile sv_oracle.c with gcc into liboracle.so next to it."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        u64 = ctypes.c_uint64
        L.or_apply_gate.argtypes = [dp, ctypes.c_int, ctypes.c_int, u64, u64, dp]
        L.or_apply_gate.restype = None
        L.or_gate_amplitude.argtypes = [dp, ctypes.c_int, ctypes.c_int, u64, u64, dp, u64, dp]
        L.or_gate_amplitude.restype = None
        L.or_pair_list.argtypes = [ctypes.c_int, ctypes.c_int, u64, u64, ctypes.POINTER(u64)]
        L.or_pair_list.restype = ctypes.c_int64
        L.or_expect_pauli.argtypes = [dp, ctypes.c_int, u64, u64, dp]
        L.or_expect_pauli.restype = None
        L.or_add_pauli.argtypes = [dp, dp, ctypes.c_int, u64, u64, ctypes.c_double]
        L.or_add_pauli.restype = None
        L.or_norm2.argtypes = [dp, ctypes.c_int]
        L.or_norm2.restype = ctypes.c_double
        L.or_basis.argtypes = [dp, ctypes.c_int, u64]
        L.or_basis.restype = None
        L.or_set_num_threads.argtypes = [ctypes.c_int]
        L.or_set_num_threads.restype = None
        L.or_apply_block_low.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp]
        L.or_apply_block_low.restype = None
        L.or_swap_qubits.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.or_swap_qubits.restype = None
        i16p = ctypes.POINTER(ctypes.c_int16)
        i8p = ctypes.POINTER(ctypes.c_int8)
        L.or_q16_scale.argtypes = [ctypes.c_float]
        L.or_q16_scale.restype = ctypes.c_int
        L.or_q16_code.argtypes = [ctypes.c_float, ctypes.c_int]
        L.or_q16_code.restype = ctypes.c_int16
        L.or_q16_encode.argtypes = [dp, ctypes.c_int, i16p, i8p]
        L.or_q16_encode.restype = None
        L.or_q16_decode.argtypes = [i16p, i8p, ctypes.c_int, dp]
        L.or_q16_decode.restype = None
        L.or_q16_apply_gate.argtypes = [i16p, i8p, ctypes.c_int, ctypes.c_int, u64, u64, dp]
        L.or_q16_apply_gate.restype = None
        i32p = ctypes.POINTER(ctypes.c_int32)
        L.or_q32_scale.argtypes = [ctypes.c_double]
        L.or_q32_scale.restype = ctypes.c_int
        L.or_q32_code.argtypes = [ctypes.c_double, ctypes.c_int]
        L.or_q32_code.restype = ctypes.c_int32
        L.or_q32_encode.argtypes = [dp, ctypes.c_int, i32p, i8p]
        L.or_q32_encode.restype = None
        L.or_q32_decode.argtypes = [i32p, i8p, ctypes.c_int, dp]
        L.or_q32_decode.restype = None
        L.or_q32_apply_gate.argtypes = [i32p, i8p, ctypes.c_int, ctypes.c_int, u64, u64, dp]
        L.or_q32_apply_gate.restype = None
        L.or_num_threads.argtypes = []
        L.or_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_num_threads(k: int) -> None:
    """Threads of later parallel loops (timing only: results do not depend
    on it)."""
    lib().or_set_num_threads(int(k))


# --------------------------------------------------------------------------
# gate matrices (Nielsen & Chuang conventions; X and H as printed in Sec. I)
# --------------------------------------------------------------------------

def gate_matrix(kind: str, theta: float = 0.0, matrix=None) -> np.ndarray:
    """2x2 complex matrix acting on (C_k, C_{k+2^t}) with bit t of k clear.

    X = [[0,1],[1,0]], H = [[1,1],[1,-1]]/sqrt2 (Sec. I); Y = [[0,-i],[i,0]],
    Z = diag(1,-1); RX/RY/RZ(theta) = exp(-i theta P/2); P(theta) =
    diag(1, e^{i theta}) so that the QFT rotation R_m is P(2 pi / 2^m).
    A kind prefixed by '~' is the conjugate transpose (the inverse)."""
    if kind.startswith("~"):
        return gate_matrix(kind[1:], theta, matrix).conj().T.copy()
    c, s = np.cos(theta / 2.0), np.sin(theta / 2.0)
    if kind == "X":
        return np.array([[0, 1], [1, 0]], dtype=np.complex128)
    if kind == "Y":
        return np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
    if kind == "Z":
        return np.array([[1, 0], [0, -1]], dtype=np.complex128)
    if kind == "H":
        return np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)
    if kind == "RX":
        return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)
    if kind == "RY":
        return np.array([[c, -s], [s, c]], dtype=np.complex128)
    if kind == "RZ":
        return np.array([[np.exp(-0.5j * theta), 0], [0, np.exp(0.5j * theta)]], dtype=np.complex128)
    if kind == "P":
        return np.array([[1, 0], [0, np.exp(1j * theta)]], dtype=np.complex128)
    if kind == "U":
        m = np.asarray(matrix, dtype=np.float64).reshape(4, 2)
        return (m[:, 0] + 1j * m[:, 1]).reshape(2, 2)
    raise ValueError("unknown gate kind %r" % kind)


def _u8(U: np.ndarray) -> np.ndarray:
    U = np.asarray(U, dtype=np.complex128).reshape(2, 2)
    return np.ascontiguousarray(np.stack([U.real, U.imag], axis=-1).reshape(8), dtype=np.float64)


def masks(controls: Sequence[int], values: Sequence[int] = ()) -> tuple:
    """Qubit-indexed (ctrl_mask, ctrl_vals) for a control list."""
    vals = values if len(values) else [1] * len(controls)
    cm = cv = 0
    for q, v in zip(controls, vals):
        cm |= 1 << int(q)
        if v:
            cv |= 1 << int(q)
    return cm, cv


def gate_angle(g, params: Optional[np.ndarray]) -> float:
    if g.param is not None and g.param >= 0:
        return float(params[g.param])
    return float(g.theta)


# --------------------------------------------------------------------------
# state operations
# --------------------------------------------------------------------------

def zero_state(n: int) -> np.ndarray:
    psi = np.empty(1 << n, dtype=np.complex128)
    lib().or_basis(_dptr(psi.view(np.float64)), n, 0)
    return psi


def apply_gate(psi: np.ndarray, n: int, target: int, controls: Sequence[int],
               values: Sequence[int], U: np.ndarray) -> np.ndarray:
    """In place: the pair-update equation on every pair whose controls hold."""
    assert psi.dtype == np.complex128 and psi.size == (1 << n)
    cm, cv = masks(controls, values)
    u = _u8(U)
    lib().or_apply_gate(_dptr(psi.view(np.float64)), n, int(target), cm, cv, _dptr(u))
    return psi


def gate_amplitudes(psi: np.ndarray, n: int, target: int, controls, values, U,
                    idx: Iterable[int]) -> np.ndarray:
    """Output amplitudes at the given indices of one gate applied to psi,
    each computed on its own from the input (psi is not modified)."""
    cm, cv = masks(controls, values)
    u = _u8(U)
    idx = np.asarray(list(idx) if not isinstance(idx, np.ndarray) else idx, dtype=np.uint64)
    out = np.empty(idx.size, dtype=np.complex128)
    o2 = np.empty(2, dtype=np.float64)
    L = lib()
    p = _dptr(psi.view(np.float64))
    for j, k in enumerate(idx):
        L.or_gate_amplitude(p, n, int(target), cm, cv, _dptr(u), int(k), _dptr(o2))
        out[j] = o2[0] + 1j * o2[1]
    return out


def pair_list(n: int, target: int, controls: Sequence[int], values: Sequence[int] = ()) -> np.ndarray:
    """Ascending first elements of every pair the gate updates (brute force)."""
    cm, cv = masks(controls, values)
    out = np.empty(max(1, 1 << (n - 1)), dtype=np.uint64)
    m = lib().or_pair_list(n, int(target), cm, cv, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return out[:m].copy()


def run_circuit(circ, params: Optional[np.ndarray] = None, psi0: Optional[np.ndarray] = None) -> np.ndarray:
    """Apply every gate of the circuit in order (one full pass per gate,
    Sec. III-A: gates are applied serially)."""
    n = circ.n
    if params is None:
        params = circ.params
    psi = zero_state(n) if psi0 is None else np.array(psi0, dtype=np.complex128, copy=True)
    for g in circ.gates:
        U = gate_matrix(g.kind, gate_angle(g, params), g.matrix)
        apply_gate(psi, n, g.target, g.controls, g.values, U)
    return psi


# --------------------------------------------------------------------------
# block-scaled 16-bit fixed-point states (format and arithmetic: the comment
# above or_q16_scale in sv_oracle.c; the paper names fixed-point precision
# as future work in Sec. V)
# --------------------------------------------------------------------------

Q16_BLOCK = 64


def q16_blocks(n: int) -> int:
    """Number of scale blocks of an n-qubit fixed-point state."""
    return max(1, (1 << n) // Q16_BLOCK)


def q16_nbytes(n: int) -> int:
    """Bytes of an n-qubit fixed-point state: 4 per amplitude, 1 per block."""
    return (4 << n) + q16_blocks(n)


def q16_views(buf: np.ndarray, n: int):
    """(codes int16 [2^n, 2], scales int8 [blocks]) views of a state buffer."""
    assert buf.dtype == np.uint8 and buf.size == q16_nbytes(n)
    N = 1 << n
    return buf[:4 * N].view(np.int16).reshape(N, 2), buf[4 * N:].view(np.int8)


def _i16p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int16))


def _i8p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))


def q16_scale(m: float) -> int:
    """Scale exponent of a block whose largest |component| is m (a float)."""
    return int(lib().or_q16_scale(float(m)))


def q16_code(v: float, s: int) -> int:
    """Code of the float v under scale exponent s."""
    return int(lib().or_q16_code(float(v), int(s)))


def q16_encode(psi: np.ndarray, n: int) -> np.ndarray:
    """Fixed-point state buffer (uint8) of a complex128 state."""
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    assert psi.size == (1 << n)
    buf = np.zeros(q16_nbytes(n), dtype=np.uint8)
    codes, scales = q16_views(buf, n)
    lib().or_q16_encode(_dptr(psi.view(np.float64)), n, _i16p(codes), _i8p(scales))
    return buf


def q16_decode(buf: np.ndarray, n: int) -> np.ndarray:
    """complex128 values of a fixed-point state buffer (exact)."""
    codes, scales = q16_views(buf, n)
    psi = np.empty(1 << n, dtype=np.complex128)
    lib().or_q16_decode(_i16p(codes), _i8p(scales), n, _dptr(psi.view(np.float64)))
    return psi


def q16_apply_gate(buf: np.ndarray, n: int, target: int, controls: Sequence[int],
                   values: Sequence[int], U: np.ndarray) -> np.ndarray:
    """In place on a fixed-point state buffer: decode, pair update in float
    on every pair whose controls hold, re-encode the blocks it touched."""
    codes, scales = q16_views(buf, n)
    cm, cv = masks(controls, values)
    u = _u8(U)
    lib().or_q16_apply_gate(_i16p(codes), _i8p(scales), n, int(target), cm, cv, _dptr(u))
    return buf


def q16_run_circuit(circ, params: Optional[np.ndarray] = None, buf0: Optional[np.ndarray] = None) -> np.ndarray:
    """Every gate of the circuit in order on a fixed-point state (from |0>
    encoded, or a copy of buf0)."""
    n = circ.n
    if params is None:
        params = circ.params
    buf = q16_encode(zero_state(n), n) if buf0 is None else np.array(buf0, dtype=np.uint8, copy=True)
    for g in circ.gates:
        U = gate_matrix(g.kind, gate_angle(g, params), g.matrix)
        q16_apply_gate(buf, n, g.target, g.controls, g.values, U)
    return buf


# 32-bit codes (same blocks and scale rule, computed in double; see the
# comment above or_q32_scale in sv_oracle.c)

def q32_nbytes(n: int) -> int:
    """Bytes of an n-qubit 32-bit fixed-point state: 8 per amplitude, 1 per block."""
    return (8 << n) + q16_blocks(n)


def q32_views(buf: np.ndarray, n: int):
    """(codes int32 [2^n, 2], scales int8 [blocks]) views of a state buffer."""
    assert buf.dtype == np.uint8 and buf.size == q32_nbytes(n)
    N = 1 << n
    return buf[:8 * N].view(np.int32).reshape(N, 2), buf[8 * N:].view(np.int8)


def _i32p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def q32_scale(m: float) -> int:
    return int(lib().or_q32_scale(float(m)))


def q32_code(v: float, s: int) -> int:
    return int(lib().or_q32_code(float(v), int(s)))


def q32_encode(psi: np.ndarray, n: int) -> np.ndarray:
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    assert psi.size == (1 << n)
    buf = np.zeros(q32_nbytes(n), dtype=np.uint8)
    codes, scales = q32_views(buf, n)
    lib().or_q32_encode(_dptr(psi.view(np.float64)), n, _i32p(codes), _i8p(scales))
    return buf


def q32_decode(buf: np.ndarray, n: int) -> np.ndarray:
    codes, scales = q32_views(buf, n)
    psi = np.empty(1 << n, dtype=np.complex128)
    lib().or_q32_decode(_i32p(codes), _i8p(scales), n, _dptr(psi.view(np.float64)))
    return psi


def q32_apply_gate(buf: np.ndarray, n: int, target: int, controls: Sequence[int],
                   values: Sequence[int], U: np.ndarray) -> np.ndarray:
    codes, scales = q32_views(buf, n)
    cm, cv = masks(controls, values)
    u = _u8(U)
    lib().or_q32_apply_gate(_i32p(codes), _i8p(scales), n, int(target), cm, cv, _dptr(u))
    return buf


def q32_run_circuit(circ, params: Optional[np.ndarray] = None, buf0: Optional[np.ndarray] = None) -> np.ndarray:
    n = circ.n
    if params is None:
        params = circ.params
    buf = q32_encode(zero_state(n), n) if buf0 is None else np.array(buf0, dtype=np.uint8, copy=True)
    for g in circ.gates:
        U = gate_matrix(g.kind, gate_angle(g, params), g.matrix)
        q32_apply_gate(buf, n, g.target, g.controls, g.values, U)
    return buf


def apply_block_low(psi: np.ndarray, n: int, k: int, M: np.ndarray) -> np.ndarray:
    """In place: every row of 2^k consecutive amplitudes becomes M . row (a
    k-qubit operator on the k lowest qubits; k <= 6)."""
    assert k <= 6 and psi.size == (1 << n)
    m = np.ascontiguousarray(np.asarray(M, dtype=np.complex128).reshape(1 << k, 1 << k))
    buf = np.ascontiguousarray(np.stack([m.real, m.imag], axis=-1).reshape(-1))
    lib().or_apply_block_low(_dptr(psi.view(np.float64)), n, k, _dptr(buf))
    return psi


def swap_qubits(psi: np.ndarray, n: int, pairs) -> np.ndarray:
    """In place: exchange the qubits of every pair (a, b), one pair after
    the other (a relabelling of index bits; no arithmetic)."""
    assert psi.size == (1 << n)
    for a, b in pairs:
        lib().or_swap_qubits(_dptr(psi.view(np.float64)), n, int(a), int(b))
    return psi


def norm2(psi: np.ndarray, n: int) -> float:
    return float(lib().or_norm2(_dptr(psi.view(np.float64)), n))


def expect_pauli(psi: np.ndarray, n: int, x: int, z: int) -> complex:
    o = np.empty(2, dtype=np.float64)
    lib().or_expect_pauli(_dptr(psi.view(np.float64)), n, int(x), int(z), _dptr(o))
    return complex(o[0], o[1])


def expect(psi: np.ndarray, n: int, terms) -> float:
    """<psi|H|psi> for H = sum_j coef_j P_j, summed term by term in order."""
    s = 0.0
    for t in terms:
        s += t.coef * expect_pauli(psi, n, t.x_mask, t.z_mask).real
    return s


def apply_hamiltonian(psi: np.ndarray, n: int, terms) -> np.ndarray:
    """H psi, by definition: sum over terms of coef * P psi."""
    out = np.zeros_like(psi)
    for t in terms:
        lib().or_add_pauli(_dptr(psi.view(np.float64)), _dptr(out.view(np.float64)), n,
                           int(t.x_mask), int(t.z_mask), float(t.coef))
    return out


def loss(circ, params: np.ndarray, terms) -> float:
    return expect(run_circuit(circ, params), circ.n, terms)


# --------------------------------------------------------------------------
# reference gradients (the adjoint method is what the GPU implements; the
# oracle differentiates by parameter shift and by finite differences)
# --------------------------------------------------------------------------

def _with_gates(circ, gates):
    from workloads import Circuit  # input containers only
    return Circuit(circ.n, gates, circ.params, dict(circ.meta))


# Conjugating a rotation by this Pauli flips the sign of its angle:
# F R(phi) F = R(-phi) because F anticommutes with the rotation's own Pauli.
_SHIFT_FLIP = {"RX": "Z", "RY": "X", "RZ": "X"}


def grad_param_shift(circ, params: np.ndarray, terms, which: Optional[Iterable[int]] = None) -> np.ndarray:
    """dL/dtheta_j by the parameter-shift rule.

    The two-term rule dL/dtheta = [L(theta + pi/2) - L(theta - pi/2)] / 2 is
    exact for a gate exp(-i theta G) whose generator G has exactly two
    eigenvalues differing by 1 (a constant added to G is a global phase,
    which cancels in L).  It is applied to the gate as it stands for
    * an uncontrolled RX/RY/RZ (G = P/2) or its adjoint (G = -P/2);
    * P(theta), with or without controls, and its adjoint: with controls the
      gate is exp(i theta Pi), Pi the projector onto the amplitudes whose
      controls hold and whose target bit is 1, and Pi has eigenvalues 0, 1.
    A controlled rotation has generator eigenvalues -1/2, 0, +1/2, so it is
    rewritten first as C-R(phi) = R(phi/2) . C^kF . R(-phi/2) . C^kF on the
    same target with the same controls (Barenco et al., Phys. Rev. A 52,
    3457 (1995)), F = X for RY and RZ and F = Z for RX, valid because
    F R(psi) F = R(-psi).  Each half-angle rotation is uncontrolled; with
    alpha = beta = phi/2 in R(alpha) . C^kF . R(-beta) . C^kF the chain rule
    gives dL/dphi = (dL/dalpha + dL/dbeta) / 2, and the shift rule holds for
    beta as well because R(-beta) = exp(+i beta P/2).  An adjoint-flagged
    controlled rotation is C-R(-theta): its derivative is minus the one at
    phi = -theta.  A parameter used by several gates sums the contributions
    of each use (product rule)."""
    from workloads import Gate
    params = np.asarray(params, dtype=np.float64)
    idx = list(range(len(params))) if which is None else list(which)
    out = np.zeros(len(idx))
    for oi, j in enumerate(idx):
        total = 0.0
        for gi, g in enumerate(circ.gates):
            if g.param != j:
                continue
            th = float(params[j])
            base = list(circ.gates)
            adj = g.kind.startswith("~")
            kind = g.kind[1:] if adj else g.kind
            if not g.controls or kind == "P":
                for sgn in (+1.0, -1.0):
                    gs = list(base)
                    gs[gi] = Gate(g.kind, g.target, g.controls, g.values, th + sgn * np.pi / 2.0)
                    total += 0.5 * sgn * loss(_with_gates(circ, gs), params, terms)
                continue
            if kind not in _SHIFT_FLIP:
                raise ValueError("controlled %s has no shift decomposition here" % g.kind)
            phi, dsign = (-th, -1.0) if adj else (th, 1.0)
            flip = Gate(_SHIFT_FLIP[kind], g.target, g.controls, g.values)
            for which_half in (0, 1):
                for sgn in (+1.0, -1.0):
                    alpha = phi / 2.0 + (sgn * np.pi / 2.0 if which_half == 0 else 0.0)
                    beta = phi / 2.0 + (sgn * np.pi / 2.0 if which_half == 1 else 0.0)
                    # circuit order (first applied first): C^kF, R(-beta), C^kF, R(alpha)
                    rep = [flip, Gate(kind, g.target, (), (), -beta), flip, Gate(kind, g.target, (), (), alpha)]
                    gs = base[:gi] + rep + base[gi + 1:]
                    total += dsign * 0.5 * 0.5 * sgn * loss(_with_gates(circ, gs), params, terms)
        out[oi] = total
    return out


def grad_finite_diff(circ, params: np.ndarray, terms, which: Optional[Iterable[int]] = None,
                     h: float = 1e-5) -> np.ndarray:
    """Central differences [L(theta_j + h) - L(theta_j - h)] / (2h)."""
    params = np.asarray(params, dtype=np.float64)
    idx = list(range(len(params))) if which is None else list(which)
    out = np.zeros(len(idx))
    for oi, j in enumerate(idx):
        pp = params.copy(); pp[j] += h
        pm = params.copy(); pm[j] -= h
        out[oi] = (loss(circ, pp, terms) - loss(circ, pm, terms)) / (2.0 * h)
    return out
