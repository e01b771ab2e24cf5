"""Binding of the observable and gradient entry points (sv_expect,
sv_expect_noalloc, sv_expect_terms, sv_apply_pauli_sum, sv_adjoint_grad, and
the planned adjoint sv_adjoint_create / sv_adjoint_run / sv_adjoint_destroy) and the
torch.autograd.Function built on them.  Argument marshalling only."""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

from . import (_L, _check, _sig, _sp, _vp, circuit_gates, state_view, stream_ptr, sv_gate_t, Circuit, SV_C128,
               SV_C64, SV_FUSE, sv_init)


class sv_pauli_t(ctypes.Structure):
    _fields_ = [("coef", ctypes.c_double), ("x_mask", ctypes.c_uint64), ("z_mask", ctypes.c_uint64)]


_sig("sv_expect", [_sp, ctypes.POINTER(sv_pauli_t), ctypes.c_int, _vp, _vp])
_sig("sv_expect_terms", [_sp, ctypes.POINTER(sv_pauli_t), ctypes.c_int, _vp, _vp])
_sig("sv_expect_noalloc", [_sp, ctypes.POINTER(sv_pauli_t), ctypes.c_int, _vp, _vp])
_sig("sv_apply_pauli_sum", [_sp, _sp, ctypes.POINTER(sv_pauli_t), ctypes.c_int, _vp])
_sig("sv_adjoint_grad", [_sp, _sp, ctypes.POINTER(sv_gate_t), ctypes.c_int, _vp, ctypes.c_int,
                         ctypes.POINTER(sv_pauli_t), ctypes.c_int, _vp, _vp, _vp, _vp])


def pauli_terms(terms) -> ctypes.Array:
    """ctypes array of sv_pauli_t from objects with coef/x_mask/z_mask (or
    (coef, x, z) tuples)."""
    if isinstance(terms, ctypes.Array):
        return terms
    arr = (sv_pauli_t * max(1, len(terms)))()
    for i, t in enumerate(terms):
        c, x, z = (t.coef, t.x_mask, t.z_mask) if hasattr(t, "coef") else t
        arr[i].coef, arr[i].x_mask, arr[i].z_mask = float(c), int(x), int(z)
    arr._sv_count = len(terms)
    return arr


def _count(arr):
    return getattr(arr, "_sv_count", len(arr))


def _ptr(t):
    return ctypes.c_void_p(0) if t is None else ctypes.c_void_p(t.data_ptr())


def sv_expect(state, terms, out=None, stream=None):
    """Device float64 tensor of shape (1,) holding <psi|H|psi>."""
    import torch
    s = state_view(state)
    arr = pauli_terms(terms)
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=state.device)
    _check(_L.sv_expect(ctypes.byref(s), arr, _count(arr), _ptr(out), stream_ptr(stream)))
    return out


def sv_expect_noalloc(state, terms, out, stream=None):
    """<psi|H|psi> into the caller's device float64 tensor out (shape >= 1),
    through the entry point that allocates nothing (at most 64 terms)."""
    s = state_view(state)
    arr = pauli_terms(terms)
    _check(_L.sv_expect_noalloc(ctypes.byref(s), arr, _count(arr), _ptr(out), stream_ptr(stream)))
    return out


def sv_expect_terms(state, terms, out=None, stream=None):
    import torch
    s = state_view(state)
    arr = pauli_terms(terms)
    if out is None:
        out = torch.empty(_count(arr), dtype=torch.float64, device=state.device)
    _check(_L.sv_expect_terms(ctypes.byref(s), arr, _count(arr), _ptr(out), stream_ptr(stream)))
    return out


def sv_apply_pauli_sum(state_in, state_out, terms, stream=None) -> None:
    a, b = state_view(state_in), state_view(state_out)
    arr = pauli_terms(terms)
    _check(_L.sv_apply_pauli_sum(ctypes.byref(a), ctypes.byref(b), arr, _count(arr), stream_ptr(stream)))


def sv_adjoint_grad(psi, lam, gates, params, terms, grad=None, loss=None, scale=None, stream=None):
    """Adjoint gradient; psi (final forward state) is consumed.  Returns
    (grad, loss) device tensors."""
    import torch
    s, l = state_view(psi), state_view(lam)
    garr = gates if isinstance(gates, ctypes.Array) else circuit_gates(gates)
    parr = pauli_terms(terms)
    nparams = 0 if params is None else int(params.numel())
    if grad is None:
        grad = torch.empty(max(1, nparams), dtype=torch.float64, device=psi.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float64, device=psi.device)
    _check(_L.sv_adjoint_grad(ctypes.byref(s), ctypes.byref(l), garr, _count(garr), _ptr(params), nparams, parr,
                              _count(parr), _ptr(grad), _ptr(loss), _ptr(scale), stream_ptr(stream)))
    return grad[:nparams], loss


_sig("sv_adjoint_create", [ctypes.c_int, ctypes.c_int, ctypes.POINTER(sv_gate_t), ctypes.c_int, ctypes.c_int,
                           ctypes.POINTER(sv_pauli_t), ctypes.c_int, ctypes.POINTER(_vp)])
_sig("sv_adjoint_run", [_vp, _sp, _sp, _vp, _vp, _vp, _vp, _vp])
_sig("sv_adjoint_destroy", [_vp])


class AdjointPlan:
    """A planned adjoint gradient (sv_adjoint_create) of one circuit and
    Hamiltonian; run() enqueues sv_adjoint_run (psi is consumed)."""

    def __init__(self, n: int, gates, terms, nparams: int, dtype: int = SV_C128):
        self.n, self.dtype, self.nparams = n, dtype, int(nparams)
        self._g = gates if isinstance(gates, ctypes.Array) else circuit_gates(gates)
        self._t = pauli_terms(terms)
        h = _vp()
        _check(_L.sv_adjoint_create(int(n), int(dtype), self._g, _count(self._g), self.nparams, self._t,
                                    _count(self._t), ctypes.byref(h)))
        self._h = h

    def run(self, psi, lam, params, grad=None, loss=None, scale=None, stream=None):
        """Returns (grad, loss) device tensors."""
        import torch
        s, l = state_view(psi), state_view(lam)
        if grad is None:
            grad = torch.empty(max(1, self.nparams), dtype=torch.float64, device=psi.device)
        if loss is None:
            loss = torch.empty(1, dtype=torch.float64, device=psi.device)
        _check(_L.sv_adjoint_run(self._h, ctypes.byref(s), ctypes.byref(l), _ptr(params), _ptr(grad), _ptr(loss),
                                 _ptr(scale), stream_ptr(stream)))
        return grad[:self.nparams], loss

    def close(self) -> None:
        if getattr(self, "_h", None):
            _L.sv_adjoint_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SvExpectation:
    """L(theta) = <0|U(theta)^dag H U(theta)|0> as a torch.autograd.Function.

    forward: sv_init + circuit run (fused plan, angles read from the params
    tensor on the device) + sv_expect.  backward: copy of the saved final
    state (so backward can run more than once), the model's planned adjoint
    (sv_adjoint_run) with the upstream gradient passed as the device scale.  At most three state
    vectors are alive: the saved forward state, its copy being un-applied and
    the co-state."""

    _fn = None

    @classmethod
    def function(cls):
        if cls._fn is None:
            import torch

            class _Fn(torch.autograd.Function):
                @staticmethod
                def forward(ctx, params, model):
                    params = params.detach().to(torch.float64).contiguous()
                    state = torch.empty(1 << model.n, dtype=model.torch_dtype, device=params.device)
                    sv_init(state, 0)
                    model.plan.run(state, params)
                    loss = sv_expect(state, model.terms)
                    ctx.model = model
                    ctx.state = state
                    ctx.save_for_backward(params)
                    return loss.reshape(())

                @staticmethod
                def backward(ctx, grad_out):
                    (params,) = ctx.saved_tensors
                    model = ctx.model
                    work = ctx.state.clone()
                    lam = torch.empty_like(work)
                    scale = grad_out.detach().to(torch.float64).reshape(1).contiguous()
                    grad, _ = model.adjoint.run(work, lam, params, scale=scale)
                    return grad, None

            cls._fn = _Fn
        return cls._fn

    @classmethod
    def apply(cls, params, model):
        return cls.function().apply(params, model)


class ExpectationModel:
    """A parameterised circuit and a Hamiltonian, ready for SvExpectation."""

    def __init__(self, circuit, terms, dtype: int = SV_C128, flags: int = SV_FUSE):
        import torch
        self.n = circuit.n
        self.gates = circuit_gates(circuit)
        self.terms = pauli_terms(terms)
        self.nparams = circuit.nparams
        self.dtype = dtype
        self.torch_dtype = torch.complex128 if dtype == SV_C128 else torch.complex64
        self.plan = Circuit(self.n, self.gates, dtype=dtype, nparams=self.nparams, flags=flags)
        self.adjoint = AdjointPlan(self.n, self.gates, self.terms, self.nparams, dtype=dtype)

    def __call__(self, params):
        return SvExpectation.apply(params, self)
