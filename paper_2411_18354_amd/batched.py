"""Binding of the batched entry points (sv_apply_circuits_batched,
sv_adjoint_grad_batched, and the planned batch sv_batch_create / sv_batch_run /
sv_batch_adjoint / sv_batch_set_timing / sv_batch_info / sv_batch_destroy).
Argument marshalling only."""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

from . import _L, _check, _sig, _vp, circuit_gates, state_view, stream_ptr, sv_gate_t, sv_state_t
from .observables import pauli_terms, sv_pauli_t

_i64p = ctypes.POINTER(ctypes.c_int64)
_sig("sv_apply_circuits_batched", [ctypes.POINTER(sv_state_t), ctypes.c_int, ctypes.POINTER(sv_gate_t), _i64p, _vp,
                                   _i64p, ctypes.c_int64, _vp])
_sig("sv_adjoint_grad_batched", [ctypes.POINTER(sv_state_t), ctypes.POINTER(sv_state_t), ctypes.c_int,
                                 ctypes.POINTER(sv_gate_t), _i64p, _vp, _i64p, ctypes.c_int64,
                                 ctypes.POINTER(sv_pauli_t), _i64p, _vp, _vp, _vp])
_sig("sv_batch_set_timing", [_vp, _vp, ctypes.POINTER(ctypes.c_double)])
_sig("sv_batch_create", [ctypes.POINTER(sv_state_t), ctypes.POINTER(sv_state_t), ctypes.c_int,
                         ctypes.POINTER(sv_gate_t), _i64p, _i64p, ctypes.c_int64, ctypes.POINTER(sv_pauli_t), _i64p,
                         ctypes.POINTER(_vp)])
_sig("sv_batch_run", [_vp, _vp, _vp])
_sig("sv_batch_adjoint", [_vp, _vp, _vp, _vp, _vp])
_sig("sv_batch_destroy", [_vp])
_sig("sv_batch_info", [_vp, _i64p, ctypes.POINTER(ctypes.c_int32), ctypes.c_int64, ctypes.POINTER(ctypes.c_uint64)])


def _states(tensors):
    arr = (sv_state_t * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = state_view(t)
    return arr


def _offsets(counts):
    arr = (ctypes.c_int64 * (len(counts) + 1))()
    acc = 0
    for i, c in enumerate(counts):
        arr[i] = acc
        acc += int(c)
    arr[len(counts)] = acc
    return arr


def _concat_gates(circuits):
    gates = [g for c in circuits for g in c.gates]
    return circuit_gates(gates), _offsets([len(c.gates) for c in circuits])


def sv_apply_circuits_batched(states: Sequence, circuits: Sequence, params=None, param_counts=None,
                              stream=None) -> None:
    """Run circuits[c] on states[c] in one persistent launch.  params: device
    float64 tensor of all circuits' angles concatenated; param_counts: number
    of parameters of each circuit (defaults to circuit.nparams)."""
    st = _states(states)
    garr, goff = _concat_gates(circuits)
    if param_counts is None:
        param_counts = [getattr(c, "nparams", 0) or 0 for c in circuits]
    poff = _offsets(param_counts)
    p = ctypes.c_void_p(0 if params is None else params.data_ptr())
    total = 0 if params is None else int(params.numel())
    _check(_L.sv_apply_circuits_batched(st, len(states), garr, goff, p, poff, total, stream_ptr(stream)))


def sv_adjoint_grad_batched(psi_states: Sequence, lam_states: Sequence, circuits: Sequence, params, hamiltonians,
                            param_counts=None, grad=None, loss=None, stream=None):
    """Batched adjoint gradients; returns (grad, loss) device tensors."""
    import torch
    ps, ls = _states(psi_states), _states(lam_states)
    garr, goff = _concat_gates(circuits)
    if param_counts is None:
        param_counts = [c.nparams for c in circuits]
    poff = _offsets(param_counts)
    terms = [t for h in hamiltonians for t in h]
    tarr = pauli_terms(terms)
    toff = _offsets([len(h) for h in hamiltonians])
    dev = psi_states[0].device
    if grad is None:
        grad = torch.empty(max(1, int(params.numel())), dtype=torch.float64, device=dev)
    if loss is None:
        loss = torch.empty(len(circuits), dtype=torch.float64, device=dev)
    _check(_L.sv_adjoint_grad_batched(ps, ls, len(circuits), garr, goff, ctypes.c_void_p(params.data_ptr()), poff,
                                      int(params.numel()), tarr, toff, ctypes.c_void_p(grad.data_ptr()),
                                      ctypes.c_void_p(loss.data_ptr()), stream_ptr(stream)))
    return grad[:int(params.numel())], loss


class Batch:
    """A planned batch on the device (sv_batch_create).  states (and, for
    gradients, lam_states and hamiltonians) are bound at creation: run()
    applies the circuits to whatever those buffers hold, adjoint() computes
    the batched gradients from the final states they hold."""

    def __init__(self, states: Sequence, circuits: Sequence, param_counts=None, lam_states=None,
                 hamiltonians=None, nparams_total: Optional[int] = None):
        self._keep = (list(states), list(lam_states) if lam_states is not None else None)
        st = _states(states)
        ls = _states(lam_states) if lam_states is not None else None
        garr, goff = _concat_gates(circuits)
        if param_counts is None:
            param_counts = [getattr(c, "nparams", 0) or 0 for c in circuits]
        poff = _offsets(param_counts)
        self.nparams_total = int(poff[len(circuits)]) if nparams_total is None else int(nparams_total)
        self.ncirc = len(circuits)
        tarr = toff = None
        if lam_states is not None:
            tarr = pauli_terms([t for h in hamiltonians for t in h])
            toff = _offsets([len(h) for h in hamiltonians])
        self.device = states[0].device
        h = _vp()
        _check(_L.sv_batch_create(st, ls, len(circuits), garr, goff, poff, self.nparams_total, tarr, toff,
                                  ctypes.byref(h)))
        self._h = h

    def run(self, params=None, stream=None) -> None:
        p = ctypes.c_void_p(0 if params is None else params.data_ptr())
        _check(_L.sv_batch_run(self._h, p, stream_ptr(stream)))

    def adjoint(self, params, grad=None, loss=None, stream=None):
        """Returns (grad, loss) device float64 tensors."""
        import torch
        if grad is None:
            grad = torch.empty(max(1, self.nparams_total), dtype=torch.float64, device=self.device)
        if loss is None:
            loss = torch.empty(self.ncirc, dtype=torch.float64, device=self.device)
        _check(_L.sv_batch_adjoint(self._h, ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
                                   ctypes.c_void_p(loss.data_ptr()), stream_ptr(stream)))
        return grad[:self.nparams_total], loss

    def set_timing(self, stamps=None) -> float:
        """Start/end clock stamps of later runs into the device uint64 (or
        int64) tensor stamps: per work item of run() (the circuits items()
        lists), per circuit of adjoint(); 2 * max(ncirc, nitems) values; None
        turns them off.  Returns the clock period in nanoseconds."""
        ns = ctypes.c_double(0.0)
        p = ctypes.c_void_p(0 if stamps is None else stamps.data_ptr())
        _check(_L.sv_batch_set_timing(self._h, p, ctypes.byref(ns)))
        self._stamps = stamps
        return ns.value

    def items(self):
        """The forward run's work items in queue order, each a circuit index
        (a circuit split over workgroups appears once per workgroup that may
        join it)."""
        n = ctypes.c_int64(0)
        _check(_L.sv_batch_info(self._h, ctypes.byref(n), None, 0, None))
        arr = (ctypes.c_int32 * max(1, n.value))()
        _check(_L.sv_batch_info(self._h, None, arr, n.value, None))
        return [int(arr[i]) for i in range(n.value)]

    def wait_timeouts(self) -> int:
        """Chunk waits of split circuits that gave up, over all runs so far
        (waits for the last run)."""
        v = ctypes.c_uint64(0)
        _check(_L.sv_batch_info(self._h, None, None, 0, ctypes.byref(v)))
        return int(v.value)

    def close(self) -> None:
        if getattr(self, "_h", None):
            _L.sv_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
