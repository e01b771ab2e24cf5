"""The paper's 29-qubit evaluation circuits at full size, checked on every
amplitude against their closed forms (the oracle cannot hold 2^29
amplitudes at the speed a test needs; the closed forms are exact).

* QFT29, the Sec. IV-A figure as drawn (H, then R_m = P(2 pi / 2^m) on j
  controlled by j+m-1; no swaps): the circuit is F . P_rev with
  F_{yx} = e^{+2 pi i xy / N} / sqrt(N) and P_rev the bit reversal of the
  input index, so a basis input |x> gives amplitude
  e^{2 pi i y rev(x) / N} / sqrt(N) at every y, and a general input psi gives
  ifft(psi[rev]) sqrt(N).
* Stream29, the Sec. IV-C figure (gate j: X on qubit j controlled by qubits
  0..j-1, in drawn order): |x> -> |x - 1 mod N>.  X gates only move
  amplitudes, so the result is the input rolled by one, bit for bit.

Each runs unfused (one scheduled kernel per gate), fused (LDS tiles) and on
the masked baseline, in complex128 (1e-12) and complex64 (1e-5 against the
double-precision closed form), relative to the largest amplitude."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

N29 = 29


def _say(*a):
    print(*a, flush=True)


def _rev_bits(idx, n):
    """Bit reversal of an int64 index tensor (n bits)."""
    r = idx.new_zeros(idx.shape)
    for b in range(n):
        r |= ((idx >> b) & 1) << (n - 1 - b)
    return r


def _flags(sv):
    return (("unfused", 0), ("fused", sv.SV_FUSE), ("masked", sv.SV_MASKED))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_qft29_basis_inputs_closed_form(gpu, dtype):
    import torch
    sv = gpu
    n, N = N29, 1 << N29
    td = torch.complex128 if dtype == "c128" else torch.complex64
    tol = 1e-12 if dtype == "c128" else 1e-5
    circ = W.qft(n)
    st = torch.empty(N, dtype=td, device="cuda")
    y = torch.arange(N, dtype=torch.int64, device="cuda")
    for x0 in (0x0A5A5A5, 1, N - 3):
        r = int(_rev_bits(torch.tensor([x0]), n)[0])
        ph = ((y * r) & (N - 1)).double() * (2 * math.pi / N)  # y rev(x) mod N, exact in int64
        want = torch.polar(torch.full_like(ph, 1.0 / math.sqrt(N)), ph)
        del ph
        for label, fl in _flags(sv):
            _say("qft29 %s %s x0=%d" % (dtype, label, x0))
            sv.sv_init(st, x0)
            sv.sv_apply_circuit(st, circ, flags=fl)
            err = float((st.to(torch.complex128) - want).abs().max()) * math.sqrt(N)
            _say("  max error / max amplitude %.3e" % err)
            assert err <= tol, (label, x0, err)
        del want
        torch.cuda.empty_cache()


def test_qft29_random_input_closed_form_c128(gpu):
    """A random input state against ifft(psi[rev]) sqrt(N), computed with the
    GPU's FFT library (a library primitive standing for the definition)."""
    import torch
    sv = gpu
    n, N = N29, 1 << N29
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2929)
    psi = torch.randn(N, dtype=torch.complex128, device="cuda", generator=gen)
    psi /= psi.abs().pow(2).sum().sqrt()
    rev = _rev_bits(torch.arange(N, dtype=torch.int64, device="cuda"), n)
    want = torch.fft.ifft(psi[rev]) * math.sqrt(N)
    del rev
    torch.cuda.empty_cache()
    scale = float(want.abs().max())
    st = torch.empty_like(psi)
    for label, fl in _flags(sv)[:2]:
        st.copy_(psi)
        sv.sv_apply_circuit(st, W.qft(n), flags=fl)
        err = float((st - want).abs().max()) / scale
        _say("qft29 random input %s: max error / max amplitude %.3e" % (label, err))
        assert err <= 1e-12, (label, err)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_stream29_shifts_by_one(gpu, dtype):
    import torch
    sv = gpu
    n, N = N29, 1 << N29
    td = torch.complex128 if dtype == "c128" else torch.complex64
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2930)
    psi = torch.randn(N, dtype=td, device="cuda", generator=gen)
    want = torch.roll(psi, -1)  # out[y] = in[y + 1]: |x> -> |x - 1>
    st = torch.empty_like(psi)
    for label, fl in _flags(sv):
        _say("stream29 %s %s" % (dtype, label))
        st.copy_(psi)
        sv.sv_apply_circuit(st, W.stream(n), flags=fl)
        assert torch.equal(st, want), label
    # a basis state walks down by one
    sv.sv_init(st, 0)
    sv.sv_apply_circuit(st, W.stream(n), flags=sv.SV_FUSE)
    assert float(st[N - 1].abs()) == 1.0 and float(st.abs().pow(2).sum()) == 1.0


@pytest.mark.parametrize("bits", [16, 32])
def test_qft29_and_stream29_fixed_point_fused(gpu, bits):
    """Fused passes over block-scaled fixed-point states at n = 29.  QFT29 on
    a basis input against its closed form: every block is re-encoded once per
    pass, each component within half a code step, at most 2^-B of the
    block's largest component (B = 15 or 31), so each pass moves the unit
    state by at most sqrt(128) 2^-B in 2-norm; add the arithmetic rounding of
    each gate (float or double).  Stream29 on a basis input moves one
    amplitude of exactly 1.0: the result is the basis state below it,
    exactly."""
    import torch
    sv = gpu
    n, N = N29, 1 << N29
    dtype = sv.SV_CQ16 if bits == 16 else sv.SV_CQ32
    arith = 1e-6 if bits == 16 else 1e-14  # per gate, 2-norm
    st = sv.FixedState(n, dtype)
    out = torch.empty(N, dtype=torch.complex128, device="cuda")
    plan = sv.Circuit(n, W.qft(n), dtype=dtype, flags=sv.SV_FUSE)
    try:
        P = plan.info()["passes"]
        x0 = 0x0A5A5A5
        r = int(_rev_bits(torch.tensor([x0]), n)[0])
        y = torch.arange(N, dtype=torch.int64, device="cuda")
        ph = ((y * r) & (N - 1)).double() * (2 * math.pi / N)
        del y
        sv.sv_init(st, x0)
        plan.run(st)
        sv.sv_convert(out, st)
        err = float((out - torch.polar(torch.full_like(ph, 1.0 / math.sqrt(N)), ph)).abs().pow(2).sum().sqrt())
        del ph
        tol = (P + 1) * math.sqrt(128) * 2.0 ** -(bits - 1) + len(W.qft(n).gates) * arith
        _say("qft29 q%d fused: %d passes, error %.3e (2-norm; bound %.3e)" % (bits, P, err, tol))
        assert err <= tol
    finally:
        plan.close()
    sv.sv_init(st, 5)
    sv.sv_apply_circuit(st, W.stream(n), flags=sv.SV_FUSE)
    sv.sv_convert(out, st)
    torch.cuda.synchronize()
    assert float(out[4].real) == 1.0 and float(out.abs().pow(2).sum()) == 1.0
