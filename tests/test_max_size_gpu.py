"""The largest register each dtype supports on one MI355X (288 GB of HBM):
n = 34 complex128 and n = 35 complex64 (256 GiB each), n = 36 16-bit and
n = 35 32-bit fixed point (257 GiB and 256.5 GiB).  64-bit indices throughout.  The checks are properties that pin
the result without a second full-size buffer: a basis state moved by a
controlled X, a gate whose controls fail on it leaving it alone, Pauli
expectations with closed forms (of the basis state, and for complex states
of the state after a Hadamard on the top qubit), and the norm (or, for fixed point, whole-array reductions of codes and scales)
showing that every other amplitude stayed zero.
"""
import numpy as np
import pytest
import torch

import workloads as W

sv = pytest.importorskip("paper_2411_18354_amd")

pytestmark = pytest.mark.gpu

X = np.array([[0, 1], [1, 0]])
H = np.array([[1, 1], [1, -1]]) / np.sqrt(2.0)


def _alloc(fn, what):
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    try:
        return fn()
    except torch.cuda.OutOfMemoryError as e:
        pytest.skip("could not allocate %s: %s" % (what, str(e).splitlines()[0]))


def _run_and_release(make, body, what):
    """Allocate with make(), run body(buffer), and free the buffer before
    reporting a failure: a traceback would otherwise keep frames (and the
    256 GiB buffer they reference) alive for the tests that follow."""
    buf = _alloc(make, what)
    err = None
    try:
        body(buf)
    except Exception as e:  # noqa: BLE001 - reported below without its frames
        err = "%s: %s" % (type(e).__name__, e)
    finally:
        del buf
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    if err:
        pytest.fail(err, pytrace=False)


def _isum(t, chunk=1 << 28):
    """Integer sum of a huge tensor in int64, chunk by chunk (a sum with
    dtype=int64 would first cast the whole tensor)."""
    return sum(int(c.sum(dtype=torch.int64).item()) for c in t.split(chunk))


def _basis(n):
    # bits 0 and 2, bit 31 (beyond 31-bit lane arithmetic) and bit n-2
    return (1 << (n - 2)) | (1 << 31) | 5


@pytest.mark.parametrize("dtype,n", [("c128", 34), ("c64", 35)])
def test_controlled_x_at_max_size(dtype, n):
    td = torch.complex128 if dtype == "c128" else torch.complex64
    print("max size: %s n=%d" % (dtype, n), flush=True)

    def body(psi):
        b = _basis(n)
        t = n - 1
        sv.sv_init(psi, b)
        sv.sv_apply_gate(psi, t, (0, n - 2), None, X)            # scheduled: controls hold on b
        sv.sv_apply_gate(psi, 3, (1,), None, X)                  # control on qubit 1 fails on b
        sv.sv_apply_gate(psi, t - 1, (2,), 0, X, mode="masked")  # negative control fails on b
        sv.sv_apply_gate(psi, 0, (), None, np.eye(2))            # every amplitude rewritten
        w = b | (1 << t)
        torch.cuda.synchronize()
        assert psi[w].item() == 1 and psi[b].item() == 0
        # <psi|I|psi> = 1 with |psi_w| = 1 forces every other amplitude to 0
        nrm = sv.sv_expect(psi, [(1.0, 0, 0)]).item()
        assert abs(nrm - 1.0) < 1e-12
        # H on the top qubit (set in w): (|w - 2^t> - |w>) / sqrt(2), whose
        # Pauli expectations are closed forms of w's bits; X and Y on qubit t
        # run a tile pass whose tile holds qubit t, Z on qubit 31 a sign from
        # outside the tile
        sv.sv_apply_gate(psi, t, (), None, H)
        terms = [(1.0, 0, 1 << t), (1.0, 1 << t, 0), (1.0, 1 << t, 1 << t), (1.0, 0, 1),
                 (1.0, 1 << t, 1 << 31), (1.0, 0, (1 << 31) | (1 << (n - 2)))]
        want = [0.0, -1.0, 0.0, -1.0 if w & 1 else 1.0, 1.0 if (w >> 31) & 1 else -1.0,
                1.0 if ((w >> 31) ^ (w >> (n - 2))) & 1 == 0 else -1.0]
        got = sv.sv_expect_terms(psi, terms).cpu().numpy()
        tol = 1e-12 if dtype == "c128" else 1e-6
        assert np.max(np.abs(got - np.array(want))) <= tol, (got, want)
        sv.sv_apply_gate(psi, t, (), None, H)
        torch.cuda.synchronize()
        assert abs(psi[w].item() - 1) <= tol and abs(psi[b].item()) <= tol
        psi[w], psi[b] = 1, 0  # H H = I up to rounding; the checks below are exact
        # the masked kernel undoes the move
        sv.sv_apply_gate(psi, t, (0, n - 2), None, X, mode="masked")
        torch.cuda.synchronize()
        assert psi[b].item() == 1 and psi[w].item() == 0

    _run_and_release(lambda: torch.empty(1 << n, dtype=td, device="cuda"), body, "%s n=%d" % (dtype, n))


@pytest.mark.parametrize("bits,n", [(16, 36), (32, 35)])
def test_fixed_point_controlled_x_at_max_size(bits, n):
    dtype = sv.SV_CQ16 if bits == 16 else sv.SV_CQ32
    one, one_scale, zero_scale = (16384, -14, -126) if bits == 16 else (1 << 30, -30, -128)
    print("max size: %d-bit fixed point n=%d" % (bits, n), flush=True)

    def body(q):
        N = 1 << n
        nb = N >> 6
        cb = N * (4 if bits == 16 else 8)
        # 16-bit: one int32 word per amplitude (re code low); 32-bit: two
        # int32 words per amplitude (re, im)
        codes = q.data[:cb].view(torch.int32)
        scales = q.data[cb:].view(torch.int8)
        word = (lambda k: k) if bits == 16 else (lambda k: 2 * k)
        b = _basis(n)
        t = n - 1
        sv.sv_init(q, b)
        sv.sv_apply_gate(q, t, (0, n - 2), None, X)
        sv.sv_apply_gate(q, 3, (1,), None, X)
        w = b | (1 << t)
        torch.cuda.synchronize()
        # 1.0 is the code 2^14 (2^30) under scale -14 (-30); every other code
        # is 0 and every other block keeps the zero-block scale
        assert codes[word(w)].item() == one and codes[word(b)].item() == 0
        assert codes.min().item() == 0 and codes.max().item() == one
        assert _isum(codes) == one
        assert scales[w >> 6].item() == one_scale
        assert scales.max().item() == one_scale and scales.min().item() == zero_scale
        assert _isum(scales) == zero_scale * (nb - 1) + one_scale
        # expectations read from the codes: the basis state w decodes to
        # exactly 1 at w, so Z terms give the sign of w's bits, X terms 0
        terms = [(1.0, 0, 0), (1.0, 0, 1 << t), (1.0, 0, (1 << 31) | 1), (1.0, 1 << t, 0), (-0.5, 1 << t, 1 << t)]
        want = [1.0, -1.0 if (w >> t) & 1 else 1.0, 1.0 if (((w >> 31) ^ w) & 1) == 0 else -1.0, 0.0, 0.0]
        got = sv.sv_expect_terms(q, terms).cpu().numpy()
        assert np.array_equal(got, np.array(want)), (got, want)
        sv.sv_apply_gate(q, t, (0, n - 2), None, X, mode="masked")
        torch.cuda.synchronize()
        assert codes[word(b)].item() == one and codes[word(w)].item() == 0
        assert scales[b >> 6].item() == one_scale and scales[w >> 6].item() == zero_scale

    _run_and_release(lambda: sv.FixedState(n, dtype), body, "%d-bit fixed point n=%d" % (bits, n))


def test_tile_launches_split_into_pieces():
    """Tile and exchange kernels launched over more than 2^22 tiles (n = 30
    complex128 with 2^7-amplitude tiles: 2^23 tiles, two pieces) give the
    same state as the unfused kernels and as an axis transpose."""
    n = 30
    print("split tile launches: n=%d, tile width 2^7" % n, flush=True)
    saved = sv.sv_tune_get("tile_log2_c128")
    sv.sv_tune_set("tile_log2_c128", 7)
    try:
        def body(buf):
            psi, ref, pre = buf
            gen = torch.Generator(device="cuda").manual_seed(36)
            psi.view(torch.float64).copy_(torch.randn(2 << n, dtype=torch.float64, device="cuda", generator=gen))
            ref.copy_(psi)
            # gates on the 7 lowest qubits (runs of tiles) and controls above
            circ = W.Circuit(n, [W.Gate("H", q) for q in range(7)]
                             + [W.Gate("U", 3, (29,), (), matrix=W.haar_unitary_2x2(37)),
                                W.Gate("X", 5, (0, 20)), W.Gate("U", 6, (2,), (0,), matrix=W.haar_unitary_2x2(38))])
            plan = sv.Circuit(n, circ, flags=sv.SV_FUSE)
            assert plan.info()["fused_runs"] >= 1
            plan.run(psi)
            sv.sv_apply_circuit(ref, circ, flags=0)
            torch.cuda.synchronize()
            assert (psi - ref).abs().max().item() <= 1e-12 * ref.abs().max().item()
            plan.close()
            # exchange of qubits 0 and 29 = transpose of those index bits; twice = identity
            pre.copy_(psi)
            ref.copy_(psi.view(2, 1 << 28, 2).transpose(0, 2).contiguous().view(-1))
            sv.sv_swap_qubits(psi, [(0, 29)])
            torch.cuda.synchronize()
            assert torch.equal(psi, ref)
            sv.sv_swap_qubits(psi, [(0, 29)])
            torch.cuda.synchronize()
            assert torch.equal(psi, pre)

        _run_and_release(lambda: [torch.empty(1 << n, dtype=torch.complex128, device="cuda") for _ in range(3)],
                         body, "three n=30 complex128 states")
    finally:
        sv.sv_tune_set("tile_log2_c128", saved)
