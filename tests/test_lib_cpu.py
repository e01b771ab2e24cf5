"""Host-only checks of libsv.so: it loads, exports every function sv.h
declares, and rejects invalid arguments before touching a device."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sv.h")
LIB = os.path.join(ROOT, "paper_2411_18354_amd", "libsv.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sv_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared()
    for required in ("sv_alloc", "sv_free", "sv_init", "sv_apply_gate", "sv_debug_pair_indices",
                     "sv_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first"
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (sv_[a-z0-9_]+)", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    L = ctypes.CDLL(LIB)
    for n in _declared():
        assert hasattr(L, n)


@pytest.fixture(scope="module")
def sv():
    import paper_2411_18354_amd as sv
    return sv


def _state(sv, n=8, dtype=0, ptr=0x10000):
    return sv.sv_state_t(ptr, n, dtype)


def _rc(fn):
    try:
        fn()
    except Exception as e:  # SvError
        return getattr(e, "code", None), str(e)
    return 0, ""


U = [0, 0, 1, 0, 1, 0, 0, 0]


@pytest.mark.parametrize("case,needle", [
    (dict(target=8), "target"),
    (dict(target=-1), "target"),
    (dict(target=2, controls=(2,)), "equals the target"),
    (dict(target=2, controls=(3, 3)), "duplicate"),
    (dict(target=2, controls=(9,)), "outside"),
    (dict(target=2, controls=(3,), ctrl_vals=1 << 4), "outside the control mask"),
    (dict(target=2, mode=9), "mode"),
    (dict(target=7, mode="wave"), "SV_MODE_WAVE"),
    (dict(target=5, controls=(3, 4, 6, 7), n=8, mode="wave"), "SV_MODE_WAVE"),
    (dict(target=12, mode="tile", n=14), "SV_MODE_TILE"),
])
def test_gate_argument_errors(sv, case, needle):
    n = case.pop("n", 8)
    s = _state(sv, n)
    code, msg = _rc(lambda: sv.sv_apply_gate(s, U=U, **case))
    assert code == sv.SV_EINVAL and needle in msg, msg


def test_state_errors(sv):
    for st, needle in ((_state(sv, 0), "n=0"), (_state(sv, 35), "n=35"), (_state(sv, 8, 4), "dtype"),
                       (_state(sv, 8, 0, 0), "NULL"), (_state(sv, 8, 0, 0x10008), "aligned")):
        code, msg = _rc(lambda: sv.sv_apply_gate(st, 0, U=U))
        assert code == sv.SV_EINVAL and needle in msg, msg
    code, msg = _rc(lambda: sv.sv_init(_state(sv, 4), 16))
    assert code == sv.SV_EINVAL and "basis" in msg
    code, msg = _rc(lambda: sv.sv_alloc(40))
    assert code == sv.SV_EINVAL
    # c64 allows one more qubit than c128
    code, msg = _rc(lambda: sv.sv_apply_gate(_state(sv, 35, 1), 40, U=U))
    assert code == sv.SV_EINVAL and "target" in msg


def test_null_matrix_and_masks(sv):
    L = sv.lib()
    s = _state(sv)
    rc = L.sv_apply_gate(ctypes.byref(s), 0, None, 0, 0, None, 0, None)
    assert rc == sv.SV_EINVAL and "U is NULL" in sv.sv_last_error()
    rc = L.sv_apply_gate(ctypes.byref(s), 0, None, 2, 0, (ctypes.c_double * 8)(*U), 0, None)
    assert rc == sv.SV_EINVAL and "controls is NULL" in sv.sv_last_error()
    code, msg = _rc(lambda: sv.sv_apply_gate_masks(s, 1, 0b10, 0, U))
    assert code == sv.SV_EINVAL and "both target and control" in msg


def test_debug_indices_errors(sv):
    L = sv.lib()
    rc = L.sv_debug_pair_indices(8, 0, None, 0, 0, ctypes.c_void_p(0x1000), 10, None)
    assert rc == sv.SV_EINVAL and "out_len" in sv.sv_last_error()
    rc = L.sv_debug_pair_indices(8, 0, None, 0, 0, None, 1 << 10, None)
    assert rc == sv.SV_EINVAL


def test_tune_cache_load(sv, tmp_path, monkeypatch):
    """A cache record for the named architecture is applied; records for other
    architectures are ignored; malformed files are rejected."""
    keys = ("granule_bits_c128", "low_policy", "wave_auto", "tile_log2_c128", "tile_low_bits_c128")
    before = {k: sv.sv_tune_get(k) for k in keys}
    p = tmp_path / "tune.json"
    p.write_text('{"arch": "gfx000", "dtype": "c128", "granule_bits": 1, "low_policy": 0, "wave_auto": 0, '
                 '"tile_log2": 9, "tile_low_bits": 4}\n'
                 '{"arch": "gfx950:sramecc+:xnack-", "dtype": "c128", "granule_bits": 2, "low_policy": 0, '
                 '"wave_auto": 0, "tile_log2": 11, "tile_low_bits": 5}\n')
    monkeypatch.setenv("SV_TUNE_ARCH", "gfx950:sramecc+:xnack-")
    try:
        sv.sv_tune_load(str(p))
        assert sv.sv_tune_get("granule_bits_c128") == 2
        assert sv.sv_tune_get("tile_log2_c128") == 11 and sv.sv_tune_get("tile_low_bits_c128") == 5
        assert sv.sv_tune_get("wave_auto") == 0 and sv.sv_tune_get("low_policy") == 0
        bad = tmp_path / "bad.json"
        bad.write_text('{"arch": "gfx950:sramecc+:xnack-", "dtype": "c128", "granule_bits": 99, '
                       '"low_policy": 0, "wave_auto": 0, "tile_log2": 11, "tile_low_bits": 5}\n')
        with pytest.raises(sv.SvError):
            sv.sv_tune_load(str(bad))
        with pytest.raises(sv.SvError):
            sv.sv_tune_load(str(tmp_path / "missing.json"))
    finally:
        for k, v in before.items():
            sv.sv_tune_set(k, v)


# ---------------------------------------------------------------- fixed-point states

def test_fixed_point_state_bytes(sv):
    for n in (1, 5, 6, 7, 12, 28, 36):
        want = (4 << n) + max(1, (1 << n) // 64)
        assert sv.sv_state_bytes(n, sv.SV_CQ16) == want == sv.q16_nbytes(n)
    for n in (1, 5, 6, 12, 35):
        want = (8 << n) + max(1, (1 << n) // 64)
        assert sv.sv_state_bytes(n, sv.SV_CQ32) == want == sv.fixed_nbytes(n, sv.SV_CQ32)
    assert _rc(lambda: sv.sv_state_bytes(36, sv.SV_CQ32))[0] == sv.SV_EINVAL
    assert sv.sv_state_bytes(28, sv.SV_C128) == 16 << 28 and sv.sv_state_bytes(28, sv.SV_C64) == 8 << 28
    code, msg = _rc(lambda: sv.sv_state_bytes(37, sv.SV_CQ16))
    assert code == sv.SV_EINVAL


@pytest.mark.parametrize("bits", [16, 32])
@pytest.mark.parametrize("n,t,ctrls,masked,name,units", [
    (28, 13, (17, 22), False, "false, true, false", 1 << 19),   # block pairs: 2^(22-1-2)
    (28, 13, (17, 22), True, "true, true, false", 1 << 21),     # every block pair
    (28, 3, (0, 20), False, "false, false, true", 1 << 21),     # blocks: 2^(22-1), qubit 0 tested
    (28, 3, (0, 1), False, "false, false, true", 1 << 22),      # only in-block controls
    (6, 5, (0,), False, "false, false, true", 1),
    (5, 4, (0, 1), False, "small", 1),
])
def test_fixed_point_gate_plan(sv, bits, n, t, ctrls, masked, name, units):
    cm = sum(1 << q for q in ctrls)
    dtype = sv.SV_CQ16 if bits == 16 else sv.SV_CQ32
    k, it = sv.sv_gate_plan(n, dtype, t, cm, cm, "masked" if masked else "auto")
    want = ("k_fix_gate_small<sv::Q%d" % bits) if name == "small" else ("k_fix_gate<sv::Q%d, %s" % (bits, name))
    assert want in k and it == units, (k, it)


def test_fixed_point_rejected_where_unsupported(sv):
    L = sv.lib()
    s = _state(sv, 10, sv.SV_CQ16)
    code, msg = _rc(lambda: sv.sv_swap_qubits(s, [(0, 9)]))
    assert code == sv.SV_ENOTSUP and "fixed-point" in msg
    code, msg = _rc(lambda: sv.sv_apply_dense_low(s, 4, __import__("numpy").eye(16)))
    assert code == sv.SV_ENOTSUP
    # expectation values read fixed-point codes; H psi (a fixed-point output) does not
    terms = (sv.sv_pauli_t * 1)()
    out = _state(sv, 10, sv.SV_CQ16, 0x900000)
    rc = L.sv_apply_pauli_sum(ctypes.byref(s), ctypes.byref(out), terms, 1, None)
    assert rc == sv.SV_ENOTSUP
    # circuits: dense blocks and remapping are not offered (fusion is)
    for flags in (sv.SV_DENSE | sv.SV_FUSE, sv.SV_REMAP):
        code, msg = _rc(lambda: sv.Circuit(10, [], dtype=sv.SV_CQ16, flags=flags))
        assert code == sv.SV_ENOTSUP and "SV_CQ16" in msg, msg
    # 16-byte alignment, and the usual gate checks
    code, msg = _rc(lambda: sv.sv_apply_gate(_state(sv, 10, sv.SV_CQ16, 0x10008), 0, U=U))
    assert code == sv.SV_EINVAL and "aligned" in msg
    code, msg = _rc(lambda: sv.sv_apply_gate(s, 3, controls=(3,), U=U))
    assert code == sv.SV_EINVAL and "equals the target" in msg
    code, msg = _rc(lambda: sv.sv_apply_gate(s, 3, U=U, mode=9))
    assert code == sv.SV_EINVAL and "mode" in msg


def test_convert_argument_errors(sv):
    code, msg = _rc(lambda: sv.sv_convert(_state(sv, 10, sv.SV_CQ32, 0x100000),
                                          _state(sv, 10, sv.SV_CQ16, 0x900000)))
    assert code == sv.SV_ENOTSUP and "complex128" in msg
    code, msg = _rc(lambda: sv.sv_swap_qubits(_state(sv, 10, sv.SV_CQ32), [(0, 9)]))
    assert code == sv.SV_ENOTSUP
    a = _state(sv, 10, sv.SV_CQ16, 0x100000)
    code, msg = _rc(lambda: sv.sv_convert(a, _state(sv, 11, sv.SV_C128, 0x900000)))
    assert code == sv.SV_EINVAL and "qubits" in msg
    code, msg = _rc(lambda: sv.sv_convert(a, _state(sv, 10, sv.SV_C128, 0x100000 + 4096)))
    assert code == sv.SV_EINVAL and "overlap" in msg


def test_expect_noalloc_rejects_too_many_terms(sv):
    """The allocation-free expectation holds at most 64 terms in its
    workspace; more is an argument error raised before any device use."""
    s = _state(sv, 8)
    arr = sv.pauli_terms([(1.0, 0, 1 << (i % 8)) for i in range(65)])
    rc = sv.lib().sv_expect_noalloc(ctypes.byref(s), arr, 65, ctypes.c_void_p(0x20000), None)
    assert rc == sv.SV_EINVAL and "allocation-free limit of 64" in sv.sv_last_error()


def test_hbm_probe_argument_errors(sv):
    s = _state(sv, 8)
    for args, needle in (((1 << 9, 0, 0), "bits >= n"), ((3, 4, 0), "outside fixed_mask"), ((0, 0, 5), "operation")):
        code, msg = _rc(lambda: sv.sv_hbm_probe(s, *args))
        assert code == sv.SV_EINVAL and needle in msg, msg


def test_two_valued_knobs(sv):
    for key, good, bad in (("pair_unroll", (1, 4), 2), ("masked_unroll", (1, 4), 3), ("masked_block", (64, 256), 128)):
        old = sv.sv_tune_get(key)
        try:
            for v in good:
                sv.sv_tune_set(key, v)
                assert sv.sv_tune_get(key) == v
            code, msg = _rc(lambda: sv.sv_tune_set(key, bad))
            assert code == sv.SV_EINVAL and "takes" in msg
        finally:
            sv.sv_tune_set(key, old)


def test_adjoint_rejects_non_unitary_matrix(sv):
    """The reverse sweep un-applies gates by their conjugate transpose, so a
    fixed matrix that is not unitary is an argument error (before any device
    use)."""
    import numpy as np
    import workloads as W
    psi, lam = _state(sv, 4, ptr=0x10000), _state(sv, 4, ptr=0x20000)
    M = np.array([[1.0, 0.0], [0.0, 1.0 + 1e-9]], dtype=np.complex128)  # off by 1e-9
    m8 = tuple(np.stack([M.real, M.imag], axis=-1).reshape(8))
    c = W.Circuit(4, [W.Gate("RY", 0, param=0), W.Gate("U", 1, (0,), matrix=m8)], np.array([0.3]))
    gates = sv.circuit_gates(c)
    terms = sv.pauli_terms([W.PauliTerm(1.0, 0, 1)])
    rc = sv.lib().sv_adjoint_grad(ctypes.byref(psi), ctypes.byref(lam), gates, 2, ctypes.c_void_p(0x30000), 1,
                                  terms, 1, ctypes.c_void_p(0x40000), None, None, None)
    assert rc == sv.SV_EINVAL and "not unitary" in sv.sv_last_error(), sv.sv_last_error()


def test_adjoint_plan_argument_errors(sv):
    import numpy as np
    """Planned adjoint: validation at creation names the bad gate; a run on
    states of another shape, or a NULL plan, is an argument error."""
    import workloads as W
    bad = W.Circuit(4, [W.Gate("RY", 7, param=0)], np.array([0.1]))
    code, msg = _rc(lambda: sv.AdjointPlan(4, bad, [W.PauliTerm(1.0, 0, 1)], 1))
    assert code == sv.SV_EINVAL and "gate 0" in msg, msg
    s = _state(sv, 4)
    assert sv.lib().sv_adjoint_run(None, ctypes.byref(s), ctypes.byref(s), None, None, None, None, None) == sv.SV_EINVAL


@pytest.mark.parametrize("dtype,mode,t,ctrls,want,units", [
    ("c128", "auto", 13, (), "sv::k_pair_xw<double, unsigned int, 1, sv::MatVal<double> >", 1 << 27),
    ("c128", "auto", 27, (3, 20), "sv::k_pair_xw<double, unsigned int, 1, sv::MatVal<double> >", 1 << 25),
    ("c64", "auto", 13, (), "sv::k_pair<float, unsigned int, 1, 1, 64, sv::MatVal<float> >", 1 << 27),
    ("c128", "masked", 13, (5,), "sv::k_pair<double, unsigned int, 1, 0, 256, sv::MatVal<double> >", 1 << 27),
    ("c64", "masked", 13, (5,), "sv::k_pair<float, unsigned int, 1, 0, 256, sv::MatVal<float> >", 1 << 27),
    ("c128", "auto", 0, (), "sv::k_wave<double, 1, 1, sv::MatVal<double> >", 1 << 22),
])
def test_single_gate_kernel_choice(sv, dtype, mode, t, ctrls, want, units):
    """The kernel a single gate launches at n=28 (its name as the profiler
    reports it) and its work items: complex128 scheduled pairs run the
    cross-wavefront form (64 pairs per workgroup), complex64 keeps one pair
    per lane, the masked baseline runs over all 2^(n-1) pairs with one pair
    per lane, low targets take the wavefront kernel."""
    cm = sum(1 << q for q in ctrls)
    code = sv.SV_C128 if dtype == "c128" else sv.SV_C64
    k, it = sv.sv_gate_plan(28, code, t, cm, cm, mode)
    assert k == want and it == units, (k, it)
