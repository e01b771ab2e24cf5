"""GPU parity of the circuit path (sv_apply_circuit / sv_circuit_*) against
the oracle: fused, unfused, masked and graph-replayed runs, device-resident
angles, the paper's QFT and streaming circuits, and the layered circuit."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}


def _say(*a):
    print(*a, flush=True)


def _err(got, ref):
    return float(np.max(np.abs(got.astype(np.complex128) - ref)) / np.max(np.abs(ref)))


def _dev_state(n, dtype, psi=None):
    import torch
    td = torch.complex128 if dtype == "c128" else torch.complex64
    if psi is None:
        return torch.empty(1 << n, dtype=td, device="cuda")
    return torch.from_numpy(psi).to(td).cuda()


def _rand_circuit(n, ngates, seed, nparams=0):
    rng = np.random.default_rng(seed)
    kinds = ("X", "Y", "Z", "H", "RX", "RY", "RZ", "P", "U", "~RY", "~U")
    gates = []
    for i in range(ngates):
        k = kinds[int(rng.integers(0, len(kinds)))]
        t = int(rng.integers(0, n))
        others = [q for q in range(n) if q != t]
        c = int(rng.integers(0, 4))
        ctrls = tuple(int(q) for q in rng.choice(others, size=c, replace=False)) if c else ()
        vals = tuple(int(v) for v in rng.integers(0, 2, size=c))
        th = float(rng.uniform(0, 2 * np.pi))
        mat = W.haar_unitary_2x2(seed * 1000 + i) if k.endswith("U") else None
        p = int(rng.integers(0, nparams)) if (nparams and k in ("RX", "RY", "RZ", "P") and rng.random() < 0.7) else -1
        gates.append(W.Gate(k, t, ctrls, vals, th, p, mat))
    params = rng.uniform(0, 2 * np.pi, size=nparams) if nparams else None
    return W.Circuit(n, gates, params)


FLAGS = {"fuse": 1, "plain": 0, "masked": 4, "fuse+graph": 3}


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("flags", list(FLAGS))
def test_random_gates_n12(gpu, dtype, flags):
    c = W.random_gates_n12()
    ref = oracle.run_circuit(c)
    d = _dev_state(c.n, dtype)
    gpu.sv_init(d, 0)
    if "graph" in flags:
        circ = gpu.Circuit(c.n, c, dtype=0 if dtype == "c128" else 1, flags=FLAGS[flags])
        for _ in range(3):
            gpu.sv_init(d, 0)
            circ.run(d)
        circ.close()
    else:
        gpu.sv_apply_circuit(d, c, flags=FLAGS[flags])
    e = _err(d.cpu().numpy(), ref)
    _say("random_gates_n12", dtype, flags, e)
    assert e <= TOL[dtype]


@pytest.mark.parametrize("tile", [6, 9, 12])
@pytest.mark.parametrize("seed", [1, 2])
def test_random_circuits_device_params(gpu, tile, seed):
    import torch
    gpu.sv_tune_set("tile_log2_c128", tile)
    try:
        for n in (7, 11, 14):
            c = _rand_circuit(n, 250, seed * 10 + n, nparams=12)
            psi0 = W.random_state(n, seed)
            ref = oracle.run_circuit(c, c.params, psi0)
            params = torch.from_numpy(c.params).cuda()
            outs = {}
            for name, fl in FLAGS.items():
                d = _dev_state(n, "c128", psi0)
                gpu.sv_apply_circuit(d, c, params=params, flags=fl)
                outs[name] = d.cpu().numpy()
                assert _err(outs[name], ref) <= 1e-12, (n, name, tile)
            # unfused and masked apply identical arithmetic in the same order
            assert np.array_equal(outs["plain"].view(np.uint8), outs["masked"].view(np.uint8))
    finally:
        gpu.sv_tune_set("tile_log2_c128", 12)


def test_graph_replay_new_params(gpu):
    """One captured graph replayed with new angle values written into the same
    device array; eager work and synchronisation between replays; every
    replay checked against the oracle and against an eager run."""
    import torch
    n = 13
    c = _rand_circuit(n, 200, 77, nparams=8)
    params = torch.zeros(8, dtype=torch.float64, device="cuda")
    circ = gpu.Circuit(n, c, nparams=8, flags=gpu.SV_FUSE | gpu.SV_GRAPH)
    eager = gpu.Circuit(n, c, nparams=8, flags=gpu.SV_FUSE)
    d = _dev_state(n, "c128")
    e = _dev_state(n, "c128")
    rng = np.random.default_rng(5)
    for rep in range(4):
        p = rng.uniform(0, 2 * np.pi, size=8)
        params.copy_(torch.from_numpy(p))
        gpu.sv_init(d, rep)
        gpu.sv_init(e, rep)
        circ.run(d, params)
        torch.cuda.synchronize()
        eager.run(e, params)
        psi0 = np.zeros(1 << n, dtype=np.complex128); psi0[rep] = 1
        ref = oracle.run_circuit(c, p, psi0)
        assert _err(d.cpu().numpy(), ref) <= 1e-12, rep
        assert torch.equal(d.view(torch.float64), e.view(torch.float64)), rep
    circ.close(); eager.close()


@pytest.mark.parametrize("n", [5, 12, 16])
def test_qft_and_stream_closed_forms(gpu, n):
    N = 1 << n
    psi0 = W.random_state(n, 3)
    for name, circ in (("qft", W.qft(n)), ("stream", W.stream(n))):
        for fl in (1, 4):
            d = _dev_state(n, "c128", psi0)
            gpu.sv_apply_circuit(d, circ, flags=fl)
            got = d.cpu().numpy()
            if name == "qft":
                rev = np.array([int(format(x, "0%db" % n)[::-1], 2) for x in range(N)])
                ref = np.fft.ifft(psi0[rev]) * np.sqrt(N)
            else:
                ref = np.roll(psi0, -1)
            assert _err(got, ref) <= 1e-12, (name, n, fl)


def test_layered_circuit_small(gpu):
    """The layered circuit's construction at n=20 (all 20 layers) against the oracle."""
    c = W.layered_circuit_n32(n=20)
    ref = oracle.run_circuit(c)
    for fl in (1, 0):
        d = _dev_state(c.n, "c128")
        gpu.sv_init(d, 0)
        gpu.sv_apply_circuit(d, c, flags=fl)
        assert _err(d.cpu().numpy(), ref) <= 1e-12, fl


def test_invalid_circuit_leaves_state(gpu):
    import torch
    n = 8
    d = _dev_state(n, "c128", W.random_state(n, 1))
    before = d.clone()
    bad = [W.Gate("H", 0), W.Gate("X", 2), W.Gate("X", 3, (3,))]
    with pytest.raises(gpu.SvError):
        gpu.sv_apply_circuit(d, bad)
    torch.cuda.synchronize()
    assert torch.equal(d, before)


@pytest.mark.parametrize("low", [2, 4, 6])
def test_qubit_set_tiles(gpu, low):
    """Fused tiles over the `low` lowest qubits plus planner-chosen ones (small
    tiles force many high qubits per run); random gates of every kind, device
    angles, against the oracle."""
    import torch
    gpu.sv_tune_set("tile_log2_c128", 8)
    gpu.sv_tune_set("tile_low_bits_c128", low)
    try:
        for n, seed in ((9, 1), (14, 2), (16, 3)):
            c = _rand_circuit(n, 300, 400 + seed, nparams=6)
            psi0 = W.random_state(n, seed)
            ref = oracle.run_circuit(c, c.params, psi0)
            params = torch.from_numpy(c.params).cuda()
            circ = gpu.Circuit(n, c, nparams=6, flags=gpu.SV_FUSE)
            info = circ.info()
            d = _dev_state(n, "c128", psi0)
            circ.run(d, params)
            circ.close()
            assert _err(d.cpu().numpy(), ref) <= 1e-12, (n, low, info)
            assert info["passes"] < len(c.gates) // 3, info
    finally:
        gpu.sv_tune_set("tile_log2_c128", 12)
        gpu.sv_tune_set("tile_low_bits_c128", 6)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_qft_fused_large(gpu, dtype):
    """QFT at n=20 (a handful of fused passes over qubit-set tiles) against
    its closed form."""
    n, N = 20, 1 << 20
    psi0 = W.random_state(n, 9)
    d = _dev_state(n, dtype, psi0)
    circ = gpu.Circuit(n, W.qft(n), dtype=0 if dtype == "c128" else 1, flags=gpu.SV_FUSE)
    assert circ.info()["passes"] <= 4
    circ.run(d)
    rev = np.array([int(format(x, "020b")[::-1], 2) for x in range(N)])
    ref = np.fft.ifft(psi0[rev]) * np.sqrt(N)
    assert _err(d.cpu().numpy(), ref) <= TOL[dtype]
    circ.close()


@pytest.mark.parametrize("tile,low", [(6, 3), (8, 4), (12, 6)])
def test_stream_fused_tile_scheduling(gpu, tile, low):
    """Streaming circuits (gate j controlled by all lower qubits): fused runs
    launch only the tiles whose shared outer control bits hold.  Closed form
    |x> -> |x-1>, plus controlled streams with negative controls against the
    oracle."""
    gpu.sv_tune_set("tile_log2_c128", tile)
    gpu.sv_tune_set("tile_low_bits_c128", low)
    try:
        for n in (10, 17):
            psi0 = W.random_state(n, n)
            d = _dev_state(n, "c128", psi0)
            gpu.sv_apply_circuit(d, W.stream(n), flags=gpu.SV_FUSE)
            assert _err(d.cpu().numpy(), np.roll(psi0, -1)) <= 1e-12, (n, tile)
            g = [W.Gate("H", q) for q in range(n)] + [
                W.Gate("RY" if j % 2 else "X", j, tuple(range(j)), tuple((j + k) % 2 for k in range(j)), 0.4 + j)
                for j in range(1, n)]
            c = W.Circuit(n, g)
            ref = oracle.run_circuit(c, psi0=psi0)
            d = _dev_state(n, "c128", psi0)
            gpu.sv_apply_circuit(d, c, flags=gpu.SV_FUSE)
            assert _err(d.cpu().numpy(), ref) <= 1e-12, (n, tile, "controlled")
    finally:
        gpu.sv_tune_set("tile_log2_c128", 12)
        gpu.sv_tune_set("tile_low_bits_c128", 6)


def _diag_heavy(n, seed, blocks=6, per_block=14):
    """Blocks of controlled phase / RZ gates on random qubits (0-3 controls,
    some negative) separated by H layers: long diagonal sweeps whose gates
    read every mix of tile-local and outer bits."""
    rng = np.random.default_rng(seed)
    gates = []
    for b in range(blocks):
        for q in rng.choice(n, size=3, replace=False):
            gates.append(W.Gate("H", int(q)))
        for i in range(per_block):
            t = int(rng.integers(0, n))
            others = [q for q in range(n) if q != t]
            k = int(rng.integers(0, 4))
            ctrls = tuple(int(q) for q in rng.choice(others, size=k, replace=False)) if k else ()
            vals = tuple(int(v) for v in rng.integers(0, 2, size=k)) if k else ()
            gates.append(W.Gate("P" if i % 2 else "RZ", t, ctrls, vals, float(rng.uniform(0, 2 * np.pi))))
    return W.Circuit(n, gates, meta={"name": "diag_heavy", "seed": seed})


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("width", [0, 8, 10])
def test_fused_diag_sweeps(gpu, dtype, width):
    """Long diagonal sweeps (the QFT's controlled phases and random
    controlled phases: phases added through tables, one sine and cosine per
    amplitude), short ones (factors multiplied), and fused runs of controlled
    pair gates, at n=16, for the default tile width and narrower ones."""
    import torch
    n = 16
    key = "tile_log2_" + dtype
    old = gpu.sv_tune_get(key)
    if width:
        gpu.sv_tune_set(key, width)
    try:
        _check_diag_circuits(gpu, dtype, n)
    finally:
        gpu.sv_tune_set(key, old)


def _check_diag_circuits(gpu, dtype, n):
    import torch
    circs = [W.qft(n), _diag_heavy(n, 5), W.random_gates_n12(seed=21, n=n, ngates=400), W.hea(n, 3, seed=8)]
    psi0 = W.random_state(n, 3)  # every amplitude nonzero, so every phase counts
    for c in circs:
        params = None if c.params is None else torch.from_numpy(c.params).cuda()
        ref = oracle.run_circuit(c, c.params, psi0)
        d = torch.from_numpy(psi0).cuda()
        if dtype == "c64":
            d = d.to(torch.complex64)
        plan = gpu.Circuit(n, c, dtype=0 if dtype == "c128" else 1, nparams=c.nparams, flags=gpu.SV_FUSE)
        plan.run(d, params)
        plan.close()
        e = float(np.max(np.abs(d.cpu().numpy().astype(np.complex128) - ref)))
        assert e <= (1e-12 if dtype == "c128" else 1e-5), (c.meta, e)


def test_layered_circuit_n32_full(gpu):
    """The layered circuit at its full size (n=32, complex128, 64 GiB per
    state), where the oracle cannot run: the fused plan agrees with the
    unfused one everywhere, the norm stays 1, and the fused inverse circuit
    brings the state back to |0...0>."""
    import torch
    free, _ = torch.cuda.mem_get_info()
    if free < (140 << 30):
        pytest.skip("needs about 130 GiB of free device memory")
    n = 32
    c = W.layered_circuit_n32()
    a = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    b = torch.empty_like(a)
    gpu.sv_init(a, 0)
    gpu.sv_apply_circuit(a, c, flags=gpu.SV_FUSE)
    gpu.sv_init(b, 0)
    gpu.sv_apply_circuit(b, c, flags=0)
    chunk = 1 << 27
    diff, norm = 0.0, 0.0
    for o in range(0, 1 << n, chunk):
        x, y = a[o:o + chunk], b[o:o + chunk]
        diff = max(diff, float((x - y).abs().max()))
        norm += float(x.abs().pow(2).sum())
    assert diff <= 1e-12, diff
    assert abs(norm - 1.0) <= 1e-10, norm
    del b
    gpu.sv_apply_circuit(a, W.inverse(c), flags=gpu.SV_FUSE)
    assert abs(complex(a[0].item()) - 1.0) <= 1e-10
    rest = 0.0
    for o in range(0, 1 << n, chunk):
        x = a[o:o + chunk]
        rest = max(rest, float(x.abs().max()) if o else float(x[1:].abs().max()))
    assert rest <= 1e-10, rest


def test_empty_circuit(gpu):
    """A circuit without gates is a valid plan that leaves the state as it is."""
    import torch
    n = 12
    psi = W.random_state(n, 9)
    for flags in (0, gpu.SV_FUSE, gpu.SV_FUSE | gpu.SV_GRAPH):
        d = torch.from_numpy(psi).cuda()
        gpu.sv_apply_circuit(d, W.Circuit(n, []), flags=flags & ~gpu.SV_GRAPH)
        plan = gpu.Circuit(n, W.Circuit(n, []), flags=flags)
        plan.run(d)
        plan.close()
        assert torch.equal(d.cpu(), torch.from_numpy(psi)), flags


def _mixed_circuit(n, seed):
    """Random controlled gates, diagonal-heavy blocks and parameterised
    rotations interleaved (draw order fixed by the seed)."""
    rng = np.random.default_rng(seed)
    gates, p = [], 0
    for block in range(4):
        gates += W.random_gates_n12(seed=seed * 10 + block, n=n, ngates=40).gates
        gates += _diag_heavy(n, seed * 10 + block, blocks=1, per_block=int(rng.integers(4, 16))).gates
        for _ in range(6):
            t = int(rng.integers(0, n))
            c = [q for q in range(n) if q != t]
            kind = ("RY", "RZ", "RX", "P")[int(rng.integers(0, 4))]
            # controls on RY/RZ only: the oracle's shift rule covers those
            ctrls = (int(rng.choice(c)),) if kind in ("RY", "RZ") and rng.random() < 0.5 else ()
            gates.append(W.Gate(kind, t, ctrls, (), param=p))
            p += 1
    return W.Circuit(n, gates, rng.uniform(0, 2 * np.pi, size=p), meta={"seed": seed})


@pytest.mark.parametrize("seed", range(6))
def test_fused_random_configurations(gpu, seed):
    """Random tile widths and low-block sizes on circuits mixing every
    operation kind, fused (with device angles) against the oracle, complex128
    and complex64."""
    import torch
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(10, 17))
    c = _mixed_circuit(n, seed)
    keys = ("tile_log2_c128", "tile_log2_c64", "tile_low_bits_c128", "tile_low_bits_c64")
    old = {k: gpu.sv_tune_get(k) for k in keys}
    try:
        w = int(rng.integers(7, 13))
        low = int(rng.integers(1, 7))
        gpu.sv_tune_set("tile_log2_c128", w)
        gpu.sv_tune_set("tile_log2_c64", w + 1)
        gpu.sv_tune_set("tile_low_bits_c128", low)
        gpu.sv_tune_set("tile_low_bits_c64", low)
        psi0 = W.random_state(n, seed)
        ref = oracle.run_circuit(c, c.params, psi0)
        params = torch.from_numpy(c.params).cuda()
        for dtype, tol in ((0, 1e-12), (1, 1e-5)):
            d = torch.from_numpy(psi0).cuda()
            if dtype == 1:
                d = d.to(torch.complex64)
            plan = gpu.Circuit(n, c, dtype=dtype, nparams=c.nparams, flags=gpu.SV_FUSE)
            plan.run(d, params)
            plan.close()
            e = float(np.max(np.abs(d.cpu().numpy().astype(np.complex128) - ref)))
            assert e <= tol, (seed, n, w, low, dtype, e)
    finally:
        for k, v in old.items():
            gpu.sv_tune_set(k, v)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_swap_qubits(gpu, dtype):
    """sv_swap_qubits is an exact relabelling: bit-identical to the oracle's
    exchange for single and multiple disjoint pairs, low and high qubits."""
    import torch
    for n, pairs in ((12, [(0, 11)]), (12, [(0, 7), (1, 9), (2, 3)]), (20, [(0, 19), (1, 18), (2, 17), (5, 6)]),
                     (7, [(0, 6), (1, 5), (2, 4)])):
        psi = W.random_state(n, n + len(pairs))
        d = torch.from_numpy(psi).cuda()
        if dtype == "c64":
            d = d.to(torch.complex64)
            psi = d.cpu().numpy().astype(np.complex128)
        ref = oracle.swap_qubits(psi.copy(), n, pairs)
        gpu.sv_swap_qubits(d, pairs)
        assert np.array_equal(d.cpu().numpy().astype(np.complex128), ref), (n, pairs)


def test_swap_qubits_rejects_bad_pairs(gpu):
    import torch
    d = torch.from_numpy(W.random_state(8, 1)).cuda()
    before = d.clone()
    for pairs in ([(0, 0)], [(0, 8)], [(1, 2), (2, 3)], [(-1, 2)]):
        with pytest.raises(gpu.SvError):
            gpu.sv_swap_qubits(d, pairs)
    torch.cuda.synchronize()
    assert torch.equal(d, before)


@pytest.mark.parametrize("flags", [0, 1, 3])
def test_remapped_circuits(gpu, flags):
    """SV_REMAP moves the heavily used low controls to high bit positions and
    back: the same state as the oracle (unfused, fused, fused + graph)."""
    import torch
    n = 14
    c = W.low_control_circuit(n=n, ngates=40, seed=4)
    psi0 = W.random_state(n, 6)
    ref = oracle.run_circuit(c, None, psi0)
    d = torch.from_numpy(psi0).cuda()
    plan = gpu.Circuit(n, c, flags=flags | gpu.SV_REMAP)
    base = gpu.Circuit(n, c, flags=flags)
    if flags == 0:  # unfused: the same gate passes plus the two exchanges
        assert plan.info()["passes"] == base.info()["passes"] + 2
    base.close()
    for rep in range(2):  # graph replays too
        d.copy_(torch.from_numpy(psi0))
        plan.run(d)
        assert _err(d.cpu().numpy(), ref) <= 1e-12, (flags, rep)
    plan.close()


def _x_runs(n, seed, nruns=40):
    """Runs of 2-10 X gates (0-3 controls anywhere, some negative) between
    single rotations and H gates: permutation runs whose gates read
    tile-local, outer and in-tile-negated controls."""
    rng = np.random.default_rng(seed)
    gates = [W.Gate("H", q) for q in range(n)]
    for _ in range(nruns):
        for _ in range(int(rng.integers(2, 11))):
            t = int(rng.integers(0, n))
            others = [q for q in range(n) if q != t]
            c = int(rng.integers(0, 4))
            ctrls = tuple(int(q) for q in rng.choice(others, size=c, replace=False)) if c else ()
            vals = tuple(int(v) for v in rng.integers(0, 2, size=c))
            gates.append(W.Gate("X", t, ctrls, vals))
        q = int(rng.integers(0, n))
        gates.append(W.Gate("RY" if rng.random() < 0.5 else "H", q, (), (), float(rng.uniform(0, 2 * np.pi))))
    return W.Circuit(n, gates)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_permutation_runs(gpu, dtype):
    """Runs of X gates applied as one gather per tile: a GHZ ladder, the
    layered circuit and random X runs, on the default tiles and on narrow
    ones, against the oracle and (exactly) against the same plans with the
    runs applied gate by gate."""
    import torch
    circs = [(14, W.ghz(14), 0), (16, W.layered_circuit_n32(n=16, layers=4), 0), (15, _x_runs(15, 3), 0),
             (13, _x_runs(13, 4), 8)]
    for n, c, width in circs:
        if width:
            gpu.sv_tune_set("tile_log2_" + dtype, width)
        psi0 = W.random_state(n, n + width)
        ref = oracle.run_circuit(c, None, psi0)
        got = {}
        for perm in (1, 0):
            gpu.sv_tune_set("fuse_perm", perm)
            d = _dev_state(n, dtype, psi0)
            circ = gpu.Circuit(n, c, dtype=0 if dtype == "c128" else 1, flags=gpu.SV_FUSE)
            circ.run(d)
            circ.close()
            got[perm] = d.cpu()
            e = _err(got[perm].numpy(), ref)
            _say("perm", perm, dtype, "n", n, "width", width, "err", e)
            assert e <= TOL[dtype], (n, perm, e)
        assert torch.equal(got[0], got[1]), n
        gpu.sv_tune_set("fuse_perm", 1)
