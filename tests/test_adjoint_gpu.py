"""GPU parity of expectation values and adjoint gradients against the
oracle: <psi|H|psi> and H psi to 1e-12, gradients to 1e-8 against the
oracle's parameter-shift rule, through the C ABI and through torch.autograd."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _rand_terms(n, nterms, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nterms):
        x = int(rng.integers(0, 1 << n))
        z = int(rng.integers(0, 1 << n))
        if rng.random() < 0.3:
            x = 0
        out.append(W.PauliTerm(float(rng.standard_normal()), x, z))
    return out


def _dev(psi, dtype="c128"):
    import torch
    t = torch.from_numpy(psi)
    return (t if dtype == "c128" else t.to(torch.complex64)).cuda()


@pytest.mark.parametrize("n", [1, 3, 8, 14])
def test_expect_random_paulis(gpu, n):
    psi = W.random_state(n, 40 + n)
    terms = _rand_terms(n, 40, n)
    d = _dev(psi)
    tot = gpu.sv_expect(d, terms).item()
    per = gpu.sv_expect_terms(d, terms).cpu().numpy()
    ref_per = np.array([oracle.expect_pauli(psi, n, t.x_mask, t.z_mask).real for t in terms])
    ref = oracle.expect(psi, n, terms)
    assert np.max(np.abs(per - ref_per)) <= 1e-12
    assert abs(tot - ref) <= 1e-12 * max(1.0, np.sum(np.abs([t.coef for t in terms])))
    # deterministic: same bits on a second evaluation
    assert gpu.sv_expect(d, terms).item() == tot
    # complex64 against the fp64 oracle
    tot64 = gpu.sv_expect(_dev(psi, "c64"), terms).item()
    assert abs(tot64 - ref) <= 1e-5 * max(1.0, np.sum(np.abs([t.coef for t in terms])))


def _tile_mix_terms(n, seed):
    """Terms for every path of the expectation passes: the chain ZZ + X
    Hamiltonian; 70 more diagonal terms (a tile set of more than 64 terms
    takes two passes); 20 terms sharing one x mask (groups split at 16);
    x masks with at most six qubits above qubit 5 (tile sets beyond the
    first) and, for n > 12, masks with more (a pass per group); Y terms on
    the lowest and highest qubits."""
    rng = np.random.default_rng(seed)
    terms = list(W.zz_x_hamiltonian(n, seed))
    terms += [W.PauliTerm(float(rng.standard_normal()), 0, int(rng.integers(0, 1 << n))) for _ in range(70)]
    xs = int(rng.integers(1, 1 << n))
    terms += [W.PauliTerm(float(rng.standard_normal()), xs, int(rng.integers(0, 1 << n))) for _ in range(20)]
    for _ in range(16):
        hi = rng.choice(np.arange(min(6, n), n), size=min(n - min(6, n), int(rng.integers(0, 7))), replace=False)
        x = int(rng.integers(0, 1 << min(6, n))) | sum(1 << int(q) for q in hi)
        terms.append(W.PauliTerm(float(rng.standard_normal()), x, int(rng.integers(0, 1 << n))))
    if n > 12:
        for _ in range(6):
            terms.append(W.PauliTerm(float(rng.standard_normal()), int(rng.integers(1, 1 << n)) | (0x7f << (n - 7)),
                                     int(rng.integers(0, 1 << n))))
    top = n - 1
    terms += [W.PauliTerm(0.5, 1, 1), W.PauliTerm(-0.25, 1 << top, 1 << top)]
    return terms


@pytest.mark.parametrize("n", [2, 5, 12, 13, 18, 20])
def test_expect_tile_passes(gpu, n):
    """Per-term values and the total against the oracle at 1e-12 for a
    Hamiltonian that reaches every pass kind (tile sets, split sets, split
    groups, masks too wide for a tile); the allocation-free entry point
    gives the total of its first 64 terms bit for bit."""
    import torch
    psi = W.random_state(n, 90 + n)
    terms = _tile_mix_terms(n, 91 + n)
    d = _dev(psi)
    per = gpu.sv_expect_terms(d, terms).cpu().numpy()
    tot = gpu.sv_expect(d, terms).item()
    ref_per = np.array([oracle.expect_pauli(psi, n, t.x_mask, t.z_mask).real for t in terms])
    l1 = float(np.sum(np.abs([t.coef for t in terms])))
    e = float(np.max(np.abs(per - ref_per)))
    _say("n", n, "terms", len(terms), "max term err", e)
    assert e <= 1e-12
    assert abs(tot - oracle.expect(psi, n, terms)) <= 1e-12 * l1
    few = terms[-64:]
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    gpu.sv_expect_noalloc(d, few, out)
    assert out.item() == gpu.sv_expect(d, few).item()
    assert abs(out.item() - oracle.expect(psi, n, few)) <= 1e-12 * float(np.sum(np.abs([t.coef for t in few])))


@pytest.mark.parametrize("n", [2, 9, 13])
def test_apply_pauli_sum(gpu, n):
    import torch
    psi = W.random_state(n, 7)
    terms = _rand_terms(n, 25, 100 + n)
    d = _dev(psi)
    out = torch.empty_like(d)
    gpu.sv_apply_pauli_sum(d, out, terms)
    ref = oracle.apply_hamiltonian(psi, n, terms)
    assert np.max(np.abs(out.cpu().numpy() - ref)) <= 1e-12 * np.max(np.abs(ref))


def _grad_check(gpu, circ, terms, ref, tol=1e-8):
    import torch
    params = torch.from_numpy(circ.params).cuda()
    psi = torch.empty(1 << circ.n, dtype=torch.complex128, device="cuda")
    gpu.sv_init(psi, 0)
    gpu.sv_apply_circuit(psi, circ, params=params)
    lam = torch.empty_like(psi)
    grad, loss = gpu.sv_adjoint_grad(psi, lam, circ, params, terms)
    g = grad.cpu().numpy()
    err = np.max(np.abs(g - ref)) / max(1.0, np.max(np.abs(ref)))
    assert err <= tol, err
    # the sweep un-applies every gate: psi is back to |0...0>
    back = psi.cpu().numpy()
    e0 = np.zeros_like(back); e0[0] = 1
    assert np.max(np.abs(back - e0)) <= 1e-12
    assert abs(loss.item() - oracle.loss(circ, circ.params, terms)) <= 1e-12 * max(1, sum(abs(t.coef) for t in terms))
    return err


@pytest.mark.parametrize("n,layers", [(4, 2), (8, 3), (12, 2)])
def test_adjoint_hea_vs_param_shift(gpu, n, layers):
    c = W.hea(n, layers, seed=n)
    terms = W.zz_x_hamiltonian(n, n)
    ref = oracle.grad_param_shift(c, c.params, terms)
    err = _grad_check(gpu, c, terms, ref)
    _say("hea n=%d err %.2e" % (n, err))


def test_adjoint_controlled_rotations_vs_param_shift(gpu):
    """Controlled RY/RZ with positive and negative controls, parameters
    shared between gates, fixed gates in between (including adjoints)."""
    n = 7
    rng = np.random.default_rng(3)
    gates, P = [], 6
    for i in range(40):
        t = int(rng.integers(0, n))
        others = [q for q in range(n) if q != t]
        c = int(rng.integers(0, 3))
        ctrls = tuple(int(q) for q in rng.choice(others, size=c, replace=False)) if c else ()
        vals = tuple(int(v) for v in rng.integers(0, 2, size=c))
        r = rng.random()
        if r < 0.5:
            gates.append(W.Gate(("RY", "RZ")[i % 2], t, ctrls, vals, param=int(rng.integers(0, P))))
        elif r < 0.7:
            gates.append(W.Gate("H", t, ctrls, vals))
        else:
            gates.append(W.Gate("~U", t, ctrls, vals, matrix=W.haar_unitary_2x2(i)))
    circ = W.Circuit(n, gates, rng.uniform(0, 2 * np.pi, size=P))
    terms = _rand_terms(n, 12, 9)
    ref = oracle.grad_param_shift(circ, circ.params, terms)
    _grad_check(gpu, circ, terms, ref)


def test_adjoint_rx_phase_and_adjoint_flags_vs_param_shift(gpu):
    """Every angle kind, uncontrolled and with up to two controls of mixed
    values: controlled RX and P and the adjoint-flagged rotations against the
    oracle's exact shift rules at 1e-8; central differences (h = 1e-5) as a
    second, looser check."""
    n = 6
    rng = np.random.default_rng(4)
    gates = []
    kinds = ("RX", "P", "~RY", "~RZ", "RZ", "~P", "~RX", "RY")
    for i in range(40):
        t = int(rng.integers(0, n))
        others = [q for q in range(n) if q != t]
        c = int(rng.integers(0, 3))
        ctrls = tuple(int(q) for q in rng.choice(others, size=c, replace=False)) if c else ()
        vals = tuple(int(v) for v in rng.integers(0, 2, size=c))
        gates.append(W.Gate(kinds[i % len(kinds)], t, ctrls, vals, param=i % 5))
        gates.append(W.Gate("H", int(rng.integers(0, n))))
    circ = W.Circuit(n, gates, rng.uniform(0, 2 * np.pi, size=5))
    terms = _rand_terms(n, 10, 5)
    ref = oracle.grad_param_shift(circ, circ.params, terms)
    err = _grad_check(gpu, circ, terms, ref, tol=1e-8)
    fd = oracle.grad_finite_diff(circ, circ.params, terms)
    assert np.max(np.abs(fd - ref)) <= 1e-7
    _say("all kinds: adjoint vs shift %.2e" % err)


def test_autograd_function(gpu):
    import torch
    n = 9
    c = W.hea(n, 2, seed=21)
    terms = W.zz_x_hamiltonian(n, 21)
    model = gpu.ExpectationModel(c, terms)
    p = torch.tensor(c.params, dtype=torch.float64, device="cuda", requires_grad=True)
    loss = model(p)
    (3.0 * loss).backward()
    ref = oracle.grad_param_shift(c, c.params, terms)
    assert abs(loss.item() - oracle.loss(c, c.params, terms)) <= 1e-12 * 20
    assert np.max(np.abs(p.grad.cpu().numpy() - 3.0 * ref)) <= 3e-8
    # a second backward through a fresh forward agrees bit for bit
    p2 = p.detach().clone().requires_grad_(True)
    model(p2).mul(3.0).backward()
    assert torch.equal(p.grad, p2.grad)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_adjoint_hea_n24_full_size(gpu):
    """The n=24 ansatz problem at full size (n=24, 16 layers, 768 parameters).
    (a) Loss and 32 seeded gradients (first, two middle and last layers, RY
    and RZ) against the oracle's parameter shift stored by
    tests/golden/make_hea_n24_grads.py, at 1e-8.  (b) All 768 gradients
    against a parameter shift evaluated on the GPU's forward path and
    sv_expect (both held to the oracle at 1e-12 elsewhere; they share no code
    with the reverse sweep), at 1e-8."""
    import torch
    c, terms = W.hea_problem_n24()
    with open(os.path.join(GOLDEN, "hea_n24_param_shift.json")) as fh:
        gold = json.load(fh)
    params = torch.from_numpy(c.params).cuda()
    psi = torch.empty(1 << c.n, dtype=torch.complex128, device="cuda")
    gpu.sv_init(psi, 0)
    gpu.sv_apply_circuit(psi, c, params=params)
    lam = torch.empty_like(psi)
    grad, loss = gpu.sv_adjoint_grad(psi, lam, c, params, terms)
    g = grad.cpu().numpy()
    _say("hea n24 loss %.15f (oracle %.15f)" % (loss.item(), gold["loss"]))
    assert abs(loss.item() - gold["loss"]) <= 1e-10
    idx = np.array(gold["params"])
    ref = np.array(gold["grad"])
    assert len(idx) == 32
    err = np.max(np.abs(g[idx] - ref)) / max(1.0, np.max(np.abs(ref)))
    _say("hea n24 golden grad err %.2e over %d parameters" % (err, len(idx)))
    assert err <= 1e-8
    # (b) every parameter: shifted angle sets, one forward pass + <H> each
    P = c.nparams
    shifts = np.repeat(c.params[None, :], 2 * P, axis=0)
    shifts[2 * np.arange(P), np.arange(P)] += np.pi / 2
    shifts[2 * np.arange(P) + 1, np.arange(P)] -= np.pi / 2
    sh = torch.from_numpy(shifts).cuda()
    losses = torch.empty(2 * P, dtype=torch.float64, device="cuda")
    plan = gpu.Circuit(c.n, c, nparams=P, flags=gpu.SV_FUSE)
    try:
        for r in range(2 * P):
            gpu.sv_init(psi, 0)
            plan.run(psi, sh[r])
            gpu.sv_expect(psi, terms, out=losses[r:r + 1])
        lv = losses.cpu().numpy()
    finally:
        plan.close()
    shift = 0.5 * (lv[0::2] - lv[1::2])
    err_all = np.max(np.abs(g - shift)) / max(1.0, np.max(np.abs(shift)))
    _say("hea n24 adjoint vs GPU parameter shift, all %d: %.2e" % (P, err_all))
    assert err_all <= 1e-8
    assert np.max(np.abs(shift[idx] - ref)) <= 1e-10


@pytest.mark.parametrize("tile,low", [(8, 3), (10, 5), (13, 6)])
def test_adjoint_fused_tiles(gpu, tile, low):
    """The fused reverse sweep under several tile shapes (small tiles force
    scattered qubit sets and many runs; 13 gives 128 KiB of LDS): gradients
    against the oracle's parameter shift, psi restored to |0>."""
    gpu.sv_tune_set("tile_log2_c128", tile)
    gpu.sv_tune_set("tile_low_bits_c128", low)
    try:
        n = 11
        rng = np.random.default_rng(tile)
        gates, P = [], 7
        for i in range(60):
            t = int(rng.integers(0, n))
            others = [q for q in range(n) if q != t]
            c = int(rng.integers(0, 3))
            ctrls = tuple(int(q) for q in rng.choice(others, size=c, replace=False)) if c else ()
            vals = tuple(int(v) for v in rng.integers(0, 2, size=c))
            kind = ("RY", "RZ", "H", "X", "RZ")[i % 5]
            p = int(rng.integers(0, P)) if kind in ("RY", "RZ") else -1
            gates.append(W.Gate(kind, t, ctrls, vals, 0.3, p))
        circ = W.Circuit(n, gates, rng.uniform(0, 2 * np.pi, size=P))
        terms = _rand_terms(n, 9, tile)
        ref = oracle.grad_param_shift(circ, circ.params, terms)
        _grad_check(gpu, circ, terms, ref)
    finally:
        gpu.sv_tune_set("tile_log2_c128", 12)
        gpu.sv_tune_set("tile_low_bits_c128", 6)


def test_adjoint_n32_product_state_closed_form(gpu):
    """The adjoint at n = 32 (64 GiB per state vector; the sweep holds the
    state and the co-state, no tape).  RY(theta_i) then RZ(phi_i) on every
    qubit leaves the product state with Bloch vectors
    (sin theta cos phi, sin theta sin phi, cos theta), so for
    H = sum a_i Z_i Z_{i+1} + sum b_i X_i the loss is
    sum a_i cos(theta_i) cos(theta_{i+1}) + sum b_i sin(theta_i) cos(phi_i),
    and every derivative has a closed form."""
    import torch
    n = 32
    rng = np.random.default_rng(56)
    gates = []
    for q in range(n):
        gates.append(W.Gate("RY", q, param=2 * q))
        gates.append(W.Gate("RZ", q, param=2 * q + 1))
    c = W.Circuit(n, gates, rng.uniform(0.0, 2 * np.pi, size=2 * n))
    terms = W.zz_x_hamiltonian(n, seed=56)
    a = np.array([t.coef for t in terms[:n - 1]])
    b = np.array([t.coef for t in terms[n - 1:]])
    th, ph = c.params[0::2], c.params[1::2]
    loss_ref = np.sum(a * np.cos(th[:-1]) * np.cos(th[1:])) + np.sum(b * np.sin(th) * np.cos(ph))
    g_th = b * np.cos(th) * np.cos(ph)
    g_th[1:] -= np.sin(th[1:]) * a * np.cos(th[:-1])
    g_th[:-1] -= np.sin(th[:-1]) * a * np.cos(th[1:])
    g_ph = -b * np.sin(th) * np.sin(ph)
    ref = np.empty(2 * n)
    ref[0::2], ref[1::2] = g_th, g_ph
    _say("adjoint n=32 (two 64 GiB vectors)")
    torch.cuda.empty_cache()
    err = None
    try:
        psi = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
        lam = torch.empty_like(psi)
        params = torch.from_numpy(c.params).cuda()
        gpu.sv_init(psi, 0)
        gpu.sv_apply_circuit(psi, c, params=params)
        grad, loss = gpu.sv_adjoint_grad(psi, lam, c, params, terms)
        g = grad.cpu().numpy()
        lv = loss.item()
        _say("adjoint n=32 loss %.12f (closed form %.12f), max grad err %.2e"
             % (lv, loss_ref, np.max(np.abs(g - ref))))
        if abs(lv - loss_ref) > 1e-10 or np.max(np.abs(g - ref)) > 1e-8 * max(1.0, np.max(np.abs(ref))):
            err = "loss %.3e off, gradient %.3e off" % (abs(lv - loss_ref), np.max(np.abs(g - ref)))
    finally:
        psi = lam = None
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    assert err is None, err


def test_adjoint_plan_matches_one_shot(gpu):
    """The planned adjoint (sv_adjoint_create / sv_adjoint_run) enqueues the
    same kernels as sv_adjoint_grad: gradients and loss bit-identical, over
    two runs with different angles, and against the oracle's shift rule."""
    import torch
    n = 10
    c = W.hea(n, 3, seed=31)
    terms = W.zz_x_hamiltonian(n, 31)
    plan = gpu.AdjointPlan(n, c, terms, c.nparams)
    fwd = gpu.Circuit(n, c, nparams=c.nparams, flags=gpu.SV_FUSE)
    rng = np.random.default_rng(32)
    try:
        for rep in range(2):
            p_host = rng.uniform(0, 2 * np.pi, size=c.nparams)
            params = torch.from_numpy(p_host).cuda()
            outs = []
            for use_plan in (True, False):
                psi = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
                gpu.sv_init(psi, 0)
                fwd.run(psi, params)
                lam = torch.empty_like(psi)
                if use_plan:
                    g, l = plan.run(psi, lam, params)
                else:
                    g, l = gpu.sv_adjoint_grad(psi, lam, c, params, terms)
                outs.append((g.cpu().numpy(), l.item()))
            assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1] == outs[1][1], rep
            cc = W.Circuit(n, c.gates, p_host)
            ref = oracle.grad_param_shift(cc, p_host, terms)
            assert np.max(np.abs(outs[0][0] - ref)) <= 1e-8 * max(1.0, np.max(np.abs(ref)))
    finally:
        plan.close()
        fwd.close()
