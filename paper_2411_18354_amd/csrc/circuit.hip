// Circuit driver: validation of a whole gate list, the fusion planner, the
// per-pass launch sequence and its HIP-graph capture.
//
// The paper applies a circuit as one kernel launch per gate, in order, since
// consecutive gates depend on each other (Sec. III-A).  Here every gate is
// still one pass unless it can join an LDS-fused run: gates whose target lies
// below the tile width m touch only amplitudes inside aligned 2^m-amplitude
// tiles, so a run of them is applied tile by tile with one HBM read and one
// HBM write per touched tile (gate fusion, future work in Sec. V).  A gate
// whose target is at or above m may be deferred past later fusable gates when
// the two commute (see commute() below), so runs are not cut by every
// unrelated high-target gate.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>

#include "circuit.hpp"
#include "gates.hpp"

namespace sv {

__global__ void k_param_mats(const ParamJob *__restrict__ jobs, int njobs, const double *__restrict__ params,
                             double *__restrict__ mats, TileGate *__restrict__ tiles, SweepMember *__restrict__ mems) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= njobs)
        return;
    const ParamJob j = jobs[i];
    double m[8];
    gate_matrix(j.kind, params[j.param], nullptr, m);
    for (int k = 0; k < 8; ++k)
        mats[8 * j.mat_slot + k] = m[k];
    if (j.tile_slot >= 0) {
        TileGate &t = tiles[j.tile_slot];
        for (int k = 0; k < 8; ++k)
            t.m[k] = m[k];
        if (t.diag) {
            diag_phases(m, t.ph, &t.unit);
            for (int s = 0; s < 2; ++s)  // the phase-sweep members holding ph
                if (t.mem[s] >= 0)
                    mems[t.mem[s]].theta = t.ph[s];
        }
    }
}

// Gates a and b commute when every qubit they share is, in each of them,
// either a control or the target of a diagonal gate: both are then block
// diagonal over the shared qubits and act on disjoint qubits inside each
// block.
static bool commute(const sv_gate_t &a, const sv_gate_t &b) {
    const uint64_t qa = a.ctrl_mask | (1ull << a.target);
    const uint64_t qb = b.ctrl_mask | (1ull << b.target);
    const uint64_t shared = qa & qb;
    if (!shared)
        return true;
    const bool da = gate_kind_diagonal(a.kind), db = gate_kind_diagonal(b.kind);
    if ((shared & (1ull << a.target)) && !da)
        return false;
    if ((shared & (1ull << b.target)) && !db)
        return false;
    return true;
}

int validate_unitary_gate(const sv_gate_t &g, int index) {
    if ((g.kind & ~SV_G_ADJOINT) != SV_G_MATRIX)
        return SV_OK;  // named kinds are unitary for every angle
    const double *u = g.U;
    // rows (a, b) and (c, d): |a|^2 + |b|^2 = 1, |c|^2 + |d|^2 = 1, a conj(c) + b conj(d) = 0
    const double r0 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2] + u[3] * u[3] - 1.0;
    const double r1 = u[4] * u[4] + u[5] * u[5] + u[6] * u[6] + u[7] * u[7] - 1.0;
    const double xr = u[0] * u[4] + u[1] * u[5] + u[2] * u[6] + u[3] * u[7];
    const double xi = u[1] * u[4] - u[0] * u[5] + u[3] * u[6] - u[2] * u[7];
    const double dev = std::max(std::max(std::fabs(r0), std::fabs(r1)), std::sqrt(xr * xr + xi * xi));
    if (!(dev <= 1e-12))
        return fail(SV_EINVAL, "gate %d: matrix is not unitary (|U U^dag - I| = %.3g); the adjoint sweep "
                               "un-applies each gate by its conjugate transpose", index, dev);
    return SV_OK;
}

int validate_circuit_gate(int n, int nparams, const sv_gate_t &g, int index) {
    if (!gate_kind_valid(g.kind))
        return fail(SV_EINVAL, "gate %d: unknown kind %d", index, g.kind);
    GateSpec gs{n, g.target, g.ctrl_mask, g.ctrl_vals};
    const int r = validate_gate(gs);
    if (r != SV_OK) {
        char msg[400];
        snprintf(msg, sizeof(msg), "%s", sv_last_error());
        return fail(r, "gate %d: %s", index, msg);
    }
    if (g.param >= 0) {
        if (!gate_kind_param(g.kind))
            return fail(SV_EINVAL, "gate %d: kind %d takes no parameter (param %d)", index, g.kind, g.param);
        if (g.param >= nparams)
            return fail(SV_EINVAL, "gate %d: param %d >= nparams %d", index, g.param, nparams);
    } else if (g.param != -1) {
        return fail(SV_EINVAL, "gate %d: param %d (use -1 for none)", index, g.param);
    }
    return SV_OK;
}

} // namespace sv

using namespace sv;

namespace sv {

// Diagonal for this gate's actual matrix (named diagonal kinds, or a
// fixed matrix with both off-diagonal entries exactly zero).
static bool gate_is_diagonal(const sv_gate_t &g, const double *mat) {
    if (gate_kind_diagonal(g.kind))
        return true;
    if (g.param >= 0)
        return false;
    return mat[2] == 0.0 && mat[3] == 0.0 && mat[4] == 0.0 && mat[5] == 0.0;
}

// Inside a fused run, gather diagonal gates into blocks.  First every
// diagonal gate moves later past the non-diagonal gates that follow it and
// commute with it, up to the next diagonal gate (scanning from the end, so
// moved gates collect).  Then a diagonal gate that can move earlier past the
// non-diagonal gates before it, all of which it commutes with, until it meets
// a diagonal gate, joins that block.  Gates only pass gates they commute
// with, so the run computes the same unitary; diagonal blocks grow (one sweep
// each) and pair gates become adjacent (coset pairs).  An ansatz layer
// RY(q) RZ(q) ... then CNOT(q -> q+1) ... becomes all RY, all RZ, the CNOTs.
static void group_diagonals(std::vector<int> &run, const std::vector<char> &diag,
                            const std::vector<sv_gate_t> &gates) {
    const int R = (int)run.size();
    for (int k = R - 2; k >= 0; --k) {
        if (!diag[run[k]])
            continue;
        for (int j = k; j + 1 < R && !diag[run[j + 1]] && commute(gates[run[j]], gates[run[j + 1]]); ++j)
            std::swap(run[j], run[j + 1]);
    }
    for (int k = 1; k < R; ++k) {
        if (!diag[run[k]] || diag[run[k - 1]])
            continue;
        int j = k;
        while (j - 1 >= 0 && !diag[run[j - 1]] && commute(gates[run[j - 1]], gates[run[k]]))
            --j;
        if (j - 1 >= 0 && diag[run[j - 1]])  // reached a block: join it
            std::rotate(run.begin() + j, run.begin() + k, run.begin() + k + 1);
    }
}

// Greedy fusion planner.
//  general: a run's tile spans the `a` lowest qubits plus up to m - a other
//    qubits picked as targets appear, and diagonal gates join any run;
//  otherwise (contiguous tiles) a gate joins when its target is below m.
// A gate that cannot join the open run is deferred; later gates may still
// join the run ahead of the deferred ones only if they commute with all of
// them.  When the run closes, the deferred gates start the next run, so the
// relative order of non-commuting gates is never changed.
// SV_REMAP: choose disjoint swaps (q, h) of a low qubit q, below the
// cache-line granule (where a scheduled skip saves no DRAM traffic, so its
// controls are tested instead), with a high qubit h, and relabel the gates.
// A control on q then sits on a high bit, where each control halves the
// traffic of an unfused gate.  The swaps cost two passes over the state
// (into the new layout and back), so a pair is taken when q controls at
// least four more gates than h.
static void apply_remap(sv_circuit *c) {
    const int n = c->n;
    const int gran = tuning().granule_bits[c->dtype == SV_C128 ? 0 : 1];
    std::vector<int> ctrl(n, 0);
    for (const sv_gate_t &g : c->gates)
        for (int q = 0; q < n; ++q)
            ctrl[q] += (int)((g.ctrl_mask >> q) & 1ull);
    std::vector<int> low, high;
    for (int q = 0; q < std::min(gran, n); ++q)
        low.push_back(q);
    for (int q = n - 1; q >= gran; --q)
        high.push_back(q);
    std::stable_sort(low.begin(), low.end(), [&](int a, int b) { return ctrl[a] > ctrl[b]; });
    std::stable_sort(high.begin(), high.end(), [&](int a, int b) { return ctrl[a] < ctrl[b]; });
    std::vector<int> perm(n);
    for (int q = 0; q < n; ++q)
        perm[q] = q;
    c->remap.clear();
    for (size_t i = 0; i < low.size() && i < high.size() && (int)c->remap.size() / 2 < kMaxSwapPairs; ++i) {
        const int q = low[i], h = high[i];
        if (ctrl[q] - ctrl[h] < 4)
            break;
        c->remap.push_back(q);
        c->remap.push_back(h);
        std::swap(perm[q], perm[h]);
    }
    if (c->remap.empty())
        return;
    for (sv_gate_t &g : c->gates) {
        g.target = perm[g.target];
        uint64_t m = 0, v = 0;
        for (int q = 0; q < n; ++q)
            if ((g.ctrl_mask >> q) & 1ull) {
                m |= 1ull << perm[q];
                v |= ((g.ctrl_vals >> q) & 1ull) << perm[q];
            }
        g.ctrl_mask = m;
        g.ctrl_vals = v;
    }
}

static int plan_circuit(sv_circuit *c, std::vector<TileGate> &tiles, std::vector<ParamJob> &jobs,
                        std::vector<double> &mats, std::vector<DenseGate> &dense_list, int &dense_runs,
                        std::vector<SweepPat> &pats, std::vector<SweepMember> &mems) {
    const int G = (int)c->gates.size();
    mats.assign((size_t)G * 8, 0.0);
    for (int i = 0; i < G; ++i) {
        const sv_gate_t &g = c->gates[i];
        if (g.param < 0)
            gate_matrix(g.kind, g.theta, g.U, &mats[(size_t)8 * i]);
    }
    // tiles hold the arithmetic type: fixed-point states decode 16-bit codes
    // to float (complex64 tiles) and 32-bit codes to double (complex128)
    const int tdt = tile_dtype(c->dtype);
    const int di = tdt == SV_C128 ? 0 : 1;
    const int phase_min = tuning().phase_sweep_min[di];
    const bool masked = c->flags & SV_MASKED;
    c->m = std::min(std::min(tuning().tile_log2[di], c->n), c->m_cap);
    const int m = c->m;
    // a fixed-point tile holds whole 64-amplitude blocks
    const bool fuse = (c->flags & SV_FUSE) && !masked && (!is_fixed(c->dtype) || m >= kQBlockBits);
    // the tile holds the a lowest qubits plus at most kTileMaxHigh others
    int a = std::max(std::min(tuning().tile_low_bits[di], m), m - kTileMaxHigh);
    if (is_fixed(c->dtype))
        a = std::min(std::max(a, kQBlockBits), m);
    const int min_run = std::max(1, tuning().fuse_min_gates);
    std::vector<int> tile_slot(G, -1);
    std::vector<char> diag(G, 0);
    for (int i = 0; i < G; ++i)
        diag[i] = gate_is_diagonal(c->gates[i], &mats[(size_t)8 * i]);

    auto single = [&](int i) -> int {
        Pass p;
        p.fused = false;
        p.gate = i;
        p.first = p.count = 0;
        const sv_gate_t &g = c->gates[i];
        GateSpec gs{c->n, g.target, g.ctrl_mask, g.ctrl_vals};
        if (is_fixed(c->dtype))
            SV_TRY(make_fixed_plan(gs, c->dtype, masked, &p.fx));
        else
            SV_TRY(make_gate_plan(gs, c->dtype, masked ? SV_MODE_MASKED : SV_MODE_AUTO, &p.plan));
        c->passes.push_back(p);
        return SV_OK;
    };
    // Gates a run starting at stream[pos] would take with the tile qubits
    // {0 .. a-1} u high, scanning at most `window` gates (a dry run of the
    // planner's scan below, with no qubits added on the way).
    auto run_size = [&](const std::vector<int> &stream, size_t pos, const std::vector<int> &high,
                        size_t window) -> int {
        std::vector<int> deferred;
        int taken = 0;
        const size_t end = std::min(stream.size(), pos + window);
        for (size_t i = pos; i < end; ++i) {
            const sv_gate_t &g = c->gates[stream[i]];
            const bool fits = diag[stream[i]] || g.target < a ||
                              std::find(high.begin(), high.end(), g.target) != high.end();
            bool free = true;
            for (int d : deferred)
                if (!commute(g, c->gates[d])) {
                    free = false;
                    break;
                }
            if (fits && free) {
                ++taken;
            } else if (taken > 0) {
                deferred.push_back(stream[i]);
                if (deferred.size() > 256)
                    break;
            } else {
                return 0;
            }
        }
        return taken;
    };
    // The high qubits of the next run, chosen one at a time: each step adds
    // the target (among the next gates') that lets the run take the most
    // gates.  Looking ahead this way keeps qubits whose gates come later in
    // the same run instead of filling the set with the first targets met.
    // depth 2: each of the six best targets is scored by the best run it
    // allows together with one more target, and the step takes the best of
    // those (a qubit whose gates pay off only with another one).
    auto choose_high = [&](const std::vector<int> &stream, size_t pos, int depth) -> std::vector<int> {
        constexpr size_t kWindow = 1024;
        std::vector<int> cand, high;
        for (size_t i = pos; i < std::min(stream.size(), pos + kWindow); ++i) {
            const sv_gate_t &g = c->gates[stream[i]];
            if (!diag[stream[i]] && g.target >= a && std::find(cand.begin(), cand.end(), g.target) == cand.end())
                cand.push_back(g.target);
        }
        std::sort(cand.begin(), cand.end());
        int cur = run_size(stream, pos, high, kWindow);
        while ((int)high.size() < m - a) {
            // score every candidate, then look one step further for the best few
            std::vector<std::pair<int, int>> sc;  // (gates taken, qubit)
            for (int q : cand) {
                if (std::find(high.begin(), high.end(), q) != high.end())
                    continue;
                std::vector<int> h2(high);
                h2.push_back(q);
                sc.push_back({run_size(stream, pos, h2, kWindow), q});
            }
            if (sc.empty())
                break;
            std::stable_sort(sc.begin(), sc.end(), [](const std::pair<int, int> &x, const std::pair<int, int> &y) {
                return x.first > y.first;
            });
            int best = -1, best_n = cur, best2 = -1;
            const size_t top = std::min<size_t>(sc.size(), depth > 1 ? 6 : 1);
            for (size_t t = 0; t < top; ++t) {
                int two = sc[t].first;
                if (depth > 1 && (int)high.size() + 2 <= m - a)
                    for (const auto &o : sc) {
                        if (o.second == sc[t].second)
                            continue;
                        std::vector<int> h3(high);
                        h3.push_back(sc[t].second);
                        h3.push_back(o.second);
                        two = std::max(two, run_size(stream, pos, h3, kWindow));
                    }
                if (two > best2 || (two == best2 && sc[t].first > best_n)) {
                    best2 = two;
                    best = sc[t].second;
                    best_n = sc[t].first;
                }
            }
            if (best < 0 || best2 <= cur)
                break;
            high.push_back(best);
            cur = best_n;
        }
        return high;
    };
    // fusion planner over one stream of gate indices
    auto fuse_stream = [&](std::vector<int> stream) -> int {
        std::vector<int> run, deferred, high;
        size_t pos = 0;
        while (pos < stream.size()) {
            run.clear();
            deferred.clear();
            high.clear();
            const int depth = std::min(tuning().plan_lookahead, c->max_lookahead);
            if (depth > 0)
                high = choose_high(stream, pos, depth);
            size_t i = pos;
            for (; i < stream.size(); ++i) {
                const int gi = stream[i];
                const sv_gate_t &g = c->gates[gi];
                bool fits = diag[gi] || g.target < a ||
                            std::find(high.begin(), high.end(), g.target) != high.end();
                const bool can_add_high = !fits && (int)high.size() < m - a;
                bool free = true;
                for (int d : deferred)
                    if (!commute(g, c->gates[d])) {
                        free = false;
                        break;
                    }
                if ((fits || can_add_high) && free) {
                    if (!fits)
                        high.push_back(g.target);
                    run.push_back(gi);
                } else if (run.empty()) {
                    // nothing is open (so nothing is deferred): a gate that
                    // cannot start a run is a pass of its own
                    SV_TRY(single(gi));
                } else {
                    deferred.push_back(gi);
                    if (deferred.size() > 256) {
                        ++i;
                        break;
                    }
                }
            }
            if ((int)run.size() >= min_run) {
                if (tuning().fuse_group)
                    group_diagonals(run, diag, c->gates);
                // fill the tile's qubit set up to m, preferring the lowest free qubits
                std::sort(high.begin(), high.end());
                for (int q = a; (int)high.size() < m - a && q < c->n; ++q)
                    if (std::find(high.begin(), high.end(), q) == high.end())
                        high.push_back(q);
                std::sort(high.begin(), high.end());
                Pass p;
                p.fused = true;
                p.gate = -1;
                p.first = (int)tiles.size();
                p.count = (int)run.size();
                // outer control bits shared (same value) by every gate of the run
                uint64_t S = (a >= 64) ? ~0ull : ((1ull << a) - 1);
                for (int q : high)
                    S |= 1ull << q;
                uint64_t fmask = ~0ull, fvals = 0;
                bool first = true;
                for (int gi : run) {
                    const sv_gate_t &g = c->gates[gi];
                    const uint64_t om = g.ctrl_mask & ~S, ov = g.ctrl_vals & ~S;
                    if (first) {
                        fmask = om;
                        fvals = ov;
                        first = false;
                    } else {
                        fmask &= om & ~(fvals ^ ov);
                    }
                }
                fvals &= fmask;
                p.tm = make_tile_map(c->n, m, a, high, fmask, fvals);
                std::vector<char> from_param;
                for (int gi : run) {
                    const sv_gate_t &g = c->gates[gi];
                    tile_slot[gi] = (int)tiles.size();
                    tiles.push_back(
                        make_tile_gate(p.tm, g.target, g.ctrl_mask, g.ctrl_vals, &mats[(size_t)8 * gi], diag[gi]));
                    tiles.back().src_gate = gi;
                    c->tile_src.push_back(gi);
                    from_param.push_back(g.param >= 0);
                }
                // Short diagonal blocks are not worth a sweep over the whole
                // tile: their gates with the target in S run as pair gates,
                // whose tile-local controls are then scheduled, not tested.
                // A block of at least phase_min gates reading tile-local bits
                // is one sweep (phases added through the tables).  Measured on
                // MI355X, complex128 tiles: 4 against 8 gives QFT29 42.3 ->
                // 41.4 ms, the n=24 ansatz forward 10.6 -> 9.8 ms, a random
                // 400-gate n=28 circuit 62.3 -> 61.1 ms, and below 4 is slower
                // (a sweep costs about three pair gates); complex64 tiles are
                // better at 8 (4096-circuit batch 69.6 against 72.3 ms).
                for (int k = p.first, end = p.first + p.count; k < end;) {
                    if (!tiles[k].diag) {
                        ++k;
                        continue;
                    }
                    int e = k, nlocal = 0;
                    for (; e < end && tiles[e].diag; ++e)
                        nlocal += (tiles[e].l_target >= 0 || tiles[e].l_mask) ? 1 : 0;
                    if (nlocal < phase_min)
                        for (int q = k; q < e; ++q)
                            if (tiles[q].l_target >= 0) {
                                const int gi = tiles[q].src_gate;
                                const sv_gate_t &g = c->gates[gi];
                                tiles[q] = make_tile_gate(p.tm, g.target, g.ctrl_mask, g.ctrl_vals,
                                                          &mats[(size_t)8 * gi], false);
                                tiles[q].src_gate = gi;
                            }
                    k = e;
                }
                mark_diag_sweeps(&tiles[p.first], p.count, from_param.data(), phase_min);
                build_sweep_patterns(&tiles[p.first], p.count, (int)p.tm.m, from_param.data(), pats, mems);
                if (tuning().fuse_pairs)
                    mark_coset_pairs(&tiles[p.first], p.count);
                if (tuning().fuse_perm)  // checked first by the tile loops
                    mark_permutation_runs(&tiles[p.first], p.count);
                c->passes.push_back(p);
                c->fused_gates += (int64_t)run.size();
                c->fused_runs++;
            } else {
                for (int gi : run)
                    SV_TRY(single(gi));
            }
            // the deferred gates, then the unscanned rest, form the next stream
            std::vector<int> next(deferred);
            next.insert(next.end(), stream.begin() + (long)i, stream.end());
            stream.swap(next);
            pos = 0;
        }
        return SV_OK;
    };
    const int dk = tuning().dense_qubits;
    const bool dense = fuse && (c->flags & SV_DENSE) && dense_supported(c->dtype, dk, c->n);
    if (!fuse) {
        for (int i = 0; i < G; ++i)
            SV_TRY(single(i));
    } else if (!dense) {
        std::vector<int> all(G);
        for (int i = 0; i < G; ++i)
            all[i] = i;
        SV_TRY(fuse_stream(all));
    } else {
        // maximal stretches of gates acting only on qubits 0 .. dk-1 become
        // dense passes when long enough; the rest is fused as usual
        c->dense_k = dk;
        const uint64_t low = (1ull << dk) - 1;
        std::vector<int> pending;
        int i = 0;
        while (i < G) {
            int j = i;
            while (j < G && (((c->gates[j].ctrl_mask | (1ull << c->gates[j].target)) & ~low) == 0))
                ++j;
            if (j - i >= std::max(1, tuning().dense_min_gates)) {
                SV_TRY(fuse_stream(pending));
                pending.clear();
                Pass p;
                p.fused = false;
                p.dense = true;
                p.first = (int)dense_list.size();
                p.count = j - i;
                for (int q = i; q < j; ++q) {
                    const sv_gate_t &g = c->gates[q];
                    dense_list.push_back(DenseGate{g.target, q, g.ctrl_mask, g.ctrl_vals});
                }
                p.gate = dense_runs++;
                c->passes.push_back(p);
                i = j;
            } else {
                for (int q = i; q < std::max(j, i + 1); ++q)
                    pending.push_back(q);
                i = std::max(j, i + 1);
            }
        }
        SV_TRY(fuse_stream(pending));
    }
    for (int i = 0; i < G; ++i) {
        const sv_gate_t &g = c->gates[i];
        if (g.param >= 0)
            jobs.push_back(ParamJob{g.kind, g.param, i, tile_slot[i]});
    }
    c->njobs = (int)jobs.size();
    return SV_OK;
}

static void free_buffers(sv_circuit *c, hipStream_t st) {
    void *bufs[7] = {c->d_mats, c->d_tiles, c->d_jobs, c->d_dense, c->d_rmat, c->d_pats, c->d_mems};
    for (void *b : bufs)
        if (b) {
            if (c->async_buffers)
                (void)hipFreeAsync(b, st);
            else
                (void)hipFree(b);
        }
    c->d_mats = nullptr;
    c->d_tiles = nullptr;
    c->d_jobs = nullptr;
    c->d_dense = nullptr;
    c->d_rmat = nullptr;
    c->d_pats = nullptr;
    c->d_mems = nullptr;
}

template <typename T> static int upload(T **dst, const std::vector<T> &src, bool async, hipStream_t st) {
    *dst = nullptr;
    if (src.empty())
        return SV_OK;
    const size_t bytes = src.size() * sizeof(T);
    hipError_t e = async ? hipMallocAsync((void **)dst, bytes, st) : hipMalloc((void **)dst, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *dst = nullptr;
        return fail(SV_ENOMEM, "device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    }
    if (async)
        SV_HIP_TRY(hipMemcpyAsync(*dst, src.data(), bytes, hipMemcpyHostToDevice, st));
    else
        SV_HIP_TRY(hipMemcpy(*dst, src.data(), bytes, hipMemcpyHostToDevice));
    return SV_OK;
}

// Dynamic LDS of a fused pass: the tile (in the arithmetic type), then the
// diagonal-sweep tables.
static size_t fused_lds(int m, int dtype) {
    return ((size_t)1 << m) * amp_bytes(tile_dtype(dtype)) +
           (size_t)diag_table_doubles((uint32_t)m) * sizeof(double);
}

// One fused pass: one workgroup per launched tile.
template <typename R>
static int launch_tile_pass(cplx_t<R> *psi, const TileMap &tm_in, const DeviceGates &dg, size_t lds,
                            hipStream_t st) {
    TileMap tm = tm_in;
    tm.tab = 1;  // lds includes the tables
    for (uint64_t t0 = 0; t0 < tm.ntiles; t0 += kMaxGridBlocks) {
        tm.tile0 = t0;
        const dim3 grid((unsigned)std::min(kMaxGridBlocks, tm_in.ntiles - t0));
        hipLaunchKernelGGL((k_tile<R, 512, DeviceGates>), grid, dim3(512), lds, st, psi, tm, dg);
        SV_LAUNCH_CHECK();
    }
    return SV_OK;
}

int circuit_create(int n, int dtype, const sv_gate_t *gates, int ngates, int nparams, int flags, bool async,
                   hipStream_t st, int m_cap, sv_circuit **out) {
    *out = nullptr;
    if (!known_dtype(dtype))
        return fail(SV_EINVAL, "unknown dtype %d", dtype);
    if (n < 1 || n > max_qubits(dtype))
        return fail(SV_EINVAL, "n=%d outside [1, %d]", n, max_qubits(dtype));
    if (ngates < 0 || (ngates > 0 && !gates))
        return fail(SV_EINVAL, "bad gate list (ngates %d, gates %p)", ngates, (const void *)gates);
    if (nparams < 0)
        return fail(SV_EINVAL, "nparams %d < 0", nparams);
    if (flags & ~(SV_FUSE | SV_GRAPH | SV_MASKED | SV_DENSE | SV_REMAP))
        return fail(SV_EINVAL, "unknown flags 0x%x", flags);
    if (is_fixed(dtype) && (flags & (SV_DENSE | SV_REMAP)))
        return fail(SV_ENOTSUP, "fixed-point (SV_CQ16, SV_CQ32) circuits take SV_FUSE, SV_GRAPH and SV_MASKED only "
                                "(flags 0x%x)", flags);
    for (int i = 0; i < ngates; ++i)
        SV_TRY(validate_circuit_gate(n, nparams, gates[i], i));
    std::unique_ptr<sv_circuit> c(new sv_circuit());
    c->n = n;
    c->dtype = dtype;
    c->flags = flags;
    c->nparams = nparams;
    c->async_buffers = async;
    c->m_cap = m_cap;
    // a one-shot plan (stream-ordered buffers, run once) keeps planning cheap:
    // the two-step lookahead pays for itself only over repeated runs
    c->max_lookahead = async ? 1 : 2;
    SV_HIP_TRY(hipGetDevice(&c->device));
    c->gates.assign(gates, gates + ngates);
    if ((flags & SV_REMAP) && !(flags & SV_MASKED))
        apply_remap(c.get());
    std::vector<TileGate> tiles;
    std::vector<ParamJob> jobs;
    std::vector<double> mats;
    std::vector<DenseGate> dense_list;
    std::vector<SweepPat> pats;
    std::vector<SweepMember> mems;
    int dense_runs = 0;
    SV_TRY(plan_circuit(c.get(), tiles, jobs, mats, dense_list, dense_runs, pats, mems));
    int r = upload(&c->d_mats, mats, async, st);
    if (r == SV_OK)
        r = upload(&c->d_pats, pats, async, st);
    if (r == SV_OK)
        r = upload(&c->d_mems, mems, async, st);
    if (r == SV_OK)
        r = upload(&c->d_tiles, tiles, async, st);
    if (r == SV_OK)
        r = upload(&c->d_jobs, jobs, async, st);
    if (r == SV_OK)
        r = upload((DenseGate **)&c->d_dense, dense_list, async, st);
    if (r == SV_OK && dense_runs > 0) {
        const size_t D = (size_t)2 << c->dense_k;
        std::vector<double> zeros(D * D * (size_t)dense_runs, 0.0);  // room for either precision
        r = upload((double **)&c->d_rmat, zeros, async, st);
    }
    if (r != SV_OK) {
        free_buffers(c.get(), st);
        return r;
    }
    // large LDS tiles need the per-kernel limit raised before any launch
    const size_t lds = fused_lds(c->m, dtype);
    if (lds > 65536 && is_fixed(dtype)) {
        SV_TRY(fixed_tile_lds_limit(dtype, lds));
    } else if (lds > 65536) {
        if (dtype == SV_C128)
            SV_HIP_TRY(hipFuncSetAttribute((const void *)k_tile<double, 512, DeviceGates>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        else
            SV_HIP_TRY(hipFuncSetAttribute((const void *)k_tile<float, 512, DeviceGates>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    }
    *out = c.release();
    return SV_OK;
}

int circuit_param_mats(sv_circuit *c, const double *params, hipStream_t st) {
    if (c->njobs > 0) {
        hipLaunchKernelGGL(k_param_mats, dim3((c->njobs + 127) / 128), dim3(128), 0, st, c->d_jobs, c->njobs,
                           params, c->d_mats, c->d_tiles, c->d_mems);
        SV_LAUNCH_CHECK();
    }
    return SV_OK;
}

void circuit_free(sv_circuit *c, hipStream_t st) {
    if (!c)
        return;
    free_buffers(c, st);
    delete c;
}

template <typename R> static int enqueue(sv_circuit *c, cplx_t<R> *psi, const double *params, hipStream_t st) {
    SV_TRY(circuit_param_mats(c, params, st));
    const int nsw = (int)(c->remap.size() / 2);
    SV_TRY(launch_swap_qubits(c->dtype, psi, c->n, c->remap.data(), nsw, st));  // into the remapped layout
    const size_t lds = fused_lds(c->m, c->dtype);
    for (const Pass &p : c->passes) {
        if (p.dense) {
            const size_t D = (size_t)2 << c->dense_k;
            void *rm = (char *)c->d_rmat + D * D * sizeof(R) * (size_t)p.gate;
            SV_TRY(launch_dense_compose(c->dtype, (const DenseGate *)c->d_dense + p.first, p.count, c->d_mats,
                                        c->dense_k, rm, st));
            SV_TRY(launch_dense(c->dtype, psi, c->n, c->dense_k, rm, st));
        } else if (p.fused) {
            DeviceGates dg{c->d_tiles + p.first, p.count, c->d_pats, c->d_mems};
            SV_TRY(launch_tile_pass<R>(psi, p.tm, dg, lds, st));
        } else {
            SV_TRY(launch_plan<R>(psi, p.plan, MatPtr<R>{c->d_mats + (size_t)8 * p.gate}, st));
        }
    }
    // back to the caller's layout (the swaps are an involution)
    SV_TRY(launch_swap_qubits(c->dtype, psi, c->n, c->remap.data(), nsw, st));
    return SV_OK;
}

// Fixed-point state: fused runs decode, run and re-encode tiles; other gates
// run the block-scaled gate kernel, matrices from the plan's device table
// (parameterised ones written there first).
static int enqueue_fixed(sv_circuit *c, void *state, const double *params, hipStream_t st) {
    SV_TRY(circuit_param_mats(c, params, st));
    const size_t lds = fused_lds(c->m, c->dtype);
    for (const Pass &p : c->passes) {
        if (p.fused) {
            DeviceGates dg{c->d_tiles + p.first, p.count, c->d_pats, c->d_mems};
            SV_TRY(launch_fixed_tile_pass(state, c->n, c->dtype, p.tm, dg, lds, st));
        } else {
            SV_TRY(launch_fixed_gate(state, p.fx, nullptr, c->d_mats + (size_t)8 * p.gate, st));
        }
    }
    return SV_OK;
}

static int enqueue_any(sv_circuit *c, const sv_state_t *s, const double *params, hipStream_t st) {
    if (is_fixed(c->dtype))
        return enqueue_fixed(c, s->data, params, st);
    if (c->dtype == SV_C128)
        return enqueue<double>(c, reinterpret_cast<double2 *>(s->data), params, st);
    return enqueue<float>(c, reinterpret_cast<float2 *>(s->data), params, st);
}

static int check_run_args(sv_circuit *c, const sv_state_t *s, const double *params) {
    if (!c)
        return fail(SV_EINVAL, "circuit is NULL");
    SV_TRY(validate_state(s, true));
    if (s->n != c->n || s->dtype != c->dtype)
        return fail(SV_EINVAL, "state (n=%d, dtype=%d) does not match the circuit (n=%d, dtype=%d)", s->n, s->dtype,
                    c->n, c->dtype);
    if (c->njobs > 0 && !params)
        return fail(SV_EINVAL, "circuit has parameterised gates but params_dev is NULL");
    return SV_OK;
}

static void drop_graph(sv_circuit *c) {
    if (c->exec)
        (void)hipGraphExecDestroy(c->exec);
    if (c->graph)
        (void)hipGraphDestroy(c->graph);
    c->exec = nullptr;
    c->graph = nullptr;
}

static int run_graph(sv_circuit *c, const sv_state_t *s, const double *params, hipStream_t st) {
    if (c->passes.empty())
        return SV_OK;  // nothing to capture
    if (!c->exec || c->g_data != s->data || c->g_params != params) {
        drop_graph(c);
        if (!c->cap)
            SV_HIP_TRY(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
        SV_HIP_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed));
        const int r = enqueue_any(c, s, params, c->cap);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(c->cap, &g);
        if (r != SV_OK) {
            if (g)
                (void)hipGraphDestroy(g);
            return r;
        }
        if (e != hipSuccess)
            return fail(SV_EHIP, "graph capture failed: %s", hipGetErrorString(e));
        c->graph = g;
        SV_HIP_TRY(hipGraphInstantiate(&c->exec, c->graph, nullptr, nullptr, 0));
        c->g_data = s->data;
        c->g_params = params;
    }
    SV_HIP_TRY(hipGraphLaunch(c->exec, st));
    return SV_OK;
}

static int circuit_plan_order(int n, int dtype, const sv_gate_t *gates, int ngates, int nparams, int flags,
                              int32_t *order, int32_t *pass_of, int64_t *npasses);

} // namespace sv

extern "C" {

int sv_gate_matrix(int kind, double theta, const double *U, double *out) {
    clear_error();
    if (!gate_kind_valid(kind))
        return fail(SV_EINVAL, "unknown kind %d", kind);
    if (!out)
        return fail(SV_EINVAL, "out is NULL");
    if ((kind & ~SV_G_ADJOINT) == SV_G_MATRIX && !U)
        return fail(SV_EINVAL, "SV_G_MATRIX needs U");
    gate_matrix(kind, theta, U, out);
    return SV_OK;
}

int sv_circuit_plan(int n, int dtype, const sv_gate_t *gates, int ngates, int nparams, int flags, int32_t *order,
                    int32_t *pass_of, int64_t *npasses) {
    clear_error();
    return circuit_plan_order(n, dtype, gates, ngates, nparams, flags, order, pass_of, npasses);
}

} // extern "C"

namespace sv {

int circuit_plan_tiles(int n, int dtype, const sv_gate_t *gates, int ngates, int nparams, int m_cap,
                       std::vector<PlanPass> *passes, std::vector<TileGate> *tiles, int *m_used,
                       std::vector<SweepPat> *pats, std::vector<SweepMember> *mems) {
    if (dtype != SV_C128 && dtype != SV_C64)
        return fail(SV_EINVAL, "unknown dtype %d", dtype);
    if (n < 1 || n > max_qubits(dtype))
        return fail(SV_EINVAL, "n=%d outside [1, %d]", n, max_qubits(dtype));
    if (ngates < 0 || (ngates > 0 && !gates))
        return fail(SV_EINVAL, "bad gate list (ngates %d, gates %p)", ngates, (const void *)gates);
    for (int i = 0; i < ngates; ++i)
        SV_TRY(validate_circuit_gate(n, nparams, gates[i], i));
    sv_circuit c;
    c.n = n;
    c.dtype = dtype;
    c.flags = SV_FUSE;
    c.nparams = nparams;
    c.m_cap = m_cap;
    c.max_lookahead = 1;  // thousands of circuits: the one-step lookahead keeps planning cheap
    c.gates.assign(gates, gates + ngates);
    std::vector<ParamJob> jobs;
    std::vector<double> mats;
    std::vector<DenseGate> dense_list;
    int dense_runs = 0;
    std::vector<SweepPat> pv;
    std::vector<SweepMember> mv;
    tiles->clear();
    SV_TRY(plan_circuit(&c, *tiles, jobs, mats, dense_list, dense_runs, pv, mv));
    if (pats)
        pats->swap(pv);
    if (mems)
        mems->swap(mv);
    passes->clear();
    for (const Pass &p : c.passes) {
        PlanPass q;
        memset(&q, 0, sizeof(q));
        q.fused = p.fused ? 1 : 0;
        q.gate = p.fused ? -1 : p.gate;
        q.first = p.fused ? p.first : 0;
        q.count = p.fused ? p.count : 1;
        if (p.fused)
            q.tm = p.tm;
        passes->push_back(q);
    }
    if (m_used)
        *m_used = c.m;
    return SV_OK;
}

// The planned order of a circuit's gates and the pass of each (host dry run).
static int circuit_plan_order(int n, int dtype, const sv_gate_t *gates, int ngates, int nparams, int flags,
                              int32_t *order, int32_t *pass_of, int64_t *npasses) {
    if (dtype != SV_C128 && dtype != SV_C64)
        return fail(SV_EINVAL, "unknown dtype %d", dtype);
    if (n < 1 || n > max_qubits(dtype))
        return fail(SV_EINVAL, "n=%d outside [1, %d]", n, max_qubits(dtype));
    if (ngates < 0 || (ngates > 0 && !gates))
        return fail(SV_EINVAL, "bad gate list (ngates %d, gates %p)", ngates, (const void *)gates);
    if (flags & ~(SV_FUSE | SV_GRAPH | SV_MASKED | SV_DENSE | SV_REMAP))
        return fail(SV_EINVAL, "unknown flags 0x%x", flags);
    for (int i = 0; i < ngates; ++i)
        SV_TRY(validate_circuit_gate(n, nparams, gates[i], i));
    sv_circuit c;
    c.n = n;
    c.dtype = dtype;
    c.flags = flags;
    c.nparams = nparams;
    c.gates.assign(gates, gates + ngates);
    if ((flags & SV_REMAP) && !(flags & SV_MASKED))
        apply_remap(&c);
    std::vector<TileGate> tiles;
    std::vector<ParamJob> jobs;
    std::vector<double> mats;
    std::vector<DenseGate> dense_list;
    int dense_runs = 0;
    std::vector<SweepPat> pats;
    std::vector<SweepMember> mems;
    SV_TRY(plan_circuit(&c, tiles, jobs, mats, dense_list, dense_runs, pats, mems));
    int k = 0;
    for (size_t pi = 0; pi < c.passes.size(); ++pi) {
        const Pass &p = c.passes[pi];
        if (p.dense) {
            for (int j = 0; j < p.count; ++j) {
                if (order)
                    order[k] = dense_list[p.first + j].mat;
                if (pass_of)
                    pass_of[k] = (int32_t)pi;
                ++k;
            }
        } else if (!p.fused) {
            if (order)
                order[k] = p.gate;
            if (pass_of)
                pass_of[k] = (int32_t)pi;
            ++k;
        } else {
            for (int j = 0; j < p.count; ++j) {
                if (order)
                    order[k] = tiles[p.first + j].src_gate;
                if (pass_of)
                    pass_of[k] = (int32_t)pi;
                ++k;
            }
        }
    }
    if (npasses)
        *npasses = (int64_t)c.passes.size() + (c.remap.empty() ? 0 : 2);
    return SV_OK;
}

} // namespace sv

extern "C" {

int sv_circuit_create(int n, int dtype, const sv_gate_t *gates, int ngates, int nparams, int flags,
                      sv_circuit_t **out) {
    clear_error();
    if (!out)
        return fail(SV_EINVAL, "out is NULL");
    return circuit_create(n, dtype, gates, ngates, nparams, flags, false, nullptr, 64, out);
}

int sv_circuit_run(sv_circuit_t *c, const sv_state_t *s, const double *params_dev, sv_stream_t st) {
    clear_error();
    SV_TRY(check_run_args(c, s, params_dev));
    int dev = 0;
    SV_HIP_TRY(hipGetDevice(&dev));
    if (dev != c->device)
        return fail(SV_EINVAL, "circuit was created on device %d, current device is %d", c->device, dev);
    int r;
    if (c->flags & SV_GRAPH)
        r = run_graph(c, s, params_dev, (hipStream_t)st);
    else
        r = enqueue_any(c, s, params_dev, (hipStream_t)st);
    if (r != SV_OK)
        return r;
    if (!c->done)
        SV_HIP_TRY(hipEventCreateWithFlags(&c->done, hipEventDisableTiming));
    SV_HIP_TRY(hipEventRecord(c->done, (hipStream_t)st));
    return SV_OK;
}

int sv_circuit_info(const sv_circuit_t *c, int64_t *passes, int64_t *fused_gates, int64_t *fused_runs) {
    clear_error();
    if (!c)
        return fail(SV_EINVAL, "circuit is NULL");
    if (passes)
        *passes = (int64_t)c->passes.size() + (c->remap.empty() ? 0 : 2);
    if (fused_gates)
        *fused_gates = c->fused_gates;
    if (fused_runs)
        *fused_runs = c->fused_runs;
    return SV_OK;
}

int sv_circuit_destroy(sv_circuit_t *c) {
    clear_error();
    if (!c)
        return SV_OK;
    if (c->done)
        (void)hipEventSynchronize(c->done);
    drop_graph(c);
    free_buffers(c, nullptr);
    if (c->cap)
        (void)hipStreamDestroy(c->cap);
    if (c->done)
        (void)hipEventDestroy(c->done);
    delete c;
    return SV_OK;
}

int sv_apply_circuit(const sv_state_t *s, const sv_gate_t *gates, int ngates, const double *params_dev, int nparams,
                     int flags, sv_stream_t st) {
    clear_error();
    SV_TRY(validate_state(s, true));
    sv_circuit *c = nullptr;
    SV_TRY(circuit_create(s->n, s->dtype, gates, ngates, nparams, flags & ~SV_GRAPH, true, (hipStream_t)st, 64, &c));
    int r = check_run_args(c, s, params_dev);
    if (r == SV_OK)
        r = enqueue_any(c, s, params_dev, (hipStream_t)st);
    free_buffers(c, (hipStream_t)st);  // stream-ordered: after the kernels above
    delete c;
    return r;
}

} // extern "C"
