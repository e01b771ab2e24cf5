// Host-side construction of fused-tile descriptors: tile maps over a qubit
// set, per-gate tile descriptors (the in-tile index expansion of Sec. III-B at
// tile scope), the diagonal-sweep summaries and the coset pairs of a run.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "tile.hpp"

namespace sv {

TileMap make_tile_map(int n, int m, int a, const std::vector<int> &high, uint64_t fixed_mask, uint64_t fixed_vals) {
    TileMap tm;
    memset(&tm, 0, sizeof(tm));
    // high qubits that continue the low block extend it
    size_t h0 = 0;
    while (h0 < high.size() && high[h0] == a) {
        ++a;
        ++h0;
    }
    tm.m = (uint32_t)m;
    tm.a = (uint32_t)a;
    tm.nh = (uint32_t)(high.size() - h0);
    uint64_t S = 0;
    for (int q = 0; q < a; ++q)
        S |= 1ull << q;
    for (size_t i = h0; i < high.size(); ++i) {
        tm.hpos[i - h0] = (uint32_t)high[i];
        S |= 1ull << high[i];
    }
    // local bit a+i goes to hpos[i]; consecutive hpos form one shifted segment
    for (uint32_t i = 0; i < tm.nh;) {
        uint32_t e = i + 1;
        while (e < tm.nh && tm.hpos[e] == tm.hpos[e - 1] + 1)
            ++e;
        const uint32_t lo = (uint32_t)a + i, len = e - i;
        tm.seg_in[tm.nseg] = ((1u << len) - 1) << lo;
        tm.seg_shift[tm.nseg] = tm.hpos[i] - lo;
        tm.nseg++;
        i = e;
    }
    fixed_mask &= ~S;
    std::vector<int> pos, bits;  // S bits (0) and the fixed outer bits (their values)
    for (int q = 0; q < n; ++q) {
        if (S & (1ull << q)) {
            pos.push_back(q);
            bits.push_back(0);
        } else if (fixed_mask & (1ull << q)) {
            pos.push_back(q);
            bits.push_back((int)((fixed_vals >> q) & 1));
        }
    }
    tm.outer = make_expand(n, pos, bits);
    tm.ntiles = 1ull << (n - (int)pos.size());
    return tm;
}

TileMap contiguous_tile_map(int n, int m) { return make_tile_map(n, m, m, {}); }

void mark_diag_sweeps(TileGate *t, int count, const char *param_gate, int phase_min) {
    int k = 0;
    while (k < count) {
        if (!t[k].diag) {
            ++k;
            continue;
        }
        int e = k;
        bool unit = true;
        int nlocal = 0;
        while (e < count && t[e].diag && e - k < 0xffff) {
            unit &= param_gate[e] != 0 || t[e].unit != 0;
            nlocal += (t[e].l_target >= 0 || t[e].l_mask) ? 1 : 0;
            ++e;
        }
        t[k].sweep_len = (uint16_t)(e - k);
        t[k].sweep_phase = (unit && nlocal >= phase_min) ? 1 : 0;
        k = e;
    }
}

namespace {

// One phase of a sweep gate before grouping: its tile-local condition and
// its member record.
struct PhasePart {
    uint32_t lm, lv;
    SweepMember mem;
    int gate, slot;  // the gate (index in the run) and which of its phases
};

// Parts of diagonal gate d: ph[1] where its target bit is 1, ph[0] where it
// is 0; a phase known to be 0 adds nothing and is left out (a parameterised
// gate keeps both, its angle changes between runs).
int phase_parts(const TileGate &d, int q, bool param, PhasePart *out) {
    int np = 0;
    for (int s = 0; s < 2; ++s) {
        if (!param && d.ph[s] == 0.0)
            continue;
        PhasePart pt;
        pt.lm = d.l_mask;
        pt.lv = d.l_vals;
        pt.mem = SweepMember{d.o_mask, d.o_vals, d.ph[s], 0};
        if (d.l_target >= 0) {
            pt.lm |= 1u << d.l_target;
            pt.lv |= (uint32_t)s << d.l_target;
        } else {
            pt.mem.om |= 1ull << d.target;
            pt.mem.ov |= (uint64_t)s << d.target;
        }
        pt.gate = q;
        pt.slot = s;
        out[np++] = pt;
    }
    return np;
}

} // namespace

void build_sweep_patterns(TileGate *t, int count, int m, const char *param_gate, std::vector<SweepPat> &pats,
                          std::vector<SweepMember> &mems) {
    if (m < 7)
        return;  // no tables below 7 tile qubits
    const int Hb = m - 6;
    for (int k = 0; k < count;) {
        if (!t[k].diag) {
            ++k;
            continue;
        }
        int end = std::min(count, k + std::max(1, (int)t[k].sweep_len));
        if (!t[k].sweep_phase) {
            k = end;
            continue;
        }
        // the gates' phases, grouped by tile-local condition (first
        // appearance numbers the patterns); a sweep that would exceed
        // kSweepMaxPats patterns ends before the gate that would
        std::vector<PhasePart> parts;
        std::vector<std::pair<uint64_t, int>> keys;  // (lm << 32 | lv, pattern id), ordered by key
        auto find = [&](uint64_t key) -> int {
            auto it = std::lower_bound(keys.begin(), keys.end(), std::make_pair(key, -1));
            return (it != keys.end() && it->first == key) ? it->second : -1;
        };
        std::vector<int> part_pat;
        int q = k;
        for (; q < end; ++q) {
            PhasePart c[2];
            const int nc = phase_parts(t[q], q, param_gate[q] != 0, c);
            int add = 0;
            for (int i = 0; i < nc; ++i) {
                const uint64_t key = ((uint64_t)c[i].lm << 32) | c[i].lv;
                if (find(key) < 0 && !(i == 1 && nc == 2 && c[0].lm == c[1].lm && c[0].lv == c[1].lv))
                    ++add;
            }
            if (q > k && (int)keys.size() + add > kSweepMaxPats)
                break;
            for (int i = 0; i < nc; ++i) {
                const uint64_t key = ((uint64_t)c[i].lm << 32) | c[i].lv;
                int id = find(key);
                if (id < 0) {
                    id = (int)keys.size();
                    keys.insert(std::lower_bound(keys.begin(), keys.end(), std::make_pair(key, -1)),
                                std::make_pair(key, id));
                }
                parts.push_back(c[i]);
                part_pat.push_back(id);
            }
        }
        if (q < end) {  // split: [k, q) now, [q, end) as a sweep of its own
            t[q].sweep_len = (uint16_t)(end - q);
            t[q].sweep_phase = 1;
            t[k].sweep_len = (uint16_t)(q - k);
            end = q;
        }
        const int npat = (int)keys.size();
        std::vector<uint32_t> plm(npat), plv(npat);
        for (size_t i = 0; i < parts.size(); ++i) {
            plm[part_pat[i]] = parts[i].lm;
            plv[part_pat[i]] = parts[i].lv;
        }
        // classes: 0 = A (bits of u only, or none), 1 = B (bits of v only),
        // 2 + q = R[q] (bits of u and bit 6 + q), 2 + Hb = rest
        std::vector<int> cls(npat);
        bool have_r = false, rank1 = true, any_rest = false;
        uint32_t um = 0, uv = 0;
        for (int p = 0; p < npat; ++p) {
            const uint32_t lo = plm[p] & 63u, hi = plm[p] >> 6;
            if (!hi) {
                cls[p] = 0;
            } else if (!lo) {
                cls[p] = 1;
            } else if (__builtin_popcount(hi) == 1) {
                cls[p] = 2 + __builtin_ctz(hi);
                if (!have_r) {
                    um = lo;
                    uv = plv[p] & 63u;
                    have_r = true;
                } else if (lo != um || (plv[p] & 63u) != uv) {
                    rank1 = false;
                }
            } else {
                cls[p] = 2 + Hb;
                any_rest = true;
            }
        }
        if (have_r && rank1)  // one table D: every R pattern in class 2
            for (int p = 0; p < npat; ++p)
                if (cls[p] >= 2 && cls[p] < 2 + Hb)
                    cls[p] = 2;
        // emit patterns by class, then each pattern's members in gate order
        std::vector<int> order(npat);
        for (int p = 0; p < npat; ++p)
            order[p] = p;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cls[x] < cls[y]; });
        std::vector<std::vector<int>> members(npat);
        for (size_t i = 0; i < parts.size(); ++i)
            members[part_pat[i]].push_back((int)i);
        TileGate &h = t[k];
        h.pat0 = (uint32_t)pats.size();
        for (int c = 0; c < kSweepClassSlots; ++c)
            h.sweep_cls[c] = (uint32_t)npat;
        for (int r = npat - 1; r >= 0; --r)
            h.sweep_cls[cls[order[r]]] = (uint32_t)r;
        for (int c = kSweepClassSlots - 2; c >= 0; --c)  // empty classes start where the next one does
            h.sweep_cls[c] = std::min(h.sweep_cls[c], h.sweep_cls[c + 1]);
        for (int r = 0; r < npat; ++r) {
            const int p = order[r];
            pats.push_back(SweepPat{plm[p], plv[p], (uint32_t)mems.size(), (uint32_t)members[p].size()});
            for (int i : members[p]) {
                t[parts[i].gate].mem[parts[i].slot] = (int32_t)mems.size();
                mems.push_back(parts[i].mem);
            }
        }
        h.npairs = kSweepInfoValid | um | (uv << 8) | (have_r ? kSweepHaveR : 0u) |
                   (have_r && rank1 ? kSweepRank1 : 0u) | (any_rest ? kSweepAnyRest : 0u);
        k = end;
    }
}

void mark_permutation_runs(TileGate *t, int count) {
    auto is_x = [](const TileGate &g) {
        return !g.diag && g.m[0] == 0.0 && g.m[1] == 0.0 && g.m[2] == 1.0 && g.m[3] == 0.0 && g.m[4] == 1.0 &&
               g.m[5] == 0.0 && g.m[6] == 0.0 && g.m[7] == 0.0;
    };
    for (int k = 0; k < count;) {
        int e = k;
        double touched = 0.0;  // tiles' worth of amplitudes the run's gates move
        while (e < count && is_x(t[e]) && e - k < 0xffff) {
            touched += std::ldexp(1.0, -__builtin_popcount(t[e].l_mask));
            ++e;
        }
        if (e - k >= 2 && touched >= 1.5)
            t[k].perm_len = (uint32_t)(e - k);
        k = std::max(e, k + 1);
    }
}

void mark_coset_pairs(TileGate *t, int count) {
    for (int k = 0; k + 1 < count;) {
        TileGate &a = t[k], &b = t[k + 1];
        const bool ok = !a.diag && !b.diag && a.target != b.target &&
                        (a.l_mask & ~(1u << b.target)) == 0 && (b.l_mask & ~(1u << a.target)) == 0;
        if (ok) {
            a.sweep_len = 2;
            k += 2;
        } else {
            ++k;
        }
    }
}

// Tile-local bit of global qubit q, or -1 when q is outside S.
static int local_bit(const TileMap &tm, int q) {
    if (q < (int)tm.a)
        return q;
    for (uint32_t i = 0; i < tm.nh; ++i)
        if ((int)tm.hpos[i] == q)
            return (int)tm.a + (int)i;
    return -1;
}

TileGate make_tile_gate(const TileMap &tm, int target, uint64_t cmask, uint64_t cvals, const double *U,
                        bool diagonal) {
    TileGate g;
    memset(&g, 0, sizeof(g));
    for (int i = 0; i < 8; ++i)
        g.m[i] = U[i];
    g.mem[0] = g.mem[1] = -1;
    if (diagonal) {
        g.diag = 1;
        g.sweep_len = 1;  // a block of one unless a run marks a longer one
        diag_phases(g.m, g.ph, &g.unit);
        g.target = (uint32_t)target;  // global qubit
        g.hi_mask = cmask;            // every control, global bits
        g.hi_vals = cvals;
        g.l_target = local_bit(tm, target);
        for (int q = 0; q < 64; ++q) {
            if (!(cmask & (1ull << q)))
                continue;
            const int lq = local_bit(tm, q);
            if (lq >= 0) {
                g.l_mask |= 1u << lq;
                g.l_vals |= (uint32_t)((cvals >> q) & 1ull) << lq;
            } else {
                g.o_mask |= 1ull << q;
                g.o_vals |= cvals & (1ull << q);
            }
        }
        return g;
    }
    const int tl = local_bit(tm, target);
    g.target = (uint32_t)tl;
    g.l_target = tl;
    std::vector<std::pair<int, int>> loc;  // (local position, required bit)
    loc.push_back({tl, 0});
    int in_tile = 0;
    for (int q = 0; q < 64; ++q) {
        if (!(cmask & (1ull << q)))
            continue;
        const int lq = local_bit(tm, q);
        if (lq >= 0) {
            loc.push_back({lq, (int)((cvals >> q) & 1)});
            g.l_mask |= 1u << lq;
            g.l_vals |= (uint32_t)((cvals >> q) & 1ull) << lq;
            ++in_tile;
        } else {
            g.hi_mask |= 1ull << q;
            g.hi_vals |= cvals & (1ull << q);
        }
    }
    std::sort(loc.begin(), loc.end());
    std::vector<int> pos, bits;
    for (auto &pb : loc) {
        pos.push_back(pb.first);
        bits.push_back(pb.second);
    }
    const Expand e = make_expand((int)tm.m, pos, bits);
    g.nseg = e.nseg;
    for (uint32_t s = 0; s < e.nseg; ++s) {
        g.shift[s] = e.shift[s];
        g.mask[s] = (uint32_t)e.mask[s];
    }
    g.fixed = (uint32_t)e.fixed;
    g.npairs = 1u << ((int)tm.m - 1 - in_tile);
    return g;
}

} // namespace sv
