// Host-side construction of fused-tile descriptors: tile maps over a qubit
// set, per-gate tile descriptors (the in-tile index expansion of Sec. III-B at
// tile scope), the diagonal-sweep summaries and the coset pairs of a run.
#include <algorithm>
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

// What the phase tables of a sweep need to know about its gates, the same
// for every tile (the first gate's npairs, unused by diagonal gates; see
// diag_sweep_tables): whether gates reading bits of u and one bit of v
// exist (R-type) and all depend on u through one condition (u & um) == uv,
// and whether gates reading bits of u and two or more bits of v exist.  A
// target bit in u counts as a required 1 only when the phase on its 0 side
// is known to be 0 (not a parameterised gate).
static uint32_t sweep_table_info(const TileGate *t, int count, const char *param_gate) {
    bool have_r = false, rank1 = true, any_rest = false;
    uint32_t um = 0, uv = 0;
    for (int q = 0; q < count; ++q) {
        const TileGate &d = t[q];
        const uint32_t lm = d.l_mask | (d.l_target >= 0 ? 1u << d.l_target : 0u);
        const uint32_t lo = lm & 63u, hi = lm >> 6;
        if (!lo || !hi)
            continue;
        if (__builtin_popcount(hi) > 1) {
            any_rest = true;
            continue;
        }
        uint32_t gm = d.l_mask & 63u, gv = d.l_vals & 63u;
        if (d.l_target >= 0 && d.l_target < 6) {
            if (param_gate[q] || d.ph[0] != 0.0)
                rank1 = false;
            gm |= 1u << d.l_target;
            gv |= 1u << d.l_target;
        }
        if (!have_r) {
            um = gm;
            uv = gv;
            have_r = true;
        } else if (gm != um || gv != uv) {
            rank1 = false;
        }
    }
    return kSweepInfoValid | um | (uv << 8) | (have_r ? kSweepHaveR : 0u) | (have_r && rank1 ? kSweepRank1 : 0u) |
           (any_rest ? kSweepAnyRest : 0u);
}

void mark_diag_sweeps(TileGate *t, int count, const char *param_gate) {
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
        t[k].sweep_phase = (unit && nlocal >= kPhaseSweepMin) ? 1 : 0;
        t[k].npairs = sweep_table_info(t + k, e - k, param_gate + k);
        k = e;
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
