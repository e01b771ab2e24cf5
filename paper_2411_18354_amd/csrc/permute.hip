// Qubit exchange: relabel the state's qubits by a set of disjoint swaps
// (a_i, b_i).  The amplitude at index k moves to the index with bits a_i and
// b_i exchanged, for every pair at once.  Used to move qubits to other bit
// positions, e.g. a heavily used control from a low bit (where skipping
// pairs saves no DRAM traffic) to a high one (SV_REMAP).
//
// The exchange runs over LDS tiles whose qubit set holds every swapped qubit
// plus a low block of contiguous qubits: a tile is read in contiguous runs,
// permuted inside LDS (each orbit {j, j'} handled by the lane with the
// smaller index), and written back in the same runs.  Reading the partner
// amplitude of every index straight from memory would instead touch one
// 16-byte amplitude per 128-byte line on one side whenever a low qubit is
// exchanged with a high one.
#include <algorithm>
#include <cstring>

#include "circuit.hpp"

namespace sv {

constexpr int kPermThreads = 512;
constexpr int kPermPairsPerPass = 4;  // 8 qubits: the tile's high slots

struct LocalSwaps {
    uint32_t np;
    uint32_t la[kPermPairsPerPass], lb[kPermPairsPerPass];  // single-bit tile-local masks
};

template <typename R>
__global__ __launch_bounds__(kPermThreads) void k_permute_tile(cplx_t<R> *__restrict__ psi, TileMap tm,
                                                               LocalSwaps sw) {
    extern __shared__ unsigned char lds_raw[];
    cplx_t<R> *tile = reinterpret_cast<cplx_t<R> *>(lds_raw);
    const uint32_t T = 1u << tm.m;
    const uint64_t base = expand_index<uint64_t>(tm.outer, tm.tile0 + blockIdx.x);
    tile_load<R, kPermThreads>(tile, psi, base, tm, T);
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < T; j += kPermThreads) {
        uint32_t d = 0;
        for (uint32_t p = 0; p < sw.np; ++p) {
            const bool x = (j & sw.la[p]) != 0, y = (j & sw.lb[p]) != 0;
            d |= (x != y) ? (sw.la[p] | sw.lb[p]) : 0u;
        }
        const uint32_t j2 = j ^ d;
        if (j2 > j) {
            const cplx_t<R> u = tile[j], v = tile[j2];
            tile[j] = v;
            tile[j2] = u;
        }
    }
    __syncthreads();
    tile_store<R, kPermThreads>(psi, tile, base, tm, T);
}

int check_swap_pairs(int n, const int32_t *pairs, int npairs) {
    if (npairs < 0 || npairs > kMaxSwapPairs)
        return fail(SV_EINVAL, "npairs %d outside [0, %d]", npairs, kMaxSwapPairs);
    if (npairs > 0 && !pairs)
        return fail(SV_EINVAL, "pairs is NULL");
    uint64_t seen = 0;
    for (int i = 0; i < 2 * npairs; ++i) {
        const int q = pairs[i];
        if (q < 0 || q >= n)
            return fail(SV_EINVAL, "qubit %d outside [0, %d)", q, n);
        if (seen & (1ull << q))
            return fail(SV_EINVAL, "qubit %d appears twice (pairs must be disjoint)", q);
        seen |= 1ull << q;
    }
    return SV_OK;
}

template <typename R> static int set_perm_lds(size_t lds) {
    if (lds > 65536)
        SV_HIP_TRY(hipFuncSetAttribute((const void *)k_permute_tile<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds));
    return SV_OK;
}

int launch_swap_qubits(int dtype, void *psi, int n, const int32_t *pairs, int npairs, hipStream_t st) {
    const int m_max = std::min(tuning().tile_log2[dtype == SV_C128 ? 0 : 1], n);
    for (int first = 0; first < npairs; first += kPermPairsPerPass) {
        const int np = std::min(kPermPairsPerPass, npairs - first);
        // tile qubit set: the low block [0, a) plus the swapped qubits >= a,
        // with a as large as the tile width allows
        std::vector<int> q;
        for (int i = 0; i < 2 * np; ++i)
            q.push_back(pairs[2 * first + i]);
        int a = std::max(1, m_max - (int)q.size());
        for (;;) {
            int nh = 0;
            for (int x : q)
                nh += x >= a ? 1 : 0;
            const int a2 = std::max(1, m_max - nh);
            if (a2 <= a)
                break;
            a = a2;
        }
        std::vector<int> high;
        for (int x : q)
            if (x >= a)
                high.push_back(x);
        std::sort(high.begin(), high.end());
        const int m = a + (int)high.size();
        if (m > n || high.size() > (size_t)kTileMaxHigh)
            return fail(SV_EINVAL, "cannot tile the exchange of these qubits (n=%d)", n);
        const TileMap tm = make_tile_map(n, m, a, high);
        // tile-local bit of each swapped qubit
        auto local = [&](int x) -> uint32_t {
            if (x < (int)tm.a)
                return 1u << x;
            for (uint32_t h = 0; h < tm.nh; ++h)
                if ((int)tm.hpos[h] == x)
                    return 1u << (tm.a + h);
            return 0u;
        };
        LocalSwaps sw;
        memset(&sw, 0, sizeof(sw));
        sw.np = (uint32_t)np;
        for (int i = 0; i < np; ++i) {
            sw.la[i] = local(pairs[2 * (first + i)]);
            sw.lb[i] = local(pairs[2 * (first + i) + 1]);
            if (!sw.la[i] || !sw.lb[i])
                return fail(SV_EINVAL, "internal: qubit outside the exchange tile");
        }
        const size_t lds = ((size_t)1 << m) * amp_bytes(dtype);
        if (dtype == SV_C128)
            SV_TRY(set_perm_lds<double>(lds));
        else
            SV_TRY(set_perm_lds<float>(lds));
        for (uint64_t t0 = 0; t0 < tm.ntiles; t0 += kMaxGridBlocks) {
            TileMap part = tm;
            part.tile0 = t0;
            const dim3 grid((unsigned)std::min(kMaxGridBlocks, tm.ntiles - t0));
            if (dtype == SV_C128)
                hipLaunchKernelGGL(k_permute_tile<double>, grid, dim3(kPermThreads), lds, st, (double2 *)psi, part,
                                   sw);
            else
                hipLaunchKernelGGL(k_permute_tile<float>, grid, dim3(kPermThreads), lds, st, (float2 *)psi, part,
                                   sw);
            SV_LAUNCH_CHECK();
        }
    }
    return SV_OK;
}

} // namespace sv

using namespace sv;

extern "C" {

int sv_swap_qubits(const sv_state_t *s, const int32_t *pairs, int npairs, sv_stream_t st) {
    clear_error();
    SV_TRY(validate_state(s));
    SV_TRY(check_swap_pairs(s->n, pairs, npairs));
    return launch_swap_qubits(s->dtype, s->data, s->n, pairs, npairs, (hipStream_t)st);
}

} // extern "C"
