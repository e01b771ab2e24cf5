// Library-wide launch choices and their C ABI (sv_tune_set / sv_tune_get).
#include <cstring>
#include <functional>
#include <mutex>

#include "sv_internal.hpp"

namespace sv {

Tuning &tuning() {
    // Defaults measured on MI355X at n=28:
    //  - controls on the 3 lowest index bits (one 128-byte line of complex128
    //    amplitudes) cannot skip memory traffic, and skipping their pairs
    //    leaves partially written lines that cost about 1.6x a full rewrite;
    //    so they are tested per lane and the unchanged values rewritten
    //    (4 bits for complex64's 8-byte amplitudes);
    //  - the wavefront kernel is the faster scheduled kernel whenever the
    //    target is among the 6 lowest free index bits;
    //  - 64 KiB LDS tiles for the fused pass.
    //  - fused tiles always hold the 3 (complex128) / 5 (complex64) lowest
    //    qubits, i.e. 128- and 256-byte contiguous runs, plus qubits picked
    //    per run: narrower runs leave more tile qubits to the planner (the
    //    n=32 layered circuit takes 80 passes with 128-byte runs, 91 with
    //    256-byte ones and 139 with 1 KiB ones), which outweighs their less
    //    efficient HBM accesses down to 128 bytes; 64-byte runs lost again.
    //  - dense blocks (SV_DENSE) on the 4 lowest qubits for stretches of at
    //    least 16 gates.
    //  - one pair (or amplitude) per lane in the scheduled pair and
    //    wavefront kernels (64-lane workgroups): in-place streams of 4 GiB
    //    reach about 6.7 TB/s that way against about 5.7 TB/s with four per
    //    lane; the masked baseline is fastest over the n=28 sweep with
    //    256-lane workgroups and one pair per lane (10.8 ms against 12.5 ms
    //    with four per lane, 16.1 ms with 64-lane workgroups, whose many
    //    workgroups cost more when most lanes only test and exit).
    static Tuning t = {{3, 4}, 1, 1, {12, 13}, {3, 5}, 2, 4, 16, 1, 1, 256, 1, 1, 2, 1, 16, {4, 8}};
    return t;
}

struct Key {
    const char *name;
    int *slot;
    int lo, hi;
};

static int find_key(const char *name, Key *out) {
    Tuning &t = tuning();
    const Key keys[] = {
        {"granule_bits_c128", &t.granule_bits[0], 0, 6},
        {"granule_bits_c64", &t.granule_bits[1], 0, 6},
        {"low_policy", &t.low_policy, 0, 1},
        {"wave_auto", &t.wave_auto, 0, 1},
        {"tile_log2_c128", &t.tile_log2[0], 6, 13},
        {"tile_log2_c64", &t.tile_log2[1], 6, 14},
        {"tile_low_bits_c128", &t.tile_low_bits[0], 1, 13},
        {"tile_low_bits_c64", &t.tile_low_bits[1], 1, 14},
        {"fuse_min_gates", &t.fuse_min_gates, 1, 1 << 20},
        {"dense_qubits", &t.dense_qubits, 4, 5},
        {"dense_min_gates", &t.dense_min_gates, 1, 1 << 20},
        {"pair_unroll", &t.pair_unroll, 1, 4},
        {"masked_unroll", &t.masked_unroll, 1, 4},
        {"masked_block", &t.masked_block, 64, 256},
        {"fuse_group", &t.fuse_group, 0, 1},
        {"fuse_pairs", &t.fuse_pairs, 0, 1},
        {"plan_lookahead", &t.plan_lookahead, 0, 2},
        {"fuse_perm", &t.fuse_perm, 0, 1},
        {"batch_split", &t.batch_split, 1, 64},
        {"phase_sweep_min_c128", &t.phase_sweep_min[0], 1, 64},
        {"phase_sweep_min_c64", &t.phase_sweep_min[1], 1, 64},
    };
    for (const Key &k : keys)
        if (name && strcmp(k.name, name) == 0) {
            *out = k;
            return SV_OK;
        }
    return fail(SV_EINVAL, "unknown tuning key '%s'", name ? name : "(null)");
}

} // namespace sv

using namespace sv;

extern "C" {

int sv_tune_set(const char *key, int64_t value) {
    clear_error();
    Key k;
    SV_TRY(find_key(key, &k));
    if (value < k.lo || value > k.hi)
        return fail(SV_EINVAL, "tuning %s=%lld outside [%d, %d]", key, (long long)value, k.lo, k.hi);
    // two-valued knobs: only the bounds themselves
    const bool two = !strcmp(key, "pair_unroll") || !strcmp(key, "masked_unroll") || !strcmp(key, "masked_block");
    if (two && value != k.lo && value != k.hi)
        return fail(SV_EINVAL, "tuning %s takes %d or %d (got %lld)", key, k.lo, k.hi, (long long)value);
    *k.slot = (int)value;
    return SV_OK;
}

int sv_tune_get(const char *key, int64_t *value) {
    clear_error();
    Key k;
    SV_TRY(find_key(key, &k));
    if (!value)
        return fail(SV_EINVAL, "value is NULL");
    *value = *k.slot;
    return SV_OK;
}

} // extern "C"

// ---------------------------------------------------------------- autotuner
//
// Times candidate launch choices on the current device with HIP events on a
// scratch state of 2^n amplitudes and keeps the fastest:
//  1. the low-control granule and policy, on controlled gates whose controls
//     sit on the lowest index bits;
//  2. whether SV_MODE_AUTO uses the wavefront kernel, on low-target gates;
//  3. the fused tile width and its contiguous low block, on two layers of
//     single-qubit gates on every qubit plus a CNOT ladder.
// Results can be written to / read from a small JSON file keyed by device
// architecture and dtype.
#include <cmath>
#include <fstream>
#include <sstream>

namespace sv {

static int time_events(hipStream_t st, int reps, float *ms_out, const std::function<int()> &fn) {
    hipEvent_t a, b;
    SV_HIP_TRY(hipEventCreate(&a));
    SV_HIP_TRY(hipEventCreate(&b));
    int r = fn();  // warm-up
    float best = 1e30f;
    for (int i = 0; i < reps && r == SV_OK; ++i) {
        (void)hipEventRecord(a, st);
        r = fn();
        (void)hipEventRecord(b, st);
        (void)hipEventSynchronize(b);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, a, b);
        best = std::min(best, ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms_out = best;
    return r;
}

bool dense_supported(int dtype, int kq, int n);

static std::string tune_json(const DeviceInfo &di, int dtype) {
    const Tuning &t = tuning();
    const int d = dtype == SV_C128 ? 0 : 1;
    std::ostringstream o;
    o << "{\"arch\": \"" << di.arch << "\", \"dtype\": \"" << (dtype == SV_C128 ? "c128" : "c64")
      << "\", \"granule_bits\": " << t.granule_bits[d] << ", \"low_policy\": " << t.low_policy
      << ", \"wave_auto\": " << t.wave_auto << ", \"tile_log2\": " << t.tile_log2[d]
      << ", \"tile_low_bits\": " << t.tile_low_bits[d] << ", \"dense_min_gates\": " << t.dense_min_gates
      << "}";
    return o.str();
}

// Apply one JSON object of the format tune_json writes (flat, integer values).
static int apply_tune_json(const std::string &line, const std::string &arch) {
    auto field = [&](const char *key, std::string *out) -> bool {
        const std::string k = std::string("\"") + key + "\":";
        size_t p = line.find(k);
        if (p == std::string::npos)
            return false;
        p += k.size();
        while (p < line.size() && (line[p] == ' ' || line[p] == '"'))
            ++p;
        size_t e = p;
        while (e < line.size() && line[e] != ',' && line[e] != '}' && line[e] != '"')
            ++e;
        *out = line.substr(p, e - p);
        return true;
    };
    std::string a, dt;
    if (!field("arch", &a) || !field("dtype", &dt))
        return fail(SV_EINVAL, "tuning record without arch/dtype");
    if (a != arch)
        return SV_OK;  // another device's record
    const char *sfx = dt == "c128" ? "_c128" : "_c64";
    const char *keys[] = {"granule_bits", "low_policy", "wave_auto", "tile_log2", "tile_low_bits"};
    for (const char *k : keys) {
        std::string v;
        if (!field(k, &v))
            return fail(SV_EINVAL, "tuning record without %s", k);
        const bool per_dtype = strcmp(k, "low_policy") != 0 && strcmp(k, "wave_auto") != 0;
        const std::string name = std::string(k) + (per_dtype ? sfx : "");
        SV_TRY(sv_tune_set(name.c_str(), atoll(v.c_str())));
    }
    // optional fields (a record may omit them)
    const char *opt[] = {"dense_min_gates"};
    for (const char *k : opt) {
        std::string v;
        if (field(k, &v))
            SV_TRY(sv_tune_set(k, atoll(v.c_str())));
    }
    return SV_OK;
}

} // namespace sv

extern "C" {

int sv_tune_load(const char *path) {
    clear_error();
    if (!path)
        return fail(SV_EINVAL, "path is NULL");
    std::ifstream f(path);
    if (!f)
        return fail(SV_EINVAL, "cannot open %s", path);
    std::string arch;
    const char *env = getenv("SV_TUNE_ARCH");  // lets a host without a device read a cache
    if (env) {
        arch = env;
    } else {
        DeviceInfo di;
        SV_TRY(device_info(&di));
        arch = di.arch;
    }
    std::string line;
    int applied = 0;
    while (std::getline(f, line)) {
        if (line.find('{') == std::string::npos)
            continue;
        SV_TRY(apply_tune_json(line, arch));
        ++applied;
    }
    if (!applied)
        return fail(SV_EINVAL, "no tuning records in %s", path);
    return SV_OK;
}

int sv_autotune(int n, int dtype, const char *cache_path, char *report, int report_len, sv_stream_t stream) {
    clear_error();
    if (dtype != SV_C128 && dtype != SV_C64)
        return fail(SV_EINVAL, "unknown dtype %d", dtype);
    if (n < 16 || n > 30)
        return fail(SV_EINVAL, "autotune register n=%d outside [16, 30]", n);
    hipStream_t st = (hipStream_t)stream;
    DeviceInfo di;
    SV_TRY(device_info(&di));
    sv_state_t s;
    SV_TRY(sv_alloc(&s, n, dtype));
    int r = sv_init(&s, 0, st);
    const double H[8] = {0.70710678118654752, 0, 0.70710678118654752, 0, 0.70710678118654752, 0,
                         -0.70710678118654752, 0};
    Tuning &t = tuning();
    const int d = dtype == SV_C128 ? 0 : 1;
    std::ostringstream rep;
    // 1. granule bits and policy
    if (r == SV_OK) {
        const uint64_t cms[] = {1, 2, 4, 3, 8, 0x28, 0x101};
        float best = 1e30f;
        int bg = t.granule_bits[d], bp = t.low_policy;
        const int grans[] = {0, 2, 3, 4};
        for (int g : grans)
            for (int pol = 0; pol < 2 && r == SV_OK; ++pol) {
                t.granule_bits[d] = g;
                t.low_policy = pol;
                float ms = 0;
                r = time_events(st, 3, &ms, [&]() -> int {
                    for (uint64_t cm : cms)
                        SV_TRY(sv_apply_gate_masks(&s, n - 2, cm, cm, H, SV_MODE_AUTO, st));
                    return SV_OK;
                });
                rep << "granule " << g << " policy " << pol << ": " << ms << " ms\n";
                if (ms < best) {
                    best = ms;
                    bg = g;
                    bp = pol;
                }
            }
        t.granule_bits[d] = bg;
        t.low_policy = bp;
    }
    // 2. wavefront kernel for low targets
    if (r == SV_OK) {
        float msw[2] = {0, 0};
        for (int w = 0; w < 2 && r == SV_OK; ++w) {
            t.wave_auto = w;
            r = time_events(st, 3, &msw[w], [&]() -> int {
                for (int tq = 0; tq < 6; ++tq)
                    SV_TRY(sv_apply_gate_masks(&s, tq, 0, 0, H, SV_MODE_AUTO, st));
                return SV_OK;
            });
            rep << "wave_auto " << w << ": " << msw[w] << " ms\n";
        }
        t.wave_auto = msw[1] <= msw[0] ? 1 : 0;
    }
    // 3. fused tile shape
    if (r == SV_OK) {
        std::vector<sv_gate_t> gates;
        for (int layer = 0; layer < 2; ++layer) {
            for (int q = 0; q < n; ++q) {
                sv_gate_t g;
                memset(&g, 0, sizeof(g));
                g.kind = layer ? SV_G_RY : SV_G_H;
                g.target = q;
                g.param = -1;
                g.theta = 0.3 + q;
                gates.push_back(g);
            }
            for (int q = 0; q + 1 < n; ++q) {
                sv_gate_t g;
                memset(&g, 0, sizeof(g));
                g.kind = SV_G_X;
                g.target = q + 1;
                g.ctrl_mask = g.ctrl_vals = 1ull << q;
                g.param = -1;
                gates.push_back(g);
            }
        }
        const int widths_c128[] = {10, 11, 12};
        const int widths_c64[] = {11, 12, 13};
        const int lows[] = {5, 6, 7};
        float best = 1e30f;
        int bw = t.tile_log2[d], bl = t.tile_low_bits[d];
        for (int wi = 0; wi < 3 && r == SV_OK; ++wi)
            for (int li = 0; li < 3 && r == SV_OK; ++li) {
                t.tile_log2[d] = d == 0 ? widths_c128[wi] : widths_c64[wi];
                t.tile_low_bits[d] = lows[li];
                sv_circuit_t *c = nullptr;
                r = sv_circuit_create(n, dtype, gates.data(), (int)gates.size(), 0, SV_FUSE, &c);
                if (r != SV_OK)
                    break;
                float ms = 0;
                r = time_events(st, 3, &ms, [&]() -> int { return sv_circuit_run(c, &s, nullptr, st); });
                (void)sv_circuit_destroy(c);
                rep << "tile " << t.tile_log2[d] << " low " << lows[li] << ": " << ms << " ms\n";
                if (ms < best) {
                    best = ms;
                    bw = t.tile_log2[d];
                    bl = lows[li];
                }
            }
        t.tile_log2[d] = bw;
        t.tile_low_bits[d] = bl;
    }
    // 4. dense blocks against fused gates for a long stretch on the low qubits
    if (r == SV_OK && dense_supported(dtype, t.dense_qubits, n)) {
        std::vector<sv_gate_t> gates;
        const int k = t.dense_qubits;
        for (int i = 0; i < 48; ++i) {
            sv_gate_t g;
            memset(&g, 0, sizeof(g));
            g.param = -1;
            g.target = i % k;
            if (i % 3 == 2) {
                g.kind = SV_G_X;
                g.ctrl_mask = g.ctrl_vals = 1ull << ((i + 1) % k);
            } else {
                g.kind = i % 3 ? SV_G_RY : SV_G_H;
                g.theta = 0.1 * i;
            }
            gates.push_back(g);
        }
        float msd[2] = {0, 0};
        for (int dn = 0; dn < 2 && r == SV_OK; ++dn) {
            sv_circuit_t *c = nullptr;
            r = sv_circuit_create(n, dtype, gates.data(), (int)gates.size(), 0, dn ? (SV_FUSE | SV_DENSE) : SV_FUSE,
                                  &c);
            if (r != SV_OK)
                break;
            r = time_events(st, 3, &msd[dn], [&]() -> int { return sv_circuit_run(c, &s, nullptr, st); });
            (void)sv_circuit_destroy(c);
            rep << (dn ? "dense block" : "fused gates") << " for a 48-gate stretch: " << msd[dn] << " ms\n";
        }
        // SV_DENSE only turns stretches into dense blocks when that is faster
        if (r == SV_OK && msd[1] >= msd[0])
            t.dense_min_gates = 1 << 20;
    }
    (void)hipStreamSynchronize(st);
    (void)sv_free(&s);
    if (r != SV_OK)
        return r;
    const std::string js = tune_json(di, dtype);
    rep << "chosen " << js << "\n";
    if (cache_path) {
        // keep other records, replace the one for this arch and dtype
        std::vector<std::string> keep;
        std::ifstream in(cache_path);
        std::string line;
        const std::string me = "\"arch\": \"" + di.arch + "\", \"dtype\": \"" + (dtype == SV_C128 ? "c128" : "c64");
        while (in && std::getline(in, line))
            if (line.find('{') != std::string::npos && line.find(me) == std::string::npos)
                keep.push_back(line);
        std::ofstream out(cache_path);
        if (!out)
            return fail(SV_EINVAL, "cannot write %s", cache_path);
        for (auto &k : keep)
            out << k << "\n";
        out << js << "\n";
    }
    if (report && report_len > 0) {
        const std::string s2 = rep.str();
        strncpy(report, s2.c_str(), (size_t)report_len - 1);
        report[report_len - 1] = '\0';
    }
    return SV_OK;
}

} // extern "C"
