// Library-wide launch choices and their C ABI (sv_tune_set / sv_tune_get).
#include <cstring>
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
    //  - fused tiles always hold the 6 (complex128) / 7 (complex64) lowest
    //    qubits, i.e. 1 KiB contiguous runs, plus qubits picked per run.
    //  - dense blocks (SV_DENSE) on the 4 lowest qubits for stretches of at
    //    least 16 gates.
    static Tuning t = {{3, 4}, 1, 1, {12, 13}, {6, 7}, 2, 4, 16};
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
