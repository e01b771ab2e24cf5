// Pauli-sum Hamiltonians H = sum_j h_j P_j with P_j = i^{|x&z|} X^x Z^z
// (bit q of x / z places X / Z on qubit q; a qubit with both bits holds
// Y = iXZ).  P|k> = i^{|x&z|} (-1)^{popcount(z & k)} |k ^ x>, so
// (P psi)_k = i^{|x&z|} (-1)^{popcount(z & (k ^ x))} psi_{k ^ x}.
// Terms sharing an x mask read the same amplitude pairs and are grouped.
#pragma once

#include <vector>

#include "reduce.hpp"

namespace sv {

struct DTerm {
    double coef;
    uint64_t z;
    int32_t ny;   // |x & z| mod 4: the power of i
    int32_t idx;  // position in the caller's term list
};

struct DGroup {
    uint64_t x;
    int32_t first, count;  // terms [first, first + count) of the sorted list
};

struct PauliPlan {
    std::vector<DGroup> groups;
    std::vector<DTerm> terms;  // sorted by x mask (stable)
};

int make_pauli_plan(int n, const sv_pauli_t *terms, int nterms, PauliPlan *p);

// i^ny * w
__device__ __forceinline__ double re_ipow(int ny, double wr, double wi) {
    return ny == 0 ? wr : ny == 1 ? -wi : ny == 2 ? -wr : wi;
}
__device__ __forceinline__ double im_ipow(int ny, double wr, double wi) {
    return ny == 0 ? wi : ny == 1 ? wr : ny == 2 ? -wi : -wr;
}

__device__ __forceinline__ bool odd_parity(uint64_t v) { return __popcll(v) & 1; }

// Device copy of a Pauli plan plus the partial-sum workspace, allocated
// stream-ordered on the caller's stream.
struct PauliDevice {
    DTerm *terms = nullptr;
    DGroup *groups = nullptr;
    double *partials = nullptr;
    int nterms = 0, ngroups = 0;
};

int pauli_upload(const PauliPlan &p, size_t partial_doubles, hipStream_t st, PauliDevice *d);
void pauli_release(PauliDevice *d, hipStream_t st);

// out = H psi (gather over the term groups), plus per-workgroup partials of
// Re <psi|H psi> written to partials[0 .. grid).  Returns the grid used.
int launch_apply_paulis(int dtype, const void *psi, void *out, int n, const PauliDevice &d, hipStream_t st,
                        unsigned *grid);

} // namespace sv
