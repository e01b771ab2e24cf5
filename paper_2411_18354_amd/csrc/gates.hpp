// Named single-qubit gates as 2x2 matrices, usable on host and device so a
// circuit can take its rotation angles from device memory.
//
// Conventions: X and H as printed in Sec. I of the paper; Y, Z and the
// rotations after Nielsen & Chuang: Y = [[0,-i],[i,0]], Z = diag(1,-1),
// R{X,Y,Z}(theta) = exp(-i theta P / 2), P(theta) = diag(1, e^{i theta})
// (the QFT rotation R_m of Sec. IV-A is P(2 pi / 2^m)).  The adjoint flag
// gives the conjugate transpose.  Output: a.re a.im b.re b.im c.re c.im d.re
// d.im of G = [[a, b], [c, d]].
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/sv.h"

namespace sv {

__host__ __device__ inline bool gate_kind_valid(int kind) {
    const int k = kind & ~SV_G_ADJOINT;
    return k >= SV_G_MATRIX && k <= SV_G_P && (kind & ~(SV_G_ADJOINT | 0xff)) == 0;
}

__host__ __device__ inline bool gate_kind_param(int kind) {
    const int k = kind & ~SV_G_ADJOINT;
    return k == SV_G_RX || k == SV_G_RY || k == SV_G_RZ || k == SV_G_P;
}

// Diagonal for every angle (commutes with any other diagonal gate).
__host__ __device__ inline bool gate_kind_diagonal(int kind) {
    const int k = kind & ~SV_G_ADJOINT;
    return k == SV_G_Z || k == SV_G_RZ || k == SV_G_P;
}

__host__ __device__ inline void gate_matrix(int kind, double theta, const double *U, double *o) {
    const int k = kind & ~SV_G_ADJOINT;
    for (int i = 0; i < 8; ++i)
        o[i] = 0.0;
    const double h = 0.5 * theta;
    switch (k) {
    case SV_G_MATRIX:
        for (int i = 0; i < 8; ++i)
            o[i] = U[i];
        break;
    case SV_G_X:
        o[2] = 1.0;
        o[4] = 1.0;
        break;
    case SV_G_Y:
        o[3] = -1.0;  // b = -i
        o[5] = 1.0;   // c = +i
        break;
    case SV_G_Z:
        o[0] = 1.0;
        o[6] = -1.0;
        break;
    case SV_G_H: {
        const double r = 0.70710678118654752440;
        o[0] = r;
        o[2] = r;
        o[4] = r;
        o[6] = -r;
        break;
    }
    case SV_G_RX: {
        const double c = cos(h), s = sin(h);
        o[0] = c;
        o[3] = -s;
        o[5] = -s;
        o[6] = c;
        break;
    }
    case SV_G_RY: {
        const double c = cos(h), s = sin(h);
        o[0] = c;
        o[2] = -s;
        o[4] = s;
        o[6] = c;
        break;
    }
    case SV_G_RZ: {
        const double c = cos(h), s = sin(h);
        o[0] = c;
        o[1] = -s;
        o[6] = c;
        o[7] = s;
        break;
    }
    case SV_G_P:
        o[0] = 1.0;
        o[6] = cos(theta);
        o[7] = sin(theta);
        break;
    default:
        break;
    }
    if (kind & SV_G_ADJOINT) {
        // conj transpose: a* c* ; b* d*
        const double ar = o[0], ai = o[1], br = o[2], bi = o[3], cr = o[4], ci = o[5], dr = o[6], di = o[7];
        o[0] = ar;
        o[1] = -ai;
        o[2] = cr;
        o[3] = -ci;
        o[4] = br;
        o[5] = -bi;
        o[6] = dr;
        o[7] = -di;
    }
}

// d/dtheta of a parameterised gate, written as A . G(theta) with the 2x2
// generator term A (so that the derivative of the controlled gate is the
// control projector times A G):  RX, RY, RZ: A = -i/2 P;  P(theta):
// A = diag(0, i).  For the adjoint flag the derivative of G^dagger is
// G^dagger . A^dagger; callers only differentiate non-adjoint gates.
__host__ __device__ inline void gate_generator(int kind, double *a) {
    const int k = kind & ~SV_G_ADJOINT;
    for (int i = 0; i < 8; ++i)
        a[i] = 0.0;
    switch (k) {
    case SV_G_RX:  // -i/2 X = [[0, -i/2], [-i/2, 0]]
        a[3] = -0.5;
        a[5] = -0.5;
        break;
    case SV_G_RY:  // -i/2 Y = [[0, -1/2], [1/2, 0]]
        a[2] = -0.5;
        a[4] = 0.5;
        break;
    case SV_G_RZ:  // -i/2 Z = diag(-i/2, +i/2)
        a[1] = -0.5;
        a[7] = 0.5;
        break;
    case SV_G_P:  // diag(0, i)
        a[7] = 1.0;
        break;
    default:
        break;
    }
}

} // namespace sv
