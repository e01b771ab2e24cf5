/*
 * CPU oracle for full-state-vector gate application (test infrastructure).
 *
 * This file is the reference that the GPU library is checked against.  It is
 * deliberately plain and slow: every operation is a loop over all 2^n basis
 * indices that tests the relevant bits, written in double precision with a
 * fixed evaluation order (build with -O2 -ffp-contract=off, no fast-math).
 * It shares no code, header or table with the GPU library.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load it.
 *
 * Conventions (paper, Sec. III "Quantum Circuit Simulation"):
 *   - the state holds 2^n complex amplitudes, stored as interleaved
 *     (re, im) doubles;
 *   - qubit q is bit q of the amplitude index, qubit 0 the least significant;
 *   - a single-qubit gate G = [[a, b], [c, d]] on target t maps each pair
 *     (C_k, C_{k+2^t}) with bit t of k clear to
 *     (a C_k + b C_{k+2^t}, c C_k + d C_{k+2^t})  (pair-update equation);
 *   - a controlled gate updates a pair only when every control bit of k holds
 *     its required value (paper: value 1; here any value, qubit-indexed in
 *     cvals), and otherwise leaves the pair unchanged (Sec. III, the paragraph
 *     on controls cancelling whole iterations, and the baseline kernel figure).
 *
 * U is passed as 8 doubles: a.re a.im b.re b.im c.re c.im d.re d.im.
 */
#include <stdint.h>
#include <stddef.h>

/* Complex product helpers with a fixed operation order. */
static inline double mul_re(double ar, double ai, double xr, double xi)
{
    return ar * xr - ai * xi;
}

static inline double mul_im(double ar, double ai, double xr, double xi)
{
    return ar * xi + ai * xr;
}

/* One gate applied in place: loop over every basis index k, skip k unless
 * bit t of k is 0 and the control bits match, then update the pair
 * (k, k + 2^t) by the 2x2 matrix.  Pair-update equation and the baseline
 * kernel figure of Sec. III-A.  Pairs are disjoint, so the loop iterations
 * are independent and may run in any order. */
void or_apply_gate(double *psi, int n, int t, uint64_t cmask, uint64_t cvals,
                   const double *U)
{
    const int64_t N = (int64_t)1 << n;
    const int64_t st = (int64_t)1 << t;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < N; ++k) {
        if (k & st)
            continue;
        if (((uint64_t)k & cmask) != cvals)
            continue;
        const int64_t k2 = k + st;
        const double xr = psi[2 * k], xi = psi[2 * k + 1];
        const double yr = psi[2 * k2], yi = psi[2 * k2 + 1];
        psi[2 * k] = mul_re(U[0], U[1], xr, xi) + mul_re(U[2], U[3], yr, yi);
        psi[2 * k + 1] = mul_im(U[0], U[1], xr, xi) + mul_im(U[2], U[3], yr, yi);
        psi[2 * k2] = mul_re(U[4], U[5], xr, xi) + mul_re(U[6], U[7], yr, yi);
        psi[2 * k2 + 1] = mul_im(U[4], U[5], xr, xi) + mul_im(U[6], U[7], yr, yi);
    }
}

/* A single output amplitude of the same gate, computed from the input state
 * without modifying it: the value that or_apply_gate would leave at index k.
 * Used to check sampled outputs of very large states one by one. */
void or_gate_amplitude(const double *psi, int n, int t, uint64_t cmask,
                       uint64_t cvals, const double *U, uint64_t k, double *out)
{
    (void)n;
    const uint64_t st = (uint64_t)1 << t;
    if ((k & cmask) != cvals) {
        out[0] = psi[2 * k];
        out[1] = psi[2 * k + 1];
        return;
    }
    const uint64_t k0 = k & ~st, k1 = k | st;
    const double xr = psi[2 * k0], xi = psi[2 * k0 + 1];
    const double yr = psi[2 * k1], yi = psi[2 * k1 + 1];
    if ((k & st) == 0) {
        out[0] = mul_re(U[0], U[1], xr, xi) + mul_re(U[2], U[3], yr, yi);
        out[1] = mul_im(U[0], U[1], xr, xi) + mul_im(U[2], U[3], yr, yi);
    } else {
        out[0] = mul_re(U[4], U[5], xr, xi) + mul_re(U[6], U[7], yr, yi);
        out[1] = mul_im(U[4], U[5], xr, xi) + mul_im(U[6], U[7], yr, yi);
    }
}

/* Brute-force list of the first pair elements a controlled gate updates, in
 * ascending order: every k with bit t clear and the control bits matching.
 * This is the set the reduced iteration index set of Sec. III-B enumerates.
 * Returns the count; out must hold 2^(n-1) entries. */
int64_t or_pair_list(int n, int t, uint64_t cmask, uint64_t cvals, uint64_t *out)
{
    const uint64_t N = (uint64_t)1 << n;
    const uint64_t st = (uint64_t)1 << t;
    int64_t m = 0;
    for (uint64_t k = 0; k < N; ++k) {
        if (k & st)
            continue;
        if ((k & cmask) != cvals)
            continue;
        out[m++] = k;
    }
    return m;
}

static int popcount64(uint64_t v)
{
    int c = 0;
    while (v) {
        c += (int)(v & 1u);
        v >>= 1;
    }
    return c;
}

/* <psi| P |psi> for the Pauli string P = i^{|x&z|} X^x Z^z, where bit q of x
 * (of z) puts an X (a Z) on qubit q and Y = iXZ.  P|j> = i^{|x&z|}
 * (-1)^{popcount(z&j)} |j ^ x>, so (P psi)_k = i^{|x&z|}
 * (-1)^{popcount(z & (k^x))} psi_{k^x}.  Serial sum over k in index order.
 * out[0], out[1] receive the real and imaginary parts (the latter is zero up
 * to rounding because P is Hermitian). */
void or_expect_pauli(const double *psi, int n, uint64_t x, uint64_t z, double *out)
{
    const uint64_t N = (uint64_t)1 << n;
    const int ny = popcount64(x & z) & 3; /* power of i */
    double sr = 0.0, si = 0.0;
    for (uint64_t k = 0; k < N; ++k) {
        const uint64_t j = k ^ x;
        double vr = psi[2 * j], vi = psi[2 * j + 1];
        if (popcount64(z & j) & 1) {
            vr = -vr;
            vi = -vi;
        }
        /* multiply by i^ny */
        double wr = vr, wi = vi;
        if (ny == 1) {
            wr = -vi;
            wi = vr;
        } else if (ny == 2) {
            wr = -vr;
            wi = -vi;
        } else if (ny == 3) {
            wr = vi;
            wi = -vr;
        }
        /* conj(psi_k) * w */
        const double ar = psi[2 * k], ai = psi[2 * k + 1];
        sr += ar * wr + ai * wi;
        si += ar * wi - ai * wr;
    }
    out[0] = sr;
    out[1] = si;
}

/* out += coef * P psi for one Pauli string (same convention as above).  Used
 * to form H psi for H = sum_j h_j P_j by definition. */
void or_add_pauli(const double *psi, double *out, int n, uint64_t x, uint64_t z,
                  double coef)
{
    const int64_t N = (int64_t)1 << n;
    const int ny = popcount64(x & z) & 3;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < N; ++k) {
        const uint64_t j = (uint64_t)k ^ x;
        double vr = psi[2 * j], vi = psi[2 * j + 1];
        if (popcount64(z & j) & 1) {
            vr = -vr;
            vi = -vi;
        }
        double wr = vr, wi = vi;
        if (ny == 1) {
            wr = -vi;
            wi = vr;
        } else if (ny == 2) {
            wr = -vr;
            wi = -vi;
        } else if (ny == 3) {
            wr = vi;
            wi = -vr;
        }
        out[2 * k] += coef * wr;
        out[2 * k + 1] += coef * wi;
    }
}

/* sum_k |psi_k|^2, serial. */
double or_norm2(const double *psi, int n)
{
    const uint64_t N = (uint64_t)1 << n;
    double s = 0.0;
    for (uint64_t k = 0; k < N; ++k)
        s += psi[2 * k] * psi[2 * k] + psi[2 * k + 1] * psi[2 * k + 1];
    return s;
}

/* Set psi to the basis state |b>. */
void or_basis(double *psi, int n, uint64_t b)
{
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < N; ++k) {
        psi[2 * k] = 0.0;
        psi[2 * k + 1] = 0.0;
    }
    psi[2 * b] = 1.0;
}

/* Number of OpenMP threads the parallel loops above use (1 without OpenMP). */
int or_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* A 2^k x 2^k complex matrix M (row-major, interleaved re/im) applied to the
 * k lowest qubits: each row of 2^k consecutive amplitudes becomes M . row.
 * Plain triple loop through a temporary row. */
void or_apply_block_low(double *psi, int n, int k, const double *M)
{
    const int64_t dim = (int64_t)1 << k;
    const int64_t rows = (int64_t)1 << (n - k);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < rows; ++r) {
        double tmp[2 * 64];
        double *row = psi + 2 * r * dim;
        for (int64_t a = 0; a < dim; ++a) {
            double sr = 0.0, si = 0.0;
            for (int64_t b = 0; b < dim; ++b) {
                const double mr = M[2 * (a * dim + b)], mi = M[2 * (a * dim + b) + 1];
                sr += mul_re(mr, mi, row[2 * b], row[2 * b + 1]);
                si += mul_im(mr, mi, row[2 * b], row[2 * b + 1]);
            }
            tmp[2 * a] = sr;
            tmp[2 * a + 1] = si;
        }
        for (int64_t a = 0; a < 2 * dim; ++a)
            row[a] = tmp[a];
    }
}

/* Exchange qubits a and b: the amplitude at index k moves to the index with
 * bits a and b of k exchanged.  Plain loop over every k, swapping each pair
 * {k, k'} once from its smaller index. */
void or_swap_qubits(double *psi, int n, int a, int b)
{
    const uint64_t N = (uint64_t)1 << n;
    for (uint64_t k = 0; k < N; ++k) {
        const uint64_t ba = (k >> a) & 1u, bb = (k >> b) & 1u;
        if (ba == bb)
            continue;
        const uint64_t k2 = k ^ (((uint64_t)1 << a) | ((uint64_t)1 << b));
        if (k2 < k)
            continue;
        const double r = psi[2 * k], i = psi[2 * k + 1];
        psi[2 * k] = psi[2 * k2];
        psi[2 * k + 1] = psi[2 * k2 + 1];
        psi[2 * k2] = r;
        psi[2 * k2 + 1] = i;
    }
}
