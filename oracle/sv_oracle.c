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
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>

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

/* Use k threads in later parallel loops (for timing; every loop writes
 * disjoint outputs, so results do not depend on k). */
void or_set_num_threads(int k)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(k > 0 ? k : 1);
#else
    (void)k;
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

/* ------------------------------------------------------------------------
 * Block-scaled 16-bit fixed-point states.
 *
 * The paper names fixed-point arithmetic as future work (Sec. V) without
 * a format.  The reading taken here: each component (re, im) of an amplitude
 * is a signed 16-bit code q, and the 64 consecutive amplitudes of a block
 * (all 2^n of them when n < 6) share one power-of-two scale s, so that a
 * component's value is q * 2^s.  A single scale for the whole state could
 * not hold both the largest and the typical amplitude of an n-qubit state
 * (2^(-n/2) when spread evenly) in 16 bits.
 *
 * Storage: 2^n (re, im) int16 pairs, then one int8 scale per block.
 *
 * Encoding a block of floats: m = largest |component|; with
 * m = f 2^e, f in [0.5, 1) (frexp), the scale is s = e - 15, clamped to
 * [-126, 112] (s = -126 for m = 0); each code is the value times 2^-s
 * rounded to nearest, ties to even, saturated to [-32767, 32767].  Codes of
 * an encoded block therefore have their largest magnitude in
 * [16384, 32767].
 *
 * A gate on a fixed-point state: decode every amplitude to float (exact),
 * apply the pair update of Sec. III to each pair whose controls hold, in
 * float with the fixed fused multiply-add order below, then re-encode every
 * block that holds an amplitude of an updated pair.  Other blocks keep
 * their codes and scale.
 * ------------------------------------------------------------------------ */

#define OR_Q16_BLOCK 64

int or_q16_scale(float m)
{
    int e = 0;
    if (m == 0.0f)
        return -126;
    (void)frexpf(m, &e);
    int s = e - 15;
    if (s < -126)
        s = -126;
    if (s > 112)
        s = 112;
    return s;
}

int16_t or_q16_code(float v, int s)
{
    float r = rintf(ldexpf(v, -s));
    if (r > 32767.0f)
        r = 32767.0f;
    if (r < -32767.0f)
        r = -32767.0f;
    return (int16_t)r;
}

static void q16_encode_block(const float *v, int64_t len, int16_t *q, int8_t *s)
{
    float m = 0.0f;
    for (int64_t i = 0; i < 2 * len; ++i) {
        const float a = fabsf(v[i]);
        if (a > m)
            m = a;
    }
    const int sc = or_q16_scale(m);
    for (int64_t i = 0; i < 2 * len; ++i)
        q[i] = or_q16_code(v[i], sc);
    *s = (int8_t)sc;
}

static int64_t q16_block_len(int n)
{
    const int64_t N = (int64_t)1 << n;
    return N < OR_Q16_BLOCK ? N : OR_Q16_BLOCK;
}

/* Encode a complex128 state: each double is first rounded to float. */
void or_q16_encode(const double *psi, int n, int16_t *q, int8_t *s)
{
    const int64_t N = (int64_t)1 << n, B = q16_block_len(n), nb = N / B;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nb; ++b) {
        float v[2 * OR_Q16_BLOCK];
        for (int64_t i = 0; i < 2 * B; ++i)
            v[i] = (float)psi[2 * b * B + i];
        q16_encode_block(v, B, q + 2 * b * B, s + b);
    }
}

void or_q16_decode(const int16_t *q, const int8_t *s, int n, double *psi)
{
    const int64_t N = (int64_t)1 << n, B = q16_block_len(n);
    for (int64_t k = 0; k < N; ++k) {
        const int sc = s[k / B];
        psi[2 * k] = (double)ldexpf((float)q[2 * k], sc);
        psi[2 * k + 1] = (double)ldexpf((float)q[2 * k + 1], sc);
    }
}

/* u * x + v * y in float: one rounding chain per component, in this order:
 *   re = u.re x.re - u.im x.im + v.re y.re - v.im y.im
 *      evaluated as fma(u.re, x.re, fma(-u.im, x.im, fma(v.re, y.re, -(v.im y.im))))
 *   im = fma(u.re, x.im, fma(u.im, x.re, fma(v.re, y.im, v.im y.re))) */
static void q16_mac(const float *u, const float *v, float xr, float xi, float yr, float yi,
                    float *outr, float *outi)
{
    *outr = fmaf(u[0], xr, fmaf(-u[1], xi, fmaf(v[0], yr, -(v[1] * yi))));
    *outi = fmaf(u[0], xi, fmaf(u[1], xr, fmaf(v[0], yi, v[1] * yr)));
}

void or_q16_apply_gate(int16_t *q, int8_t *s, int n, int t, uint64_t cmask, uint64_t cvals,
                       const double *U)
{
    const int64_t N = (int64_t)1 << n, B = q16_block_len(n), nb = N / B;
    const int64_t st = (int64_t)1 << t;
    float u[8];
    for (int i = 0; i < 8; ++i)
        u[i] = (float)U[i];
    float *v = (float *)malloc(sizeof(float) * 2 * (size_t)N);
    char *touched = (char *)calloc((size_t)nb, 1);
    for (int64_t k = 0; k < N; ++k) {
        const int sc = s[k / B];
        v[2 * k] = ldexpf((float)q[2 * k], sc);
        v[2 * k + 1] = ldexpf((float)q[2 * k + 1], sc);
    }
    for (int64_t k = 0; k < N; ++k) {
        if (k & st)
            continue;
        if (((uint64_t)k & cmask) != cvals)
            continue;
        const int64_t k2 = k + st;
        const float xr = v[2 * k], xi = v[2 * k + 1], yr = v[2 * k2], yi = v[2 * k2 + 1];
        q16_mac(u, u + 2, xr, xi, yr, yi, &v[2 * k], &v[2 * k + 1]);
        q16_mac(u + 4, u + 6, xr, xi, yr, yi, &v[2 * k2], &v[2 * k2 + 1]);
        touched[k / B] = 1;
        touched[k2 / B] = 1;
    }
    for (int64_t b = 0; b < nb; ++b)
        if (touched[b])
            q16_encode_block(v + 2 * b * B, B, q + 2 * b * B, s + b);
    free(touched);
    free(v);
}

/* ------------------------------------------------------------------------
 * Block-scaled 32-bit fixed-point states: the same layout and block rule
 * with 32-bit codes, computed in double.  Each component is a signed
 * 32-bit code; the 64 amplitudes of a block share one int8 scale s, so a
 * value is code * 2^s.  Encoding a block: m = largest |component| (double),
 * m = f 2^e with f in [0.5, 1), s = e - 31 clamped to [-128, 96] (-128 for
 * m = 0), codes rounded to nearest, ties to even, saturated to
 * +-(2^31 - 1); the largest code magnitude of a block is then in
 * [2^30, 2^31 - 1].  A gate decodes (exact in double), applies the pair
 * update of Sec. III in double with the fma order below, and re-encodes
 * every block holding an element of an updated pair.
 * ------------------------------------------------------------------------ */

int or_q32_scale(double m)
{
    int e = 0;
    if (m == 0.0)
        return -128;
    (void)frexp(m, &e);
    int s = e - 31;
    if (s < -128)
        s = -128;
    if (s > 96)
        s = 96;
    return s;
}

int32_t or_q32_code(double v, int s)
{
    double r = rint(ldexp(v, -s));
    if (r > 2147483647.0)
        r = 2147483647.0;
    if (r < -2147483647.0)
        r = -2147483647.0;
    return (int32_t)r;
}

static void q32_encode_block(const double *v, int64_t len, int32_t *q, int8_t *s)
{
    double m = 0.0;
    for (int64_t i = 0; i < 2 * len; ++i) {
        const double a = fabs(v[i]);
        if (a > m)
            m = a;
    }
    const int sc = or_q32_scale(m);
    for (int64_t i = 0; i < 2 * len; ++i)
        q[i] = or_q32_code(v[i], sc);
    *s = (int8_t)sc;
}

void or_q32_encode(const double *psi, int n, int32_t *q, int8_t *s)
{
    const int64_t N = (int64_t)1 << n, B = q16_block_len(n), nb = N / B;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nb; ++b)
        q32_encode_block(psi + 2 * b * B, B, q + 2 * b * B, s + b);
}

void or_q32_decode(const int32_t *q, const int8_t *s, int n, double *psi)
{
    const int64_t N = (int64_t)1 << n, B = q16_block_len(n);
    for (int64_t k = 0; k < N; ++k) {
        const int sc = s[k / B];
        psi[2 * k] = ldexp((double)q[2 * k], sc);
        psi[2 * k + 1] = ldexp((double)q[2 * k + 1], sc);
    }
}

/* u * x + v * y in double, one rounding chain per component, in the order
 * of q16_mac above. */
static void q32_mac(const double *u, const double *v, double xr, double xi, double yr, double yi,
                    double *outr, double *outi)
{
    *outr = fma(u[0], xr, fma(-u[1], xi, fma(v[0], yr, -(v[1] * yi))));
    *outi = fma(u[0], xi, fma(u[1], xr, fma(v[0], yi, v[1] * yr)));
}

void or_q32_apply_gate(int32_t *q, int8_t *s, int n, int t, uint64_t cmask, uint64_t cvals,
                       const double *U)
{
    const int64_t N = (int64_t)1 << n, B = q16_block_len(n), nb = N / B;
    const int64_t st = (int64_t)1 << t;
    double *v = (double *)malloc(sizeof(double) * 2 * (size_t)N);
    char *touched = (char *)calloc((size_t)nb, 1);
    or_q32_decode(q, s, n, v);
    for (int64_t k = 0; k < N; ++k) {
        if (k & st)
            continue;
        if (((uint64_t)k & cmask) != cvals)
            continue;
        const int64_t k2 = k + st;
        const double xr = v[2 * k], xi = v[2 * k + 1], yr = v[2 * k2], yi = v[2 * k2 + 1];
        q32_mac(U, U + 2, xr, xi, yr, yi, &v[2 * k], &v[2 * k + 1]);
        q32_mac(U + 4, U + 6, xr, xi, yr, yi, &v[2 * k2], &v[2 * k2 + 1]);
        touched[k / B] = 1;
        touched[k2 / B] = 1;
    }
    for (int64_t b = 0; b < nb; ++b)
        if (touched[b])
            q32_encode_block(v + 2 * b * B, B, q + 2 * b * B, s + b);
    free(touched);
    free(v);
}
