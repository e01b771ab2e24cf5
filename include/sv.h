/*
 * sv.h — C ABI of the MI355X state-vector library (libsv.so).
 *
 * The library applies single-qubit gates with any number of controls to a
 * 2^n complex state vector held in device memory, enumerating only the
 * amplitude pairs whose control bits hold (control-aware iteration
 * scheduling, arXiv:2411.18354 Sec. III-B), and builds circuits, Pauli-sum
 * expectation values, adjoint gradients and batched runs on top of it.
 *
 * Conventions shared by every entry point
 *  - Amplitude k of an n-qubit state is complex; qubit q is bit q of k, qubit
 *    0 the least significant (paper Sec. III).  Storage is interleaved
 *    (re, im): complex128 = two doubles (16 B), complex64 = two floats (8 B).
 *  - A 2x2 gate G = [[a, b], [c, d]] on target t updates each pair
 *    (C_k, C_{k+2^t}) with bit t of k clear to (a C_k + b C_{k+2^t},
 *    c C_k + d C_{k+2^t}) (pair-update equation, Sec. III).  Matrices are
 *    passed as 8 doubles: a.re a.im b.re b.im c.re c.im d.re d.im.
 *  - Controls are qubit-indexed: bit q of ctrl_mask marks qubit q as a
 *    control and bit q of ctrl_vals is its required value (the paper uses
 *    value 1; value 0 is the negative control of its Sec. I figure).
 *  - Every function returns SV_OK (0) or a negative sv_status; the reason is
 *    available from sv_last_error() (thread-local, valid until the next call
 *    on the same thread).  Arguments are validated before anything is
 *    enqueued, so an argument error leaves device memory untouched.
 *  - sv_stream_t is a hipStream_t (NULL selects the null stream).  Work is
 *    enqueued on it and calls return without synchronising; host arrays
 *    passed in are copied before the call returns, device outputs are valid
 *    once the stream reaches them.
 *  - The library never frees memory it did not allocate.  sv_state_t is a
 *    non-owning view; data may be any device allocation of the right size
 *    and 16-byte (complex128) or 8-byte (complex64) alignment.
 */
#ifndef SV_H
#define SV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *sv_stream_t;

typedef enum sv_status {
    SV_OK = 0,
    SV_EINVAL = -1,  /* invalid argument (range, duplicate, null, mismatch) */
    SV_ENOMEM = -2,  /* device allocation failed */
    SV_EHIP = -3,    /* a HIP runtime call failed */
    SV_ENOTSUP = -4  /* valid request the library does not handle */
} sv_status;

/* SV_CQ16, SV_CQ32: block-scaled fixed-point complex with 16-bit or 32-bit
 * codes, the fixed-point state precision the paper lists as future work
 * (Sec. V).  Layout: 2^n amplitudes of two signed codes (re, im; 4 bytes
 * per amplitude for SV_CQ16, 8 for SV_CQ32), followed by one int8 scale per
 * block of 64 consecutive amplitudes (a single block of all 2^n when n < 6);
 * a component's value is code * 2^scale.  Encoding a block takes m, its
 * largest |component|, writes m = f 2^e with f in [0.5, 1), uses the scale
 * e - B (B = 15 for SV_CQ16, 31 for SV_CQ32; clamped to [-126, 112] and
 * [-128, 96], the minimum for an all-zero block) and rounds each
 * value / 2^scale to the nearest code, ties to even, saturated to
 * +-(2^B - 1).  Arithmetic is in float for SV_CQ16 and in double for
 * SV_CQ32.  Storage is sv_state_bytes(n, dtype) bytes, 16-byte aligned.
 * Fixed-point states are taken by sv_alloc, sv_free, sv_init,
 * sv_copy_state, sv_convert, sv_apply_gate(_masks), sv_gate_plan, and
 * circuits without SV_FUSE, SV_DENSE or SV_REMAP; every other call returns
 * SV_ENOTSUP for them. */
typedef enum sv_dtype { SV_C128 = 0, SV_C64 = 1, SV_CQ16 = 2, SV_CQ32 = 3 } sv_dtype;

/* Largest supported register: 2^34 complex128 amplitudes is 256 GiB. */
#define SV_MAX_QUBITS_C128 34
#define SV_MAX_QUBITS_C64 35
#define SV_MAX_QUBITS_CQ16 36
#define SV_MAX_QUBITS_CQ32 35

typedef struct sv_state {
    void *data;    /* device pointer to the state's storage, caller-owned */
    int32_t n;     /* number of qubits, 1 <= n <= SV_MAX_QUBITS_* */
    int32_t dtype; /* sv_dtype */
} sv_state_t;

/* Message for the last failing call on this thread ("" if none). */
const char *sv_last_error(void);

/* Library ABI version (major * 10000 + minor * 100 + patch). */
int sv_version(void);

/* Allocate 2^n amplitudes of the given dtype on the current device and fill
 * s; the caller releases it with sv_free.  SV_ENOMEM if hipMalloc fails. */
int sv_alloc(sv_state_t *s, int n, int dtype);

/* Release memory obtained from sv_alloc and clear s->data.  Passing a state
 * whose data came from elsewhere is undefined. */
int sv_free(sv_state_t *s);

/* Set the state to the basis state |basis_index> (all amplitudes zero except
 * amplitude basis_index = 1).  basis_index < 2^n. */
int sv_init(const sv_state_t *s, uint64_t basis_index, sv_stream_t st);

/* Copy one state into another of the same n and dtype (non-overlapping
 * device buffers; a state copied onto itself is a no-op). */
int sv_copy_state(const sv_state_t *dst, const sv_state_t *src, sv_stream_t st);

/* Bytes of storage of an n-qubit state of the given dtype: 2^n * 16
 * (complex128), 2^n * 8 (complex64), 2^n * 4 + max(1, 2^n / 64) (SV_CQ16),
 * 2^n * 8 + max(1, 2^n / 64) (SV_CQ32).  Host-only. */
int sv_state_bytes(int n, int dtype, uint64_t *bytes);

/* Convert src into dst, two states of the same n, in non-overlapping
 * buffers (same dtype: a copy).  complex128 -> complex64 rounds each
 * component to nearest.  To a fixed-point dtype each component is first
 * taken to the format's arithmetic type (float for SV_CQ16: rounded to
 * nearest; double for SV_CQ32: exact) and every block is encoded as
 * described at SV_CQ16; decoded values code * 2^scale are exact in double
 * (and in float from SV_CQ16).  Between the two fixed-point dtypes:
 * SV_ENOTSUP (convert through complex128). */
int sv_convert(const sv_state_t *dst, const sv_state_t *src, sv_stream_t st);

/* Kernel selection for sv_apply_gate. */
typedef enum sv_mode {
    SV_MODE_AUTO = 0,   /* scheduled enumeration, kernel chosen from the target */
    SV_MODE_MASKED = 1, /* baseline: all 2^(n-1) pairs, control test per pair
                           (the paper's baseline kernel figure, Sec. III-A) */
    SV_MODE_PAIR = 2,   /* scheduled, one pair per iteration (Sec. III-B) */
    SV_MODE_WAVE = 3,   /* scheduled at amplitude granularity, 64 per
                           wavefront, partner exchanged across lanes; the
                           target must be among the 6 lowest index bits that
                           are not scheduled controls */
    SV_MODE_TILE = 4    /* scheduled, LDS-staged tile of 2^m amplitudes;
                           target < m (m chosen by the library) */
} sv_mode;

/* Apply one single-qubit gate with controls (paper Sec. III and III-B).
 *   target      0 <= target < n
 *   controls    ncontrols distinct qubits in [0, n), none equal to target,
 *               in any order (the library sorts them; the skip-interval map
 *               of Sec. III-B needs them ascending); may be NULL when
 *               ncontrols == 0
 *   ctrl_vals   qubit-indexed required values; bits outside the control set
 *               must be 0
 *   U           8 doubles, host memory (converted to float for complex64)
 *   mode        sv_mode; every mode gives the same result
 * Scheduled modes launch 2^(n-1-ncontrols) pair updates; SV_MODE_MASKED
 * launches 2^(n-1) and skips the pairs whose controls fail.
 * Fixed-point states: the 64-amplitude block is the unit of work.  Controls
 * on qubits >= 6 are scheduled over the block index (2^(n-7-c_high) block
 * pairs for a target >= 6, 2^(n-6-c_high) blocks below), controls on qubits
 * < 6 are tested per amplitude; SV_MODE_MASKED visits every block (pair) and
 * tests every control, every other mode is the scheduled kernel.  Each
 * visited block is decoded, updated (SV_CQ16: float, U rounded to float;
 * SV_CQ32: double), and re-encoded as described at SV_CQ16; other blocks
 * keep their bytes. */
int sv_apply_gate(const sv_state_t *s, int target, const int32_t *controls,
                  int ncontrols, uint64_t ctrl_vals, const double *U, int mode,
                  sv_stream_t st);

/* Same gate with controls given as (ctrl_mask, ctrl_vals) bit masks. */
int sv_apply_gate_masks(const sv_state_t *s, int target, uint64_t ctrl_mask,
                        uint64_t ctrl_vals, const double *U, int mode,
                        sv_stream_t st);

/* Describe, without launching anything, the kernel sv_apply_gate would run
 * for this gate: its demangled name (written to kernel, at most kernel_len
 * bytes including the terminator; may be NULL) and its number of work items
 * (pairs for the pair kernels, 64-amplitude chunks for SV_MODE_WAVE, tiles
 * for SV_MODE_TILE; iterations may be NULL).  Host-only; needs no device. */
int sv_gate_plan(int n, int dtype, int target, uint64_t ctrl_mask,
                 uint64_t ctrl_vals, int mode, char *kernel, int kernel_len,
                 uint64_t *iterations);

/* Measurement helper (not part of the method): stream over the amplitudes
 * whose index bits match fixed_vals on fixed_mask (all amplitudes for mask
 * 0), with the access pattern of the scheduled gate kernels and no
 * arithmetic.  It measures the HBM bandwidth a gate's own address set can
 * reach and is a kernel of known traffic for calibrating profiler byte
 * counters.  op: 0 reads and writes back every selected amplitude (values
 * unchanged), 1 reads only (the state is unchanged), 2 writes zeros to the
 * selected amplitudes.  complex128 and complex64 states. */
int sv_hbm_probe(const sv_state_t *s, uint64_t fixed_mask, uint64_t fixed_vals, int op, sv_stream_t st);

/* Launch-choice knobs shared by every call of the process (not per device).
 * Keys and ranges:
 *   "granule_bits_c128", "granule_bits_c64"  [0, 6]  controls on index bits
 *       below this value are tested per pair/lane instead of scheduled (a
 *       skipped pair there shares cache lines with updated ones)
 *   "low_policy"      [0, 1]  0: such failing pairs are skipped; 1: they are
 *       read and rewritten unchanged so writes cover whole cache lines
 *   "wave_auto"       [0, 1]  SV_MODE_AUTO may choose the wavefront kernel
 *   "tile_log2_c128" [6, 13], "tile_log2_c64" [6, 14]  LDS tile width m of
 *       the fused pass and of SV_MODE_TILE (2^m amplitudes per tile)
 *   "tile_low_bits_c128" [1, 13], "tile_low_bits_c64" [1, 14]  lowest
 *       qubits every fused tile holds (runs of 2^bits contiguous amplitudes);
 *       the other tile qubits are chosen per run
 *   "fuse_min_gates"  [1, 2^20]  shortest gate run fused into one LDS pass
 *   "dense_qubits"    [4, 5]  k of dense blocks (SV_DENSE)
 *   "dense_min_gates" [1, 2^20]  shortest stretch made a dense block
 *   "pair_unroll"     1 or 4  pairs (or 64-amplitude wavefronts) per lane in
 *       large launches of the scheduled pair and wavefront kernels
 *   "masked_unroll"   1 or 4  the same for the masked baseline kernel
 *   "masked_block"    64 or 256  lanes per workgroup of the masked kernel
 *   "fuse_group"      [0, 1]  inside a fused run, move diagonal gates past
 *       gates they commute with so that they form blocks (one sweep each)
 *   "fuse_pairs"      [0, 1]  apply two adjacent pair gates of a fused run
 *       together over 4-amplitude cosets when each one's tile-local controls
 *       lie only on the other's target
 *   "plan_lookahead"  [0, 2]  pick a fused run's tile qubits one at a time,
 *       each the target that lets the run take the most of the next gates
 *       (1), or the most together with one further target (2); 0: the first
 *       targets met, in order.  Batches and one-shot calls (sv_apply_circuit,
 *       sv_adjoint_grad) plan with at most 1.
 *   "fuse_perm"       [0, 1]  apply runs of consecutive X gates (any controls)
 *       of a fused run as one permutation of the tile
 *   "batch_split"     [1, 64]  most workgroups a batched circuit may be split
 *       over (read when a batch is planned; 1: one workgroup per circuit)
 *   "phase_sweep_min_c128", "phase_sweep_min_c64" [1, 64]  a fused run's
 *       diagonal block with at least this many gates reading tile-local bits
 *       is one sweep adding phases; the gates of shorter blocks run as pair
 *       gates (fixed-point states follow their tiles' arithmetic type)
 * None of them changes results beyond floating-point rounding (fusion
 * choices change the order in which commuting operations are rounded).
 * SV_EINVAL for an unknown key or a value out of range.  Not thread-safe
 * against concurrent launches. */
int sv_tune_set(const char *key, int64_t value);
int sv_tune_get(const char *key, int64_t *value);

/* Autotuner: time candidate values of the knobs above on the current device
 * (HIP events on st, a scratch state of 2^n amplitudes of the given dtype,
 * 16 <= n <= 30) and keep the fastest: the low-control granule and policy,
 * "wave_auto", and the fused tile width and contiguous low block.  Blocking
 * (synchronises st).  When cache_path is not NULL the choice is stored there
 * as one JSON object per line, keyed by device architecture and dtype (other
 * lines are kept).  report (may be NULL) receives the timings, truncated to
 * report_len bytes including the terminator.  Results never change. */
int sv_autotune(int n, int dtype, const char *cache_path, char *report, int report_len, sv_stream_t st);

/* Apply the records of a cache written by sv_autotune that match the current
 * device's architecture (the environment variable SV_TUNE_ARCH, when set,
 * names the architecture instead; then no device is needed).  SV_EINVAL for
 * a missing file, a file without records or a malformed record. */
int sv_tune_load(const char *path);

/* ------------------------------------------------------------------ circuits
 *
 * A circuit is a sequence of gates applied in order (the paper schedules one
 * launch per gate, serially, Sec. III-A).  Gate kinds (named gates follow
 * Nielsen & Chuang; X and H as in Sec. I; R_m of the QFT is SV_G_P with angle
 * 2 pi / 2^m):
 *   SV_G_MATRIX  the 8 doubles in U
 *   SV_G_X, SV_G_Y, SV_G_Z, SV_G_H
 *   SV_G_RX, SV_G_RY, SV_G_RZ   exp(-i theta P / 2)
 *   SV_G_P       diag(1, e^{i theta})
 * OR-ing SV_G_ADJOINT into kind applies the conjugate transpose. */
typedef enum sv_gate_kind {
    SV_G_MATRIX = 0,
    SV_G_X = 1,
    SV_G_Y = 2,
    SV_G_Z = 3,
    SV_G_H = 4,
    SV_G_RX = 5,
    SV_G_RY = 6,
    SV_G_RZ = 7,
    SV_G_P = 8
} sv_gate_kind;
#define SV_G_ADJOINT 0x100

typedef struct sv_gate {
    int32_t kind;       /* sv_gate_kind, optionally | SV_G_ADJOINT */
    int32_t target;     /* 0 <= target < n */
    uint64_t ctrl_mask; /* qubit-indexed controls (target bit clear) */
    uint64_t ctrl_vals; /* required control values (subset of ctrl_mask) */
    int32_t param;      /* RX/RY/RZ/P: >= 0 takes the angle from
                           params[param] on the device at run time; -1 uses
                           theta.  Must be -1 for the other kinds. */
    int32_t reserved;   /* 0 */
    double theta;       /* angle when param < 0 */
    double U[8];        /* SV_G_MATRIX only */
} sv_gate_t;

/* Circuit flags. */
#define SV_FUSE 1    /* fuse runs of gates into one pass over LDS tiles: a
                        tile spans the lowest qubits plus qubits the planner
                        picks per run (gate fusion, the future work of
                        Sec. V); diagonal gates join a run whatever their
                        target; gates are moved only past gates they commute
                        with */
#define SV_GRAPH 2   /* capture the launch sequence once as a HIP graph and
                        replay it (per state and parameter pointer pair) */
#define SV_MASKED 4  /* every gate on the masked baseline kernel, no fusion */
#define SV_REMAP 16  /* move low qubits that control many gates (below the
                        cache-line granule, where their skips save no DRAM
                        traffic) to high bit positions: one qubit-exchange
                        pass before the circuit and one after; results are
                        the same, the state is back in the caller's layout */
#define SV_DENSE 8   /* with SV_FUSE: stretches of at least "dense_min_gates"
                        gates acting only on the "dense_qubits" lowest qubits
                        become one dense block applied with matrix cores
                        (complex128: 4 qubits; complex64: 4 or 5; n >= k+6) */

/* Write the 2x2 matrix of a gate kind (8 doubles, layout as above) for angle
 * theta; U is read for SV_G_MATRIX only (may be NULL otherwise).  Host-only. */
int sv_gate_matrix(int kind, double theta, const double *U, double *out);

typedef struct sv_circuit sv_circuit_t;

/* Validate a gate list for an n-qubit state of the given dtype, plan it
 * (fusion, kernel choice per pass) and copy it to the current device.
 * nparams is the length of the parameter array later passed to
 * sv_circuit_run (every gate's param must be < nparams).  Validation covers
 * every gate before anything is allocated, so an error names the first bad
 * gate (its index is in the message) and creates nothing.  The returned
 * handle is released with sv_circuit_destroy.  Fixed-point circuits take
 * SV_FUSE, SV_GRAPH and SV_MASKED (SV_ENOTSUP for SV_DENSE and SV_REMAP):
 * without SV_FUSE each gate runs the block-scaled gate kernel; with it, a
 * fused run decodes each tile (whole 64-amplitude blocks: the tile holds
 * qubits 0..5) to float (SV_CQ16) or double (SV_CQ32), applies the run's
 * operations as for complex64 / complex128 tiles, and re-encodes every
 * block of the tile once (as described at SV_CQ16), so blocks are rounded
 * once per pass instead of once per gate; tiles no operation of the run
 * touches keep their bytes. */
int sv_circuit_create(int n, int dtype, const sv_gate_t *gates, int ngates, int nparams, int flags,
                      sv_circuit_t **out);

/* Apply the circuit to s (same n and dtype as at creation).  params_dev is a
 * device array of nparams doubles (may be NULL when nparams == 0), read by
 * the kernels when the stream reaches them.  Calls on one handle must not
 * run concurrently with each other. */
int sv_circuit_run(sv_circuit_t *c, const sv_state_t *s, const double *params_dev, sv_stream_t st);

/* Plan statistics: number of HBM passes (fused runs + single-gate launches),
 * number of gates inside fused runs, and number of fused runs.  Any output
 * pointer may be NULL. */
int sv_circuit_info(const sv_circuit_t *c, int64_t *passes, int64_t *fused_gates, int64_t *fused_runs);

/* Host-only dry run of sv_circuit_create's planner (no device needed):
 * validates the gates and writes the execution order the plan uses
 * (order[k] = index of the k-th gate applied; gates moved ahead only past
 * gates they commute with) and the pass each belongs to (pass_of[k]; gates of
 * one fused run share a pass).  order and pass_of hold ngates entries each
 * (either may be NULL); npasses (may be NULL) receives the pass count. */
int sv_circuit_plan(int n, int dtype, const sv_gate_t *gates, int ngates, int nparams, int flags, int32_t *order,
                    int32_t *pass_of, int64_t *npasses);

/* Release the plan (waits for the device work of earlier runs to finish). */
int sv_circuit_destroy(sv_circuit_t *c);

/* Apply a dense 2^k x 2^k matrix M (host, row-major, 8 bytes per real:
 * M[a][b] at M[2(a 2^k + b)] (re) and M[2(a 2^k + b) + 1] (im)) to the k
 * lowest qubits: every row of 2^k consecutive amplitudes becomes M row.
 * Runs as a real-embedded GEMM on MFMA.  k = 4 for complex128, 4 or 5 for
 * complex64, n >= k + 6; SV_ENOTSUP otherwise. */
int sv_apply_dense_low(const sv_state_t *s, int k, const double *M, sv_stream_t st);

/* Exchange qubits: for each of the npairs disjoint pairs (pairs[2i],
 * pairs[2i+1]) the amplitude at index k moves to the index with those two
 * bits of k exchanged, all pairs at once (a relabelling of index bits, no
 * arithmetic; the basis for moving qubits between bit positions, as
 * SV_REMAP does).  Every qubit in [0, n) at most
 * once, npairs <= 32.  One read and one write of every moved amplitude. */
int sv_swap_qubits(const sv_state_t *s, const int32_t *pairs, int npairs, sv_stream_t st);

/* One-shot: create, run on st, destroy.  SV_GRAPH is ignored here. */
int sv_apply_circuit(const sv_state_t *s, const sv_gate_t *gates, int ngates, const double *params_dev,
                     int nparams, int flags, sv_stream_t st);

/* ------------------------------------------------------------ observables
 *
 * A Hamiltonian is a list of Pauli strings with real coefficients,
 * H = sum_j coef_j P_j, P_j = i^{|x&z|} X^x Z^z: bit q of x_mask (z_mask)
 * puts an X (Z) on qubit q, both bits a Y = iXZ.  Reductions are
 * deterministic (fixed grid, fixed summation order, no atomics). */
typedef struct sv_pauli {
    double coef;
    uint64_t x_mask;
    uint64_t z_mask;
} sv_pauli_t;

/* out_dev[0] = <psi|H|psi> (real), written when the stream reaches it.
 * nterms >= 1; masks must lie within the n qubits.  Any dtype: a
 * fixed-point state (SV_CQ16, SV_CQ32) is read through its codes, each
 * amplitude code * 2^scale taken exactly to double, so the result is that
 * of the decoded state (no decoded copy is made).  sv_expect_noalloc and
 * sv_expect_terms take every dtype the same way. */
int sv_expect(const sv_state_t *s, const sv_pauli_t *terms, int nterms, double *out_dev, sv_stream_t st);

/* Allocation-free variant of sv_expect, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  It writes the same out_dev[0] as sv_expect, bit for
 * bit (same kernels, same summation order), and neither allocates nor copies
 * from host memory (the term table travels as a kernel argument).  Its
 * workspace (term table and partial sums, about 1 MiB) is one device array
 * inside the library, one copy per device, held until the process ends; every
 * partial a call reads is first written by that call.  At most
 * SV_EXPECT_NOALLOC_MAX_TERMS terms (SV_EINVAL beyond).  All calls on one
 * device share the workspace, so calls that could overlap on one device
 * (other streams, other threads) race: the caller orders them.  The state
 * must be on the current device. */
#define SV_EXPECT_NOALLOC_MAX_TERMS 64
int sv_expect_noalloc(const sv_state_t *s, const sv_pauli_t *terms, int nterms, double *out_dev, sv_stream_t st);

/* out_dev[j] = <psi|P_j|psi> for every term j (coefficients not applied). */
int sv_expect_terms(const sv_state_t *s, const sv_pauli_t *terms, int nterms, double *out_dev, sv_stream_t st);

/* out = H in (out and in distinct, same n and dtype; SV_C128 or SV_C64,
 * SV_ENOTSUP for fixed-point states). */
int sv_apply_pauli_sum(const sv_state_t *in, const sv_state_t *out, const sv_pauli_t *terms, int nterms,
                       sv_stream_t st);

/* Adjoint gradient of L(theta) = <psi(theta)|H|psi(theta)> for the circuit
 * psi(theta) = U_G ... U_1 psi_0 (Jones & Gacon, arXiv:2009.02823, extended to
 * controlled gates: a controlled gate's derivative is summed over exactly the
 * control-satisfying amplitude pairs, the set scheduled in Sec. III-B).
 *   psi       in: the final forward state psi(theta); out: psi_0 recovered by
 *             un-applying every gate (the forward state is consumed)
 *   lam       workspace state of the same n and dtype (overwritten)
 *   gates     the circuit as given to sv_circuit_create; only RX/RY/RZ/P
 *             gates with param >= 0 are differentiated; every SV_G_MATRIX
 *             gate must be unitary to 1e-12 (the sweep un-applies each gate
 *             by its conjugate transpose), SV_EINVAL otherwise
 *   params_dev device array of nparams angles
 *   grad_dev  device array of nparams doubles, overwritten with dL/dtheta_j
 *             (summed over every gate using parameter j; 0 for unused ones),
 *             times scale_dev[0] when scale_dev is not NULL
 *   loss_dev  device double receiving L (may be NULL)
 * Uses two state vectors; stream-ordered, no host synchronisation. */
int sv_adjoint_grad(const sv_state_t *psi, const sv_state_t *lam, const sv_gate_t *gates, int ngates,
                    const double *params_dev, int nparams, const sv_pauli_t *terms, int nterms, double *grad_dev,
                    double *loss_dev, const double *scale_dev, sv_stream_t st);

/* A planned adjoint gradient, for differentiating the same circuit and
 * Hamiltonian many times (new angles, new states): sv_adjoint_create
 * validates the gates (as sv_adjoint_grad does, unitarity of fixed matrices
 * included) and the terms, plans the reverse sweep and uploads its tables to
 * the current device; sv_adjoint_run then enqueues exactly the work of
 * sv_adjoint_grad for states of that n and dtype (arguments as there; psi is
 * consumed), with no host planning and no allocation.  Runs of one plan
 * share its reduction buffers: enqueue them on one stream (or order them).
 * sv_adjoint_destroy waits for the device, then frees the plan; NULL is a
 * no-op. */
typedef struct sv_adjoint sv_adjoint_t;
int sv_adjoint_create(int n, int dtype, const sv_gate_t *gates, int ngates, int nparams, const sv_pauli_t *terms,
                      int nterms, sv_adjoint_t **out);
int sv_adjoint_run(sv_adjoint_t *plan, const sv_state_t *psi, const sv_state_t *lam, const double *params_dev,
                   double *grad_dev, double *loss_dev, const double *scale_dev, sv_stream_t st);
int sv_adjoint_destroy(sv_adjoint_t *plan);

/* ------------------------------------------------------------------ batches
 *
 * Many independent circuits, each on its own state (n may differ; one dtype
 * per batch), run by one persistent launch: each workgroup takes the next
 * work item from a device work queue (longest first) and applies all its
 * gates; a state of at most 64 KiB stays in LDS for the whole circuit, a
 * larger one runs its fused plan pass by pass (a fused run through LDS tiles
 * over the run's qubit set, other gates as pair loops over the state).  A
 * forward circuit that costs more than the batch's mean load per workgroup
 * is split over about cost / mean workgroups (at most the "batch_split"
 * knob): its passes are cut into chunks of whole tiles or pair-loop steps
 * that the workgroups joining it take in order, a pass's chunks starting once
 * every chunk of the earlier passes is written (device-scope counters; no
 * workgroup waits for another to arrive).  Results do not depend on the
 * split.
 *   states        ncirc state views (device buffers must not overlap)
 *   gates         all circuits' gates concatenated; circuit c owns
 *                 gates[gate_offsets[c] .. gate_offsets[c+1])
 *   params_dev    concatenated angles (device); circuit c's gate with
 *                 param p reads params_dev[param_offsets[c] + p];
 *                 param_offsets may be NULL when no gate has a parameter
 *   nparams_total length of params_dev
 * Every circuit is validated before anything is enqueued; errors name the
 * circuit. */
int sv_apply_circuits_batched(const sv_state_t *states, int ncirc, const sv_gate_t *gates,
                              const int64_t *gate_offsets, const double *params_dev, const int64_t *param_offsets,
                              int64_t nparams_total, sv_stream_t st);

/* Batched adjoint gradients: for each circuit c, psi_states[c] holds its
 * final forward state (consumed, as in sv_adjoint_grad), lam_states[c] is a
 * distinct workspace state of the same shape, its Hamiltonian is
 * terms[term_offsets[c] .. term_offsets[c+1]) (at least one term),
 * grad_dev[param_offsets[c] + j] receives dL_c/dtheta_j and loss_dev[c] the
 * loss.  One workgroup per circuit; sums are reduced in a fixed order.
 * n <= 31 per circuit. */
int sv_adjoint_grad_batched(const sv_state_t *psi_states, const sv_state_t *lam_states, int ncirc,
                            const sv_gate_t *gates, const int64_t *gate_offsets, const double *params_dev,
                            const int64_t *param_offsets, int64_t nparams_total, const sv_pauli_t *terms,
                            const int64_t *term_offsets, double *grad_dev, double *loss_dev, sv_stream_t st);

/* A planned batch kept on the device, for running the same circuits many
 * times (new angles, new states in the same buffers).  sv_batch_create
 * validates and plans every circuit (host threads for large batches) and
 * uploads the tables; the batch keeps the state pointers given here, so those
 * buffers must outlive it and keep their shapes.  Arguments are those of
 * sv_apply_circuits_batched / sv_adjoint_grad_batched; with lam_states NULL
 * (terms and term_offsets ignored) the batch only runs forward.
 *   sv_batch_run      the forward circuits (fused plan), angles from
 *                     params_dev as in sv_apply_circuits_batched
 *   sv_batch_adjoint  the batched adjoint gradients, as in
 *                     sv_adjoint_grad_batched (psi_states hold the final
 *                     forward states and are consumed)
 * Runs of one batch use one device counter: enqueue them on one stream (or
 * order them).  sv_batch_destroy waits for the last run, then frees the
 * device tables; NULL is a no-op. */
typedef struct sv_batch sv_batch_t;
int sv_batch_create(const sv_state_t *states, const sv_state_t *lam_states, int ncirc, const sv_gate_t *gates,
                    const int64_t *gate_offsets, const int64_t *param_offsets, int64_t nparams_total,
                    const sv_pauli_t *terms, const int64_t *term_offsets, sv_batch_t **out);
int sv_batch_run(sv_batch_t *b, const double *params_dev, sv_stream_t st);
int sv_batch_adjoint(sv_batch_t *b, const double *params_dev, double *grad_dev, double *loss_dev, sv_stream_t st);
int sv_batch_destroy(sv_batch_t *b);

/* Measurement helper: with stamps_dev not NULL, every later run of b writes
 * the device's constant-rate clock when a workgroup starts a work item
 * (stamps_dev[2i]) and when that workgroup has finished it (stamps_dev[2i +
 * 1]).  sv_batch_run's items are those sv_batch_info lists (i in queue
 * order); sv_batch_adjoint's are the circuits (i = c).  stamps_dev holds
 * 2 * max(ncirc, nitems) uint64 values on the batch's device and must
 * outlive those runs.  NULL turns the stamps off.  ns_per_tick (may be NULL)
 * receives the clock period in nanoseconds.  Results of the runs are
 * unchanged. */
int sv_batch_set_timing(sv_batch_t *b, uint64_t *stamps_dev, double *ns_per_tick);

/* The work items of b's forward runs: *nitems (may be NULL) receives their
 * number (ncirc plus one more per extra workgroup a split circuit may take),
 * item_circuit (host, may be NULL, cap >= nitems entries) the circuit of
 * each item in queue order.  wait_timeouts (may be NULL) receives the number
 * of chunk waits of split circuits that gave up (after 10 s; the run's
 * results are then undefined) over all runs so far: it waits for b's last
 * run.  SV_EINVAL when cap is too small. */
int sv_batch_info(sv_batch_t *b, int64_t *nitems, int32_t *item_circuit, int64_t cap, uint64_t *wait_timeouts);

/* Write, for each reduced iteration index i_r in [0, 2^(n-1-ncontrols)), the
 * index of the first pair element (bit target clear) that the scheduled
 * kernels update for it, computed with the same device function they use
 * (Sec. III-B: the reduced set mapped back to the global set, then to the
 * pair index).  out_dev is a device array of out_len >= 2^(n-1-ncontrols)
 * uint64 values; n <= 34. */
int sv_debug_pair_indices(int n, int target, const int32_t *controls,
                          int ncontrols, uint64_t ctrl_vals, uint64_t *out_dev,
                          int64_t out_len, sv_stream_t st);

#ifdef __cplusplus
}
#endif

#endif /* SV_H */
