/*
 * spod.h - C ABI of the MI355X (gfx950) SPOD library, libspod.so.
 *
 * Spectral proper orthogonal decomposition of a real snapshot matrix
 * Q in R^{M x N_t} (M = nspace * nvar degrees of freedom), following the
 * discrete SPOD of Sec. 2.3 of Rogowski et al., "Unlocking massively parallel
 * spectral proper orthogonal decompositions in the PySPOD package":
 *
 *   1. remove the long-time mean of every degree of freedom (Sec. 2.1, 2.3);
 *   2. split time into L blocks of N_f snapshots overlapping by N_overlap
 *      (eq. (blocks)), window them and take the DFT of every block in time
 *      (eq. (blocks-ft)), regrouped per frequency (eq. (blocks-k));
 *   3. form the weighted inner-product matrix M_k = Qhat_k^* W Qhat_k of the
 *      method of snapshots (eq. (spod-discrete-snapshots));
 *   4. solve M_k Psi_k = Psi_k Lambda_k for every frequency;
 *   5. build the modes Phi_k = Qhat_k Psi_k Lambda_k^{-1/2}.
 *
 * Conventions (where the paper is silent; all are fixed by this library):
 *   - DOF index m = v * nspace + s; q is row-major [M][nt] (time contiguous).
 *   - nblocks L = floor((nt - noverlap) / (nfft - noverlap)); block l covers
 *     snapshots [l*s, l*s + nfft), s = nfft - noverlap; later snapshots only
 *     enter the mean.
 *   - nfreq K = nfft/2 + 1 one-sided bins k = 0..nfft/2, DFT sign e^{-2 pi i kn/N}.
 *   - Qhat is scaled by kappa = 1/sqrt((L-1) * sum_n w[n]^2): this folds the
 *     1/(L-1) of eq. (csd-discrete) into Qhat so that the eigenvalues are those
 *     of Chat_k W and the modes satisfy Phi_k^* W Phi_k = I.
 *   - Eigenvalues descending; each eigenvector's entry of largest modulus
 *     (lowest index on ties) is real and positive.
 *   - Complex arrays are interleaved (re, im).  qhat and phi are complex128
 *     under SPOD_PREC_FP64 and complex64 otherwise; gram, psi and lam are
 *     always float64.
 *
 * Ownership and threading:
 *   - The caller allocates every device buffer, including the workspace
 *     (size from spod_plan_query).  The plan owns only its device copies of
 *     the window, the weights and the twiddle tables, made synchronously in
 *     spod_plan_create on the current device and freed by spod_plan_destroy.
 *   - Host arrays passed in are read during the call only.
 *   - Options and precision may be changed only before the first stage call;
 *     after that the plan is read-only and may be shared by concurrent streams,
 *     each with its own workspace.
 *   - Every stage call is asynchronous on `stream` (a hipStream_t; NULL is the
 *     default stream): it validates synchronously, enqueues, and returns.
 *
 * Errors: a negative spod_status is returned synchronously and nothing is
 * enqueued.  Launch failures return SPOD_ERR_HIP.  Device-side numeric
 * outcomes (Jacobi convergence, valid-mode counts) are written to the `info`
 * and `n_valid` arrays, readable after the stream is synchronised.
 * spod_last_error() returns a thread-local description of the last failure.
 * Nothing throws across this interface.
 */
#ifndef SPOD_H
#define SPOD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spod_plan_s* spod_plan;
typedef void* spod_stream; /* a hipStream_t */

typedef enum {
  SPOD_OK = 0,
  SPOD_ERR_INVALID_ARG = -1, /* bad size, pointer, dtype, window or weights        */
  SPOD_ERR_UNSUPPORTED = -2, /* valid SPOD but not implemented here (e.g. nfft)    */
  SPOD_ERR_ALLOC = -3,       /* device or host allocation failed                   */
  SPOD_ERR_HIP = -4,         /* HIP runtime error (no device, launch failure, ...) */
  SPOD_ERR_NUMERIC = -5,     /* non-finite values where finite ones are required   */
  SPOD_ERR_WORKSPACE = -6,   /* workspace missing or smaller than required         */
  SPOD_ERR_IO = -7,          /* a reader callback reported a failure               */
  SPOD_ERR_INTERNAL = -8     /* unexpected host-side failure (e.g. no thread)      */
} spod_status;

typedef enum { SPOD_F32 = 0, SPOD_F64 = 1 } spod_dtype; /* stored type of q and g_q */

/* info value of an eigenproblem whose Gram matrix is not finite (spod_eig). */
#define SPOD_INFO_NONFINITE ((int32_t)(-2147483647 - 1))

typedef enum {
  SPOD_PREC_FP64 = 0,   /* FP64 transform, Gram and modes; complex128 qhat/phi            */
  SPOD_PREC_FP32 = 1,   /* FP32 transform; Gram on FP32 MFMA, each 4-wide partial sum
                           added into FP64; FP32 modes; complex64 qhat/phi               */
  SPOD_PREC_BF16X4 = 2, /* FP32 transform; Gram on BF16 MFMA with a block floating
                           point split: per 32-wide contraction step, y 2^-E = h + l with
                           the integer h (|h| <= 2^8) and l rounded to BF16, all four
                           products (h h, h l, l h, l l); the h h sums are exact in FP32,
                           each step is scaled by 2^(2E) into FP64; FP32 modes; complex64 */
  SPOD_PREC_FP16X4 = 3  /* as BF16X4 with FP16 operands (|h| <= 2^9, l to FP16): 2^-20
                           of each step's largest operand instead of 2^-17; no range
                           scaling is needed, the step exponent E carries the range     */
} spod_precision;

typedef enum {
  SPOD_OPT_MAX_SWEEPS = 0, /* Jacobi sweep cap (default 40; 0 forces non-convergence)   */
  SPOD_OPT_GRAM_SPLIT = 1, /* slices of M per frequency in the Gram (0 = automatic)     */
  SPOD_OPT_FFT_TILE = 2,   /* degrees of freedom per transform workgroup: 16 or 32
                              (0 = automatic: 32 for nfft <= 256, else 16)            */
  SPOD_OPT_QHAT_FORMAT = 3, /* storage of qhat: SPOD_QHAT_COMPLEX (default) or
                              SPOD_QHAT_BFP20 (complex64 forms, power-of-two nfft)    */
  SPOD_OPT_MODES_KERNEL = 4, /* complex64 modes of complex qhat: 0 = vector ALU (default),
                              1 = v_mfma_f32_16x16x4f32 (FP32 products and sums)      */
  SPOD_OPT_GENERAL_PASSES = 5 /* transform of an nfft other than a power of two <= 1024:
                              0 = automatic (one pass while the block fits one
                              workgroup's LDS, else two), 1 = one pass, 2 = two passes
                              (nfft > 1024 with two factors <= 4096, else
                              SPOD_ERR_UNSUPPORTED here)                                 */
} spod_option;

/* Storage of the Fourier blocks qhat between the stages.
 *   SPOD_QHAT_COMPLEX: [K][L][M] interleaved complex (complex128 under
 *     SPOD_PREC_FP64, complex64 otherwise).
 *   SPOD_QHAT_BFP20: 20-bit block floating point, 5 bytes per complex value
 *     plus one exponent per 16 degrees of freedom (about 0.63 of complex64):
 *     row r = k * L + l occupies ceil(M / 128) superblocks of 656 bytes at byte
 *     (r * ceil(M / 128) + b) * 656.  Superblock b covers degrees of freedom
 *     128 b .. 128 b + 127 as 8 groups of 16: bytes 0..7 hold the groups'
 *     int8 exponents E (bytes 8..15 are zero); group g starts at byte
 *     16 + 80 g with the 8 pairs p (degrees of freedom 16 g + 2 p, + 1) as four
 *     int16 h at 8 p (re, im of the first, re, im of the second), then at
 *     64 + 2 p one uint16 whose nibble i (bits 4 i .. 4 i + 3) is n of value i.
 *     A value is (16 h + n) 2^E (a 20-bit two's complement mantissa, rounded to
 *     nearest, below 2^19 in magnitude); E = 127 marks a group that holds a
 *     NaN or an infinity (decoded as NaN); degrees of freedom past M are zero.
 *     Byte size from spod_plan_qhat_bytes.  Rounding: 2^-19 to 2^-20 of the
 *     group's largest value (the split forms' Gram operands carry 2^-20 of the
 *     step's largest).  spod_backward then needs qhat = NULL. */
typedef enum { SPOD_QHAT_COMPLEX = 0, SPOD_QHAT_BFP20 = 1 } spod_qhat_format;

/* Create a plan.  Follows the problem statement of Sec. 2.3: Q is M x N_t with
 * M = nspace * nvar (eq. (data-matrix)); blocks of nfft snapshots overlapping by
 * noverlap (eq. (blocks)).
 *   window  : host[nfft] or NULL for the periodic Hann window
 *             w[n] = 1/2 - 1/2 cos(2 pi n / nfft); finite, sum w^2 > 0.
 *   weights : host[nspace*nvar] diagonal of W (the spatial weighting of the
 *             inner product, eq. (innerprod_spacetime)) or NULL for 1/M each;
 *             finite, >= 0, not all zero.
 * Returns SPOD_ERR_INVALID_ARG for nspace, nvar < 1; nfft < 2; noverlap outside
 * [0, nfft); nt < nfft; L < 2; a bad window or weights; out == NULL.
 * Returns SPOD_ERR_UNSUPPORTED for nfft outside [8, 2^20].  Powers of two up
 * to 1024 take the register-resident radix-8 transform; every other nfft (the
 * paper's hourly records use 8760 = 2^3 3 5 73) takes a mixed-radix transform
 * held in LDS, up to nfft = 10240 under SPOD_PREC_FP64 (complex128 blocks)
 * and about 20400 otherwise (the block and its stage twiddles share 160 KiB
 * of LDS), with prime factors up to 1024 (SPOD_ERR_UNSUPPORTED from
 * spod_blocks_fft).  Longer blocks (the paper's ten-year blocks: 87600) take a
 * two-pass transform nfft = A B (A-point DFTs of the B columns, twiddles, then
 * B-point DFTs of the A rows; A the largest divisor <= sqrt(nfft), A and B at
 * most 4096, prime factors up to 1024; otherwise SPOD_ERR_UNSUPPORTED here)
 * whose intermediate lives in the workspace.  Validation happens before any
 * HIP call. */
spod_status spod_plan_create(int64_t nspace, int64_t nvar, int64_t nt, int64_t nfft,
                             int64_t noverlap, const double* window, const double* weights,
                             spod_plan* out);

/* Shape of a problem without creating a plan (host only, no HIP call). */
spod_status spod_shape(int64_t nt, int64_t nfft, int64_t noverlap, int64_t* nblocks,
                       int64_t* nfreq);

/* Arithmetic used by the stages (default SPOD_PREC_FP64).  Only before the first
 * stage call; SPOD_ERR_INVALID_ARG afterwards or for an unknown value. */
spod_status spod_plan_set_precision(spod_plan plan, spod_precision prec);

/* Tuning / test options (see spod_option); same timing rule as the precision. */
spod_status spod_plan_set_option(spod_plan plan, spod_option opt, int64_t value);

/* Bytes of one qhat buffer of this plan in its storage format. */
spod_status spod_plan_qhat_bytes(spod_plan plan, size_t* bytes);

/* nblocks L, nfreq K and the workspace size (bytes) that every stage call of
 * this plan accepts.  Any output pointer may be NULL. */
spod_status spod_plan_query(spod_plan plan, int64_t* nblocks, int64_t* nfreq,
                            size_t* workspace_bytes);

/* Steps 1-2 (Sec. 2.3; eqs. (blocks), (blocks-ft), (blocks-k); step 2 of the
 * algorithm of Sec. 3.1): temporal mean, windowed DFT of every block.
 *   q     : device [M][nt] of `dtype`.
 *   qhat  : device [K][L][M] complex (complex128 for SPOD_PREC_FP64, else
 *           complex64); qhat[k][l][m] = kappa * sum_n w[n](q[m][l s + n] - mean[m])
 *           e^{-2 pi i k n / nfft}.
 *   mean  : device [M] float64 or NULL; the long-time mean, accumulated in FP64.
 *   ws    : device workspace of ws_bytes >= spod_plan_query's size. */
spod_status spod_blocks_fft(spod_plan plan, const void* q, spod_dtype dtype, void* qhat,
                            double* mean, void* ws, size_t ws_bytes, spod_stream stream);

/* Steps 3-4 (eq. (spod-discrete-snapshots); Sec. 3.1 steps 3-4): the weighted
 * inner product of the method of snapshots for every frequency,
 *   gram[k][i][j] = sum_m conj(qhat[k][i][m]) W_m qhat[k][j][m]
 * (complex128 [K][L][L], Hermitian).  The sum over m, which the paper reduces
 * across MPI ranks, is split across workgroups and combined in FP64.
 * Up to 64 blocks a workgroup computes every 16 x 16 block pair of its
 * frequency and slice; up to 160 blocks (the paper's jet analysis has 155) the
 * pairs are spread over several workgroups (SPOD_PREC_FP64, BF16X4, FP16X4 with
 * complex qhat; SPOD_ERR_UNSUPPORTED for FP32 or packed qhat there, and for
 * nblocks > 160). */
spod_status spod_csd(spod_plan plan, const void* qhat, void* gram, void* ws, size_t ws_bytes,
                     spod_stream stream);

/* Bytes of device scratch the library holds for spod_csd_noalloc, per device. */
#define SPOD_CSD_NOALLOC_MAX_BYTES ((size_t)64 << 20)

/* spod_csd for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops that must not call hipMalloc, harnesses that
 * forbid it): the same weighted inner product, with the Gram partials in a
 * static device array of the library (SPOD_CSD_NOALLOC_MAX_BYTES = 64 MiB on
 * every device the library runs on, held until the process ends) instead of a
 * workspace.  The caller still passes qhat and gram as for spod_csd.  The
 * number of slices of M is the plan's, reduced to what fits the array; it is
 * written to *slices when slices != NULL (0 when even one slice does not fit).
 * Calls no allocation routine.  Calls that overlap on one device (several
 * streams, several host threads) share the array and race: the caller must
 * order them.  Results differ from spod_csd's only in the FP64 summation order
 * of the slices, and are identical when the slice counts agree.
 * SPOD_ERR_UNSUPPORTED when one slice of partials, nfreq * (16 ceil(nblocks /
 * 16))^2 * 16 bytes, exceeds the array. */
spod_status spod_csd_noalloc(spod_plan plan, const void* qhat, void* gram, int64_t* slices,
                             spod_stream stream);

/* Step 5 (eq. (spod-discrete-snapshots); Sec. 3.1 step 5): eigendecomposition
 * of every Hermitian gram[k] by cyclic Jacobi in FP64.  One workgroup per
 * frequency; A and V live in LDS up to 64 blocks and in the workspace (size
 * from spod_plan_query; required then) up to 160.
 *   lam  : device [K][L] float64, descending.
 *   psi  : device [K][L][L] complex128; psi[k][i][j] = component i of
 *          eigenvector j (unit 2-norm, phase convention above).
 *   info : device [K] int32 or NULL: > 0 converged, the number of sweeps
 *          used (the last one made no rotation); <= 0 not converged after
 *          -info sweeps (the cap set with SPOD_OPT_MAX_SWEEPS was reached);
 *          SPOD_INFO_NONFINITE when gram[k] holds a NaN or an infinity (from
 *          non-finite data): lam[k][*] and psi[k] are then written as NaN, and
 *          spod_modes counts no valid mode for k (its modes are zero).
 * The stage calls are asynchronous, so a non-finite input is reported here,
 * after a stream synchronisation, and not as a status; the synchronous
 * out-of-core call returns SPOD_ERR_NUMERIC for it. */
spod_status spod_eig(spod_plan plan, const void* gram, double* lam, void* psi, int32_t* info,
                     void* ws, size_t ws_bytes, spod_stream stream);

/* Modes (eq. (spod-discrete-snapshots)): for j < n_modes (1 <= n_modes <= L)
 *   phi[k][j][m] = sum_l qhat[k][l][m] psi[k][l][j] / sqrt(lam[k][j])
 * when lam[k][0] > 0 and lam[k][j] > eps * lam[k][0] (eps = 1e-12 for
 * SPOD_PREC_FP64, 1e-6 otherwise); otherwise phi[k][j][:] = 0.
 *   phi     : device [K][n_modes][M], complex type of qhat.
 *   n_valid : device [K] int32 or NULL: number of valid modes per frequency. */
spod_status spod_modes(spod_plan plan, const void* qhat, const double* lam, const void* psi,
                       int64_t n_modes, void* phi, int32_t* n_valid, void* ws, size_t ws_bytes,
                       spod_stream stream);

/* Adjoint of steps 1-5 (not in the paper): the gradient of a real loss E with
 * respect to the raw data q, given the gradients with respect to the outputs
 * of spod_eig and spod_modes.  Complex gradients follow the convention
 * dE/dRe + i dE/dIm.
 *   q      : device [M][nt] of `dtype`; only read when qhat is NULL.
 *   dtype  : SPOD_F32 or SPOD_F64; the type of q and of g_q.
 *   qhat   : device [K][L][M], the output of spod_blocks_fft for the same q,
 *            or NULL: the Fourier blocks are then recomputed from q (at the
 *            selected bins only) into g_qhat, so nothing of size K*L*M needs
 *            to be kept from the forward pass.
 *   lam, psi : the outputs of spod_eig for the same q.
 *   g_lam  : device [n_bins][L] float64 (dE/dlam at the selected bins) or NULL
 *            (zero).
 *   g_phi  : device [n_bins][n_modes][M] in phi's complex type (dE/dphi at the
 *            selected bins), or NULL (zero; n_modes is then ignored).
 *   bins   : host [n_bins] strictly increasing frequencies in [0, K): row s of
 *            g_lam, g_phi and g_qhat belongs to frequency bins[s], and the
 *            gradients at every other frequency are zero.  Copied during the
 *            call.  NULL means all K frequencies in order (n_bins ignored).
 *   g_qhat : device [n_bins][L][M] scratch of qhat's complex type (n_bins = K
 *            when bins is NULL): receives dE/dqhat at the selected bins.  With
 *            bins == NULL it may be the same buffer as qhat (qhat is then
 *            overwritten); with a selection it must not overlap qhat.
 *   g_q    : device [M][nt] of `dtype`: receives dE/dq (every entry written).
 * The chain, per selected frequency: modes adjoint (Phi = Qhat Psi
 * Lambda^{-1/2}); derivative of the phase convention of spod_eig; eigenvector
 * and eigenvalue adjoint of M_k (distinct-eigenvalue formula: pairs closer
 * than 1e-12 of the largest eigenvalue contribute nothing); Gram adjoint
 * 2 W Qhat G; then the adjoint of the windowed one-sided DFT, the overlap-add
 * of the blocks and the mean removal.  Modes that spod_modes zero-fills are
 * constants here.  Power-of-two nfft in [16, 1024] needs a hop nfft - noverlap
 * of nfft/4, nfft/2 or nfft.  Any other nfft the forward supports (the
 * mixed-radix transform, any hop) runs the adjoint of that transform and
 * needs qhat (no recomputation) and at most 513 bins (bins may be NULL only
 * when nfreq <= 513).  Returns SPOD_ERR_UNSUPPORTED otherwise, for nfft < 16,
 * or when nblocks > 64. */
spod_status spod_backward(spod_plan plan, const void* q, spod_dtype dtype, const void* qhat,
                          const double* lam, const void* psi, const double* g_lam,
                          const void* g_phi, int64_t n_modes, const int32_t* bins,
                          int64_t n_bins, void* g_qhat, void* g_q, void* ws, size_t ws_bytes,
                          spod_stream stream);

/* ------------------------------------------------------------------------
 * Batches: many independent problems of uneven shapes (not in the paper; the
 * paper runs one problem per job).  A batch owns one plan per problem, all
 * with the same precision.  A forward pass enqueues the five steps for every
 * problem with one launch per step and shape group (problems that share N_f
 * for the transform, ceil(L/16) for the Gram; all problems for the mean-free
 * bookkeeping, eigensolve and modes): workgroup b of a grouped launch finds
 * its problem in a device work table.  By default the launches are captured
 * once into a hipGraph and replayed.
 * ------------------------------------------------------------------------ */
typedef struct spod_batch_s* spod_batch;

typedef struct {
  int64_t nspace, nvar, nt, nfft, noverlap;
  const double* window;   /* host [nfft], copied; NULL = periodic Hann            */
  const double* weights;  /* host [nspace*nvar], copied; NULL = 1/M for every DOF */
} spod_problem;

typedef struct {
  int64_t M, nblocks, nfreq, n_modes; /* n_modes = min(requested, nblocks) */
  /* byte offsets of this problem's results in the output buffer `out`:
   * mean [M] f64, lam [K][L] f64, psi [K][L][L] c128, info [K] int32,
   * phi [K][n_modes][M] (c128 under SPOD_PREC_FP64, else c64), n_valid [K] int32 */
  size_t mean, lam, psi, info, phi, n_valid;
} spod_batch_item;

typedef enum {
  SPOD_BATCH_GROUPED = 0,     /* 1 (default): grouped launches; 0: one launch per problem and step */
  SPOD_BATCH_GRAPH = 1,       /* 1 (default): capture into a hipGraph on first use and replay      */
  SPOD_BATCH_GRAM_TARGET = 2, /* Gram workgroups aimed at per problem (default 8192, >= 64)       */
  SPOD_BATCH_FFT_TILE = 3,    /* DOFs per transform workgroup: 0 (default: 32 up to nfft 256,
                                 else 16), 16 or 32; results do not depend on it              */
  SPOD_BATCH_EIG_THREADS = 4, /* threads per eigenproblem: 0 (default: 1024 above 32 blocks,
                                 else 256), 256 or 1024; results do not depend on it          */
  SPOD_BATCH_PERSISTENT = 5   /* 1: persistent workgroups (as many as the device holds) take the
                                 work units of every grouped stage from a device queue, zeroed
                                 by a kernel at the start of each pass; 0 (default): one
                                 workgroup per unit.  Results do not depend on it            */
} spod_batch_option;

/* Create plans for problems[0..n) on the current device (n >= 1).  Every
 * problem is validated as in spod_plan_create; the first failure is returned
 * and nothing is kept. */
spod_status spod_batch_create(const spod_problem* problems, int64_t n, spod_precision precision,
                              int64_t n_modes, spod_batch* out);

/* Options, before the first forward pass or autotune. */
spod_status spod_batch_set_option(spod_batch batch, spod_batch_option opt, int64_t value);

/* The current value of an option (after spod_batch_autotune: its choice). */
spod_status spod_batch_get_option(spod_batch batch, spod_batch_option opt, int64_t* value);

/* Bytes of the device workspace (Fourier blocks, Gram partials and Grams of
 * every problem) and of the output buffer. */
spod_status spod_batch_query(spod_batch batch, size_t* workspace_bytes, size_t* output_bytes);

/* Shape and result offsets of problem i. */
spod_status spod_batch_item_info(spod_batch batch, int64_t i, spod_batch_item* item);

/* Forward pass of every problem.  q: host array of n device pointers, problem
 * i's snapshots [M_i][nt_i] of `dtype` (one dtype for the batch).  out, ws:
 * device buffers of the queried sizes, 256-byte aligned.  When q, out or ws
 * differ from the previous call the work tables are rebuilt (a synchronous
 * copy) and the graph is captured again.  Calls on one batch must not
 * overlap.  With grouped launches, the problems with more than 32 blocks run
 * on a second stream that the batch owns, forked from `stream` (after all
 * work already queued on it) and joined back into it before the call's work
 * ends, so the caller sees one stream either way. */
spod_status spod_batch_forward(spod_batch batch, const void* const* q, spod_dtype dtype,
                               void* out, void* ws, size_t ws_bytes, spod_stream stream);

/* Choose the launch shapes by timing grouped forward passes (no graph; the
 * best of two timed passes per candidate) on these buffers, one shape at a
 * time from the defaults: SPOD_BATCH_GRAM_TARGET over 2048, 4096, 8192 and
 * 16384 workgroups per problem, then SPOD_BATCH_FFT_TILE over 16 and 32, then
 * SPOD_BATCH_EIG_THREADS over 256 and 1024, then SPOD_BATCH_PERSISTENT = 1;
 * each is kept when it is faster.  With cache_path != NULL the choice is read
 * from (when its key, a hash of the problem shapes and precision, is present)
 * or appended to that JSON-lines file, one line with the chosen shapes and
 * every candidate's time in ms.  Synchronises the stream.  *chosen (nullable)
 * receives the Gram target; spod_batch_get_option reads the others. */
spod_status spod_batch_autotune(spod_batch batch, const void* const* q, spod_dtype dtype,
                                void* out, void* ws, size_t ws_bytes, spod_stream stream,
                                const char* cache_path, int64_t* chosen);

/* Free the batch and its plans (NULL-safe; synchronises the device). */
void spod_batch_destroy(spod_batch batch);

/* ---------------------------------------------------------------------------
 * Expansion coefficients and reconstruction (SPOD for data compression,
 * eq. (coeffs) and eq. (SPODrec)).  Phi_r gathers the retained modes arranged
 * by frequency as in eq. (discrete_modes): column r = i * n_r + j is mode j of
 * frequency bins[i].  With R = n_bins * n_r retained modes:
 *
 *   A  = (Phi_r^* W Phi_r)^{-1} Phi_r^* W (Q - qbar 1^T)     (R x N_t)
 *   Q~ = Re(Phi_r A) + qbar 1^T                               (M x N_t)
 *
 * The mean is removed before the projection and added back after it (the
 * modes describe the fluctuations); only the one-sided frequencies are
 * retained, so the reconstruction of real data is the real part.  Every
 * product runs in FP64 (complex64 modes and float32 snapshots are widened
 * as they are read); Phi_r^* W Phi_r is factored by Cholesky, so every
 * retained mode must be valid (n_r <= n_valid at each retained bin).
 * ------------------------------------------------------------------------ */

/* Workspace bytes of spod_coeffs for R = n_bins * n_r in [1, 1024]. */
spod_status spod_coeffs_query(spod_plan plan, int64_t n_bins, int64_t n_r, size_t* workspace);

/* A = (Phi_r^* W Phi_r)^{-1} Phi_r^* W (Q - qbar 1^T)  (eq. (coeffs)).
 *   q      : device [M][nt] of dtype (the snapshots the modes came from, or
 *            any others of the same shape);
 *   mean   : device [M] f64 (the long-time mean from spod_blocks_fft);
 *   phi    : device [K][n_modes][M], complex128 under SPOD_PREC_FP64 else
 *            complex64 (spod_modes' output);
 *   bins   : host [n_bins], strictly increasing in [0, K), read during the call;
 *   n_r    : modes kept per retained frequency, in [1, n_modes];
 *   a      : device [R][nt] in phi's complex type (row r = coefficient of
 *            column r of Phi_r over time);
 *   info   : device [1] int32: 0, or j + 1 when pivot j of the Cholesky
 *            factorisation is not positive (a retained mode is zero or the
 *            retained modes are linearly dependent); a is then zero;
 *   ws     : device workspace of spod_coeffs_query's size.
 * Asynchronous on stream.  SPOD_ERR_UNSUPPORTED when R > 1024. */
spod_status spod_coeffs(spod_plan plan, const void* q, spod_dtype dtype, const double* mean,
                        const void* phi, int64_t n_modes, const int32_t* bins, int64_t n_bins,
                        int64_t n_r, void* a, int32_t* info, void* ws, size_t ws_bytes,
                        spod_stream stream);

/* Q~ = Re(Phi_r A) + qbar 1^T  (eq. (SPODrec)).  phi, bins, n_r as in
 * spod_coeffs; a: device [R][nt] in phi's complex type; mean: device [M] f64;
 * q_rec: device [M][nt] of dtype.  Asynchronous on stream; needs no
 * workspace. */
spod_status spod_reconstruct(spod_plan plan, const void* phi, int64_t n_modes, const int32_t* bins,
                             int64_t n_bins, int64_t n_r, const void* a, const double* mean,
                             void* q_rec, spod_dtype dtype, spod_stream stream);

/* ---------------------------------------------------------------------------
 * Out-of-core SPOD: the snapshot matrix stays in host memory (or behind a
 * reader) and reaches the device in chunks of rows.  This is the spatial
 * split of Sec. 3.1 (every process owns a slice of the degrees of freedom and
 * its share of Qhat_k^* W Qhat_k adds up to the Gram of
 * eq. (spod-discrete-snapshots)) run through one device, with the chunked
 * reading of the data that Sec. 3.1 describes.
 *
 *   pass 1: for every chunk: copy it in, mean + blocks + DFT, add its
 *           weighted Gram into the Gram of every frequency;
 *   then:   the eigensolve of every frequency (spod_eig);
 *   pass 2: for every chunk: blocks + DFT again, the modes of its rows
 *           (eq. (discrete_modes) is row by row), copy them out.
 *
 * Copies run on library-owned streams (default priority) and overlap the
 * kernels of the previous chunk: two device slots take the streamed chunks in
 * turn.  The last `resident` chunks of pass 1 get slots of their own and stay
 * on the device, so pass 2 reads only the other chunks again; with
 * resident >= the number of chunks the host data crosses the link once.
 * Results equal the in-memory path's up to the order of the Gram sums
 * (bit-identical with one chunk).
 * ------------------------------------------------------------------------ */
typedef struct spod_ooc_s* spod_ooc;

/* Reader: fill dst (pinned host memory, [nrows][nt] of the object's dtype,
 * row-major) with rows [row0, row0 + nrows) of Q.  Return 0 on success; any
 * other value stops the forward pass with SPOD_ERR_IO. */
typedef int (*spod_read_fn)(void* user, int64_t row0, int64_t nrows, void* dst);

/* Create an out-of-core driver for `plan` (which must outlive it; its
 * precision and options are used as they are).  dtype: stored type of Q.
 * chunk_rows: rows per chunk, rounded up to a multiple of 256 (>= 1; values
 * >= M give one chunk).  n_modes in [1, nblocks].  resident in [0, ...):
 * chunks kept on the device between the passes.  Allocates every device
 * buffer and the streams now (on the plan's device, which must be current);
 * pinned host staging buffers are allocated on the first forward pass that
 * needs them.  SPOD_ERR_UNSUPPORTED when nblocks > 160. */
spod_status spod_ooc_create(spod_plan plan, spod_dtype dtype, int64_t chunk_rows,
                            int64_t n_modes, int64_t resident, spod_ooc* out);

/* Chunk rows after rounding, number of chunks, chunks kept resident, bytes of
 * device memory held by the object and of pinned host memory it may allocate
 * (all pointers nullable). */
spod_status spod_ooc_query(spod_ooc ooc, int64_t* chunk_rows, int64_t* n_chunks,
                           int64_t* n_resident, size_t* device_bytes, size_t* pinned_bytes);

/* One SPOD of Q.  Exactly one source:
 *   q     : [M][nt] of dtype, row-major.  Device memory or pinned host memory
 *           is copied from directly; other host memory is copied through
 *           pinned staging buffers by host threads;
 *   read  : called in row order, twice per chunk that is not resident (once
 *           per pass), on the calling thread, with user passed through.
 * Outputs:
 *   mean  : [M] f64, host or device memory;
 *   lam   : device [K][L] f64;  psi: device [K][L][L] c128;  info: device [K]
 *           int32 (as spod_eig) or NULL;
 *   phi   : [K][n_modes][M], c128 under SPOD_PREC_FP64 else c64, host (pinned
 *           or not) or device memory;
 *   n_valid: device [K] int32 (as spod_modes).
 * `stream` runs the kernels and is waited on before the first copy.  The call
 * returns after every result is in place (it synchronises the streams).  On
 * an error nothing is left running; the outputs are then undefined.  Calls on
 * one object must not overlap.  SPOD_ERR_NUMERIC when the data hold a NaN or
 * an infinity: every output is still written, and the frequencies concerned
 * carry SPOD_INFO_NONFINITE in info (NaN eigenpairs, no valid mode). */
spod_status spod_ooc_forward(spod_ooc ooc, const void* q, spod_read_fn read, void* user,
                             double* mean, double* lam, void* psi, int32_t* info, void* phi,
                             int32_t* n_valid, spod_stream stream);

/* Free the object's device and pinned buffers, streams and events
 * (NULL-safe; synchronises its streams). */
void spod_ooc_destroy(spod_ooc ooc);

/* Free the plan's device copies.  NULL-safe.  Synchronises the plan's device. */
void spod_plan_destroy(spod_plan plan);

/* Static description of a status code. */
const char* spod_status_string(spod_status status);

/* Thread-local description of the last non-OK status returned on this thread. */
const char* spod_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SPOD_H */
