// Internal declarations shared by the libspod sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <exception>
#include <new>
#include <string>

#include "spod.h"

namespace spod {

// --------------------------------------------------------------------------
// plan
// --------------------------------------------------------------------------
// Radix factorisation of N_f for the general transform (radices 8, 4, 2, 3,
// 5, 7, then any remaining primes in increasing order).  For an odd radix,
// kpt is the number of output pairs one work item computes and toff the
// offset of the stage's table of W_r^{jk} in the plan's d_oddw (entries);
// both are 0 for the radices 2, 4 and 8.
struct Radices {
  int n = 0;
  int r[32] = {};
  int kpt[32] = {};
  int toff[32] = {};
};
// Output pairs per work item of an odd stage of radix r with nb butterflies
// (from a cost model of the stage's instructions per SIMD).
int general_odd_kpt(int r, int nb);
// Entries of the odd stage's table: G (h - 1) kpt with h = (r + 1) / 2 and
// G = ceil(h / kpt).
int general_odd_entries(int r, int kpt);
constexpr int GENERAL_MAX_KPT = 6;
constexpr int SPOD_MAX_NBLOCKS = 160;          // Gram, eigensolve and modes (backward, batch: 64)
constexpr int SPOD_SMALL_NBLOCKS = 64;         // above this: the L > 64 kernels
constexpr int SPOD_GENERAL_MAX_NFFT = 20480;   // complex64 blocks of one transform fill 160 KiB LDS
constexpr int64_t SPOD_LONG_MAX_NFFT = int64_t(1) << 20;   // two-pass transform (N = A B) above that
constexpr int SPOD_LONG_MAX_FACTOR = 4096;     // A, B: the sub-transform lengths

struct Plan {
  int64_t nspace = 0, nvar = 0, M = 0, nt = 0, nfft = 0, noverlap = 0, step = 0;
  int64_t nblocks = 0, nfreq = 0;
  spod_precision prec = SPOD_PREC_FP64;
  int device = 0;
  bool frozen = false;  // set by the first stage call

  double kappa = 0.0;   // 1/sqrt((L-1) sum w^2)

  // Bins where the window's own DFT  What_k = sum_n w[n] e^{-2 pi i k n / N}
  // is not zero (k = 0, 1 for the periodic Hann window).  When there are at
  // most SPOD_MAX_MEAN_BINS of them, the transform removes the mean in the
  // same pass over q (see fft.hip); otherwise it runs a separate mean pass.
  static constexpr int SPOD_MAX_MEAN_BINS = 4;
  int n_mean_bins = -1;                    // -1: too many, use the separate pass
  int mean_bin[SPOD_MAX_MEAN_BINS] = {0, 0, 0, 0};
  double what_re[SPOD_MAX_MEAN_BINS] = {0, 0, 0, 0};
  double what_im[SPOD_MAX_MEAN_BINS] = {0, 0, 0, 0};

  // N_f not a power of two in [8, 1024]: the general transform and its radices
  bool general = false;
  Radices radices;
  // N_f above SPOD_GENERAL_MAX_NFFT (complex128: half): the two-pass
  // transform N = A B (four-step: A-point DFTs of the B columns, twiddles
  // W_N^{c k1}, B-point DFTs of the A rows), with the rows and columns in LDS
  // and the intermediate [A][B] in a workspace slot per workgroup
  bool long_dft = false;
  int long_a = 0, long_b = 0;       // A <= B
  int long_ga = 0, long_gb = 0;     // columns, rows per LDS batch
  int long_grid = 0;                // workgroups (one per CU)
  Radices rad_a, rad_b;

  // options
  int max_sweeps = 40;
  int64_t gram_split_opt = 0;
  int64_t fft_tile_opt = 0;
  bool qhat_packed = false;   // SPOD_QHAT_BFP20: qhat in the packed layout below
  bool modes_mfma = false;    // complex64 modes on the matrix cores (SPOD_OPT_MODES_KERNEL)
  int general_passes = 0;     // SPOD_OPT_GENERAL_PASSES: 0 automatic, 1 or 2

  // derived launch shapes (fixed when frozen)
  int gram_split = 1;       // slices of M per frequency
  int gram_dim = 0;         // L rounded up to a multiple of 16 (Gram tile size)
  size_t ws_bytes = 0;

  // device copies owned by the plan
  double* d_window = nullptr;  // [nfft]
  float* d_window32 = nullptr; // [nfft]
  double* d_weights = nullptr; // [M]
  double* d_sqrtw = nullptr;   // [M]
  double2* d_what = nullptr;   // [K] DFT of the window, What_k
  float* d_sqrtw32 = nullptr;  // [M]
  double2* d_tw64 = nullptr;   // [nfft] e^{-2 pi i j / nfft}
  float2* d_tw32 = nullptr;    // [nfft]
  // general transform: per odd stage, T[g][j][c] = W_r^{(j + 1) k}, k =
  // min(g + c G, (r - 1) / 2), for g < G, j < (r - 1) / 2, c < kpt
  double2* d_oddw64 = nullptr;
  float2* d_oddw32 = nullptr;
  // two-pass transform: W_A^t, W_B^t and the odd stages' tables of A and B
  double2* d_tw_a64 = nullptr;
  float2* d_tw_a32 = nullptr;
  double2* d_tw_b64 = nullptr;
  float2* d_tw_b32 = nullptr;
  double2* d_oddw_a64 = nullptr;
  float2* d_oddw_a32 = nullptr;
  double2* d_oddw_b64 = nullptr;
  float2* d_oddw_b32 = nullptr;
};

bool is_complex128(const Plan& p);
size_t qhat_bytes(const Plan& p);   // bytes of one plan's qhat in its format
int64_t gram_split_for(const Plan& p, int64_t target);   // slices for ~target workgroups
void plan_set_gram_split(Plan& p, int64_t s);            // internal: owner of the plan only
size_t workspace_bytes(const Plan& p);
void freeze(Plan& p);
// A view of rows [row0, row0 + rows) of p's degrees of freedom: the same
// tables offset to row0, launch shapes derived for `rows` (no allocation; the
// view must not outlive p and is never destroyed).
Plan plan_rows(const Plan& p, int64_t row0, int64_t rows);

// error reporting (thread local message)
// Record the message of a failing call (spod_last_error) and return s.
spod_status fail(spod_status s, const char* msg) noexcept;
spod_status fail(spod_status s, const std::string& msg) noexcept;
spod_status hip_fail(hipError_t e, const char* where) noexcept;

// Runs an entry point's body so that no exception crosses the C ABI: host
// allocation failures become SPOD_ERR_ALLOC, anything else SPOD_ERR_INTERNAL.
template <typename F>
spod_status guarded(F&& body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    return fail(SPOD_ERR_ALLOC, "host memory");
  } catch (const std::exception& e) {
    return fail(SPOD_ERR_INTERNAL, e.what());
  } catch (...) {
    return fail(SPOD_ERR_INTERNAL, "unexpected exception");
  }
}

// --------------------------------------------------------------------------
// stage launchers (each returns SPOD_OK or an error, never throws)
// --------------------------------------------------------------------------
// Optional frequency selection of the block transform: output row s holds
// frequency d_sel[s] (device table, nsel rows); h_slot[k] (host, nfreq
// entries) is the row of frequency k or -1.  d_sel == NULL: all frequencies.
struct FftSel {
  const int* d_sel = nullptr;
  int nsel = 0;
  const int* h_slot = nullptr;
};

spod_status launch_blocks_fft(const Plan& p, const void* q, spod_dtype dtype, void* qhat,
                              double* mean, void* ws, hipStream_t st, const FftSel& fs = FftSel{});
// accumulate: gram += Qhat^* W Qhat instead of gram = ...
// the transform of steps 1-2 for any N_f (mean from the FP64 mean pass)
spod_status launch_blocks_dft_general(const Plan& p, const void* q, spod_dtype dtype,
                                      const double* mean, void* qhat, hipStream_t st);
// the two-pass transform (p.long_dft); scratch: p.long_grid * N complex
spod_status launch_blocks_dft_long(const Plan& p, const void* q, spod_dtype dtype,
                                   const double* mean, void* qhat, void* scratch, hipStream_t st);
size_t long_scratch_bytes(const Plan& p);
// Adjoint of that transform (and of the mean removal) for the selected bins:
// g_q = dE/dq from g_qhat = dE/dqhat [bins.n][L][M].  bins: strictly
// increasing frequencies; mean: the selected bins whose window DFT is not
// zero (slot into the selection and What_k), or n < 0 for every selected bin
// with the plan's What table.
constexpr int GEN_ADJ_MAXB = 513;
struct GenAdjBins {
  int n;
  int16_t k[GEN_ADJ_MAXB];
};
struct GenAdjMean {
  int n;
  int slot[Plan::SPOD_MAX_MEAN_BINS];
  double wr[Plan::SPOD_MAX_MEAN_BINS], wi[Plan::SPOD_MAX_MEAN_BINS];
};
spod_status launch_general_adjoint(const Plan& p, const void* g_qhat, spod_dtype dtype, void* g_q,
                                   const GenAdjBins& bins, const GenAdjMean& mean, hipStream_t st);
spod_status launch_csd(const Plan& p, const void* qhat, void* gram, void* ws, hipStream_t st,
                       bool accumulate = false);
// spod_csd with the partials in the library's static device scratch (no
// allocation); csd_noalloc_split: the slice count it uses (0: does not fit)
spod_status launch_csd_noalloc(const Plan& p, const void* qhat, void* gram, hipStream_t st);
int64_t csd_noalloc_split(const Plan& p);
spod_status launch_eig(const Plan& p, const void* gram, double* lam, void* psi, int32_t* info,
                       void* ws, hipStream_t st);
spod_status launch_modes(const Plan& p, const void* qhat, const double* lam, const void* psi,
                         int n_modes, void* phi, int32_t* n_valid, void* ws, hipStream_t st);
spod_status launch_backward(const Plan& p, const void* q, spod_dtype dtype, const void* qhat,
                            const double* lam, const void* psi, const double* g_lam,
                            const void* g_phi, int n_modes, const int32_t* bins, int n_bins,
                            void* g_qhat, void* g_q, void* ws, hipStream_t st);

// nrow rows of width_bytes from a packed device buffer to dst with row stride
// dpitch_bytes (device memory, or pinned host memory through its device
// address); 8-byte units and alignment
spod_status launch_store_rows(const void* src, void* dst, size_t width_bytes, size_t dpitch_bytes,
                              int64_t nrow, hipStream_t st);

// Expansion coefficients and reconstruction: the retained modes (mode j < n_r
// of every frequency bin[i], column i * n_r + j of Phi_r) and the workspace
// layout of one problem with R = n_bins * n_r columns.
struct CoeffSel {
  static constexpr int MAX_BINS = 513;
  static constexpr int MAX_R = 1024;
  int n_bins = 0, n_r = 0, n_modes = 0;
  int bin[MAX_BINS] = {};
};
struct CoeffLayout {
  int R = 0, S_rhs = 1, S_gram = 1;   // columns, slices of M for C and for B
  size_t off_B = 0, off_C = 0, off_part = 0, off_X = 0, bytes = 0;
};
CoeffLayout coeff_layout(const Plan& p, int R);
spod_status launch_coeffs(const Plan& p, const void* q, spod_dtype dtype, const double* mean,
                          const void* phi, const CoeffSel& cs, void* a, int32_t* info, void* ws,
                          hipStream_t st);
spod_status launch_reconstruct(const Plan& p, const void* phi, const CoeffSel& cs, const void* a,
                               const double* mean, void* qrec, spod_dtype dtype, hipStream_t st);

// workspace sizes of the individual stages
size_t fft_workspace(const Plan& p);  // only used when the caller passes no mean buffer
size_t csd_workspace(const Plan& p);
size_t backward_workspace(const Plan& p);
size_t eig_workspace(const Plan& p);  // A and V of every frequency for L > 64

// --------------------------------------------------------------------------
// grouped (batched) launches: one launch covers the workgroups of several
// problems; item i owns workgroups [start_i, start_{i+1}) of the grid
// --------------------------------------------------------------------------
// Bins whose window DFT What_k is non-zero, for the single-pass mean removal.
struct MeanBins {
  int n;
  int k[4];
  double wr[4], wi[4];
};

struct FftItem {                 // blocks_fft, fused mean, all blocks per tile
  const void* q;
  double* mean;
  const double* window;
  const void* tw;
  void* qhat;
  int64_t M, ldq, nt;            // ldq: row stride of qhat (>= M)
  int step, L;
  double kappa;
  MeanBins mb;
  int start;
};

struct GramItem {                // gram partials, work unit = (slice, k)
  const void* qhat;
  const void* sqrtw;
  double* part;
  int64_t M, ldq;
  int L, S, K, vec;
  int start;
};

struct CombineItem {             // gram_combine, work unit = k
  const void* part;              // partials [K][S][D][D]
  void* gram;                    // [K][L][L]
  int L, D, S;
  int start;
};

struct EigItem {                 // jacobi, work unit = k
  const void* gram;
  double* lam;
  void* psi;
  int32_t* info;
  int L;
  int start;
};

struct ModesItem {               // modes, work unit = (k, tile of 256 DOFs)
  const void* qhat;
  const double* lam;
  const void* psi;
  void* phi;
  int32_t* n_valid;
  int64_t M, ldq;
  int L, n_modes, tiles;
  int pair;                      // two DOFs per thread (complex64, even M, aligned)
  double eps;
  int start;
};

// index of the item that owns workgroup b (items sorted by start, start_0 = 0)
template <typename It>
__device__ __forceinline__ int find_item(const It* __restrict__ items, int n, int b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].start <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Next work unit of a grouped launch.  queue == NULL: one workgroup per unit,
// unit blockIdx.x (first call), then none (INT_MAX).  Otherwise persistent
// workgroups: each takes the next value of the device counter *queue (zeroed
// before the launch) until the units run out; a workgroup barrier on either
// side keeps the previous unit's LDS in use until every thread is done with
// it.  Every thread of the workgroup gets the same value.
__device__ __forceinline__ int next_unit(int* queue, int* slot, bool first) {
  if (!queue) return first ? (int)blockIdx.x : 0x7fffffff;
  __syncthreads();
  if (threadIdx.x == 0) *slot = atomicAdd(queue, 1);
  __syncthreads();
  return *slot;
}

// grouped stage launchers (items already in device memory; `wgs` = total
// work units).  queue: NULL (one workgroup per unit) or a zeroed device
// counter (persistent workgroups, as many as fit the device at once).  Each
// returns SPOD_OK or an error.
spod_status launch_fft_group(int nfft, spod_precision prec, spod_dtype dtype, int shift, int tile,
                             const FftItem* d_items, int n, int wgs, int* queue, hipStream_t st);
int fft_group_tile(int nfft, spod_precision prec, int tile);   // degrees of freedom per tile
spod_status launch_gram_group(spod_precision prec, int nt16, const GramItem* d_items, int n,
                              int wgs, int* queue, hipStream_t st);
int gram_groups(int nt16);                           // pair groups per (slice, k)
int64_t gram_group_wgs(int nt16, int64_t S, int64_t K);   // workgroups of one problem
spod_status launch_gram_combine_group(const CombineItem* d_items, int n, int wgs, hipStream_t st);
spod_status launch_eig_group(const EigItem* d_items, int n, int wgs, int max_sweeps, int lmax,
                             int threads, int* queue, hipStream_t st);
// (lmax: the group's largest L (16, 32 or 64); threads: 256, 1024, or 0 for the
// single-problem rule)
spod_status launch_modes_group(bool c128, const ModesItem* d_items, int n, int wgs,
                               size_t lds_bytes, int* queue, hipStream_t st);
spod_status launch_queue_reset(int* queue, int n, hipStream_t st);   // n counters to zero
// workgroups of a persistent launch: as many as the device holds at once (at
// most `units`)
int persistent_grid(const void* kernel, int threads, size_t lds_bytes, int units);

// --------------------------------------------------------------------------
// packed Fourier blocks (SPOD_QHAT_BFP20): every row (k, l) of M degrees of
// freedom is stored as ceil(M / 128) superblocks of 656 bytes.  A superblock
// holds 8 groups of 16 degrees of freedom: bytes 0..7 are the groups' int8
// exponents E (8..15 are zero), then group g at byte 16 + 80 g: the 8 pairs p
// (degrees of freedom 16 g + 2 p, + 1) as four int16 h at 8 p (re a, im a,
// re b, im b), then at 64 + 2 p one uint16 of the four low nibbles n (value i
// in bits 4 i .. 4 i + 3).  A value is (16 h + n) 2^E: a 20-bit two's
// complement mantissa with the group's shared exponent, |16 h + n| < 2^19.
// E = 127 marks a group with a non-finite value (decoded as NaN); an all-zero
// group has E = -128.  Degrees of freedom past M are zero.
// --------------------------------------------------------------------------
constexpr int PK_SB_DOFS = 128;
constexpr int PK_SB_BYTES = 656;
constexpr int PK_HDR_BYTES = 16;
constexpr int PK_GROUP_BYTES = 80;
constexpr int PK_EXP_NONFINITE = 127;
constexpr int PK_MANT_BITS = 20;
__host__ __device__ inline int64_t pk_superblocks(int64_t M) { return (M + PK_SB_DOFS - 1) / PK_SB_DOFS; }
__host__ __device__ inline int64_t pk_row_bytes(int64_t M) { return pk_superblocks(M) * PK_SB_BYTES; }

// Scale of a group's mantissas: 2^E, or NaN for the non-finite marker.
__device__ __forceinline__ float pk_scale(int e) {
  return e == PK_EXP_NONFINITE ? __builtin_nanf("") : ldexpf(1.0f, e);
}

// Decode four values from their int16 high parts (two packed per word) and
// the uint16 of low nibbles.
__device__ __forceinline__ void pk_decode4(uint32_t h01, uint32_t h23, uint32_t nib, float scale,
                                           float* v) {
  const int32_t h[4] = {(int32_t)(int16_t)(h01 & 0xffffu), (int32_t)h01 >> 16,
                        (int32_t)(int16_t)(h23 & 0xffffu), (int32_t)h23 >> 16};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int32_t mant = h[i] * 16 + (int32_t)((nib >> (4 * i)) & 15u);
    v[i] = (float)mant * scale;
  }
}

// Largest of x over the 4 lanes of an aligned quad (DPP quad swaps).
__device__ __forceinline__ uint32_t max4_u32(uint32_t x) {
  uint32_t y = (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4e, 0xf, 0xf, false);   // quad_perm [2,3,0,1]
  x = x > y ? x : y;
  y = (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xb1, 0xf, 0xf, false);            // quad_perm [1,0,3,2]
  return x > y ? x : y;
}

// Encode the eight values v (re, im of degrees of freedom 16 g + 4 c .. + 3)
// of quarter c of group g of the superblock at `sb`: two pairs, one 16-byte
// store of their int16 high parts and one 4-byte store of their nibbles.  The
// 4 lanes of a group (an aligned quad, all active) call it together and share
// the group's exponent.  The largest magnitude is taken on the bit patterns
// (|v| as unsigned integers order like the values, and infinities and NaNs
// lie above every finite value).  Plain (cached) stores: the 81 bytes of a
// group share cache lines with the neighbouring tiles, which the caller keeps
// on the same XCD.
__device__ __forceinline__ void pk_store_quarter(char* sb, int g, int c, const float* v) {
  uint32_t mb = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const uint32_t u = __float_as_uint(v[i]) & 0x7fffffffu;
    mb = mb > u ? mb : u;
  }
  mb = max4_u32(mb);
  const bool bad = mb >= 0x7f800000u;
  // mx < 2^ex with ex = biased exponent - 126; e = ex - 19 (|v| 2^-e < 2^19)
  int e = (int)(mb >> 23) - 145;
  e = e < -128 ? -128 : e;
  if (mb == 0) e = -128;
  uint32_t h[4] = {0, 0, 0, 0}, nib = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    // round to nearest even through the 1.5 2^23 offset (|v 2^-e| < 2^19)
    const float t = bad ? 0.0f : ldexpf(v[i], -e) + 12582912.0f;
    int32_t mant = (int32_t)(__float_as_uint(t) - 0x4b400000u);
    mant = mant > 524287 ? 524287 : mant;
    h[i >> 1] |= (((uint32_t)mant >> 4) & 0xffffu) << (16 * (i & 1));
    nib |= ((uint32_t)mant & 15u) << (4 * i);
  }
  char* grp = sb + PK_HDR_BYTES + PK_GROUP_BYTES * g;
  typedef unsigned int v4u __attribute__((ext_vector_type(4)));
  typedef unsigned int v2u __attribute__((ext_vector_type(2)));
  *reinterpret_cast<v4u*>(grp + 16 * c) = v4u{h[0], h[1], h[2], h[3]};
  *reinterpret_cast<uint32_t*>(grp + 64 + 4 * c) = nib;
  if (c == 0) sb[g] = (char)(signed char)(bad ? PK_EXP_NONFINITE : e);
  if (c == 0 && g == 0) *reinterpret_cast<v2u*>(sb + 8) = v2u{0u, 0u};   // unused header bytes
}

// Workgroup b of n -> tile, so that each XCD (workgroups are dealt to the 8
// XCDs in turn) takes a contiguous run of tiles: neighbouring tiles share
// cache lines of the packed rows, which then meet in one L2, and each XCD
// writes long runs of every frequency row.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t n) {
  const int64_t x = b & 7, i = b >> 3, q = n >> 3, r = n & 7;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

// --------------------------------------------------------------------------
// small device helpers
// --------------------------------------------------------------------------
template <typename T> struct cpx;
template <> struct cpx<float> { using type = float2; };
template <> struct cpx<double> { using type = double2; };
template <typename T> using cpx_t = typename cpx<T>::type;

template <typename C>
__device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C>
__device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename C>
__device__ __forceinline__ C cmulc(C a, C b) {
  return C{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
// multiply by -i
template <typename C>
__device__ __forceinline__ C cmul_mi(C a) { return C{a.y, -a.x}; }

}  // namespace spod
