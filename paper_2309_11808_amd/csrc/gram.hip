// Steps 3-4 of SPOD (eq. (spod-discrete-snapshots); Sec. 3.1 steps 3-4): the
// weighted inner product M_k = Qhat_k^* W Qhat_k for every frequency.
//
// Complex form.  With A = sqrt(W) Re(Qhat_k) and B = sqrt(W) Im(Qhat_k),
//   Re M_k = A A^T + B B^T,   Im M_k = A B^T - B A^T,
// four real products with a long contraction over the degrees of freedom, run
// on MFMA in 16 x 16 blocks of M_k (upper blocks only; M_k is Hermitian).  The
// paper reduces this sum over space across MPI ranks; here the M axis is split
// into S slices, one workgroup per (slice, frequency), whose four waves share
// LDS-staged chunks of the slice (splitting the chunk's degrees of freedom,
// or, for L > 32, the 16 x 16 block pairs), and the S partial Grams are
// combined in FP64 by a second kernel.
//
// Arithmetic per precision:
//   FP64    v_mfma_f64_16x16x4f64, FP64 accumulation, three real products
//           per complex one: T1 = A_a A_b^T, T2 = B_a B_b^T and
//           T3 = (A_a - B_a)(A_b + B_b)^T give Re = T1 + T2 and
//           Im = T3 - T1 + T2 (this path is bound by FP64 MFMA issue).
//   FP32    v_mfma_f32_16x16x4f32; the two products of one 4-wide step start
//           from zero and are added into FP64 registers at once.
//   BF16X4  block floating point split, per wave and 32-wide contraction
//   FP16X4  step: with E chosen so that |y| 2^-E < 2^H for every operand of
//           the step (H = 8 for BF16, 9 for FP16), y 2^-E = h + l with the
//           integer h = rint(y 2^-E) (exact in the 16-bit type) and
//           l = y 2^-E - h rounded to the 16-bit type (|l| <= 1/2).  All four
//           products h h^T + h l^T + l h^T + l l^T run on
//           v_mfma_f32_16x16x32_{bf16,f16}.  The h h^T sums are integers of
//           at most 64 * 2^(2H) <= 2^24, so their FP32 accumulation is exact;
//           only the representation of l is rounded (2^-(H+9) of the step's
//           largest operand for BF16, 2^-(H+11) for FP16).  Every step's sums
//           are scaled by 2^(2E) and added into FP64.  Dropping l l^T (the
//           common three-product scheme) is not done: on a Gram matrix it is
//           a one-signed bias of the diagonal that shifts every small
//           eigenvalue.  The integer form needs no range scaling of the data,
//           so FP16 and BF16 take the same path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "internal.h"

namespace spod {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

enum GramMode { G_F64 = 0, G_F32 = 1, G_BF16X4 = 2, G_FP16X4 = 3 };

template <int MODE> struct GramCfg;
template <> struct GramCfg<G_F64> {
  using T = double;               // arithmetic type of the operands
  using C = double2;              // qhat element
  static constexpr int DPL = 4;   // consecutive degrees of freedom loaded per lane
  using ACC = v4d;
};
template <> struct GramCfg<G_F32> {
  using T = float;
  using C = float2;
  static constexpr int DPL = 4;
  using ACC = v4f;
};
template <> struct GramCfg<G_BF16X4> {
  using T = float;
  using C = float2;
  static constexpr int DPL = 8;
  using ACC = v4f;
};
template <> struct GramCfg<G_FP16X4> {
  using T = float;
  using C = float2;
  static constexpr int DPL = 8;
  using ACC = v4f;
};

// ex with max_lanes x < 2^ex (x >= 0 in every lane; 0 when all are zero; a
// NaN or an infinity gives 129, which keeps them non-finite downstream).  The
// maximum is taken on the bit patterns, which order like non-negative floats:
// within each row of 16 lanes by DPP (quad swaps, half-row and row mirrors),
// then across the 4 rows on the scalar unit.
__device__ __forceinline__ int wave_max_exp(float x) {
  uint32_t u = __float_as_uint(x), v;
  v = (uint32_t)__builtin_amdgcn_mov_dpp((int)u, 0xb1, 0xf, 0xf, false);   // quad_perm [1,0,3,2]
  u = u > v ? u : v;
  v = (uint32_t)__builtin_amdgcn_mov_dpp((int)u, 0x4e, 0xf, 0xf, false);   // quad_perm [2,3,0,1]
  u = u > v ? u : v;
  v = (uint32_t)__builtin_amdgcn_mov_dpp((int)u, 0x141, 0xf, 0xf, false);  // row_half_mirror
  u = u > v ? u : v;
  v = (uint32_t)__builtin_amdgcn_mov_dpp((int)u, 0x140, 0xf, 0xf, false);  // row_mirror
  u = u > v ? u : v;
  uint32_t m = (uint32_t)__builtin_amdgcn_readlane((int)u, 0);
  uint32_t r = (uint32_t)__builtin_amdgcn_readlane((int)u, 16);
  m = m > r ? m : r;
  r = (uint32_t)__builtin_amdgcn_readlane((int)u, 32);
  m = m > r ? m : r;
  r = (uint32_t)__builtin_amdgcn_readlane((int)u, 48);
  m = m > r ? m : r;
  return m == 0 ? 0 : (int)(m >> 23) - 126;
}

// y 2^-E = h + l (see the header): h exact, l rounded to nearest even.
template <typename T16, typename FR>
__device__ __forceinline__ void split_int(const float* y, int e, FR& hi, FR& lo) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float ys = ldexpf(y[i], -e);
    const float h = rintf(ys);
    hi[i] = (T16)h;
    lo[i] = (T16)(ys - h);
  }
}

// One 16 x 16 x 32 product of the split operands, FP32 accumulation.
template <int MODE, typename FR>
__device__ __forceinline__ v4f mfma_split(FR x, FR y, v4f c) {
  if constexpr (MODE == G_BF16X4) return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c, 0, 0, 0);
  else return __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, c, 0, 0, 0);
}

template <typename V>
__device__ __forceinline__ V negate(V x) {
#pragma unroll
  for (int e = 0; e < 8; ++e) x[e] = -x[e];
  return x;
}

// Complex form.  With A = sqrt(W) Re(qhat_k) and B = sqrt(W) Im(qhat_k) as
// [L rows = blocks][M columns = degrees of freedom],
//   Re M_k = A A^T + B B^T,   Im M_k = A B^T - B A^T.
// The L rows are cut into NT tiles of 16; tile pairs (a <= b) give 16 x 16
// blocks of M_k (the lower blocks follow from Hermitian symmetry).  Every lane
// loads its MFMA fragments straight from HBM: lane l owns row 16a + l%16 and
// DPL consecutive degrees of freedom starting at (l/16)*DPL of the current
// group of 4*DPL; the contraction index is permuted accordingly (any fixed
// permutation of the summation order gives the same sum), so each lane reads
// one contiguous run of DPL complex values per tile.  A group is a
// 16 x 16 x 16 (FP64/FP32, four 4-wide MFMA steps) or 16 x 16 x 32
// (BF16/FP16, one MFMA step) product per real term.
constexpr int PG = 3;   // tile pairs per wave (grid z splits larger sets)

template <int NT, int P0, int NPG>
__host__ __device__ constexpr unsigned tiles_needed() {
  unsigned mask = 0;
  int pi = 0;
  for (int a = 0; a < NT; ++a)
    for (int b = a; b < NT; ++b, ++pi)
      if (pi >= P0 && pi < P0 + NPG) mask |= (1u << a) | (1u << b);
  return mask;
}

template <int MODE, int NT>
struct Raw {
  using Cfg = GramCfg<MODE>;
  typename Cfg::C x[NT][Cfg::DPL];
  typename Cfg::T w[Cfg::DPL];
};

// Any group (ragged end, unaligned rows): element-wise loads with bounds checks.
template <int MODE, int NT, unsigned NEED>
__device__ __forceinline__ void gram_load_any(Raw<MODE, NT>& r, const typename GramCfg<MODE>::C* __restrict__ qk,
                                              const typename GramCfg<MODE>::T* __restrict__ sqrtw,
                                              int64_t m, int64_t M, int64_t ldq, int L, int r16) {
  using Cfg = GramCfg<MODE>;
  using C = typename Cfg::C;
  using T = typename Cfg::T;
  constexpr int DPL = Cfg::DPL;
#pragma unroll
  for (int a = 0; a < NT; ++a) {
    if (!((NEED >> a) & 1u)) continue;
    const int row = 16 * a + r16;
#pragma unroll
    for (int e = 0; e < DPL; ++e)
      r.x[a][e] = (row < L && m + e < M) ? qk[(int64_t)row * ldq + m + e] : C{0, 0};
  }
#pragma unroll
  for (int e = 0; e < DPL; ++e) r.w[e] = (m + e < M) ? sqrtw[m + e] : (T)0;
}

// LDS staging of the contraction.  A chunk is 1 KB of every row of qhat_k
// (CD = 1024 / sizeof(C) degrees of freedom) plus the matching weights.  The
// workgroup loads it with fully coalesced 16-byte global-to-LDS loads (lane i
// of an instruction fills bytes [16 i, 16 i + 16) of one row), two chunks in
// flight, and every wave then multiplies its quarter of the chunk.  Rows are
// RSB = 1040 bytes apart in LDS, so the 16 lanes of one fragment read (16
// rows, same column) fall in distinct banks.  Each wave issues exactly NI load
// instructions per chunk (slots past the real rows re-read a valid row into a
// spare LDS slot), so the wait for a chunk is the constant vmcnt(NI).
template <int NT, int CHUNKB = 1024>
struct GramStage {
  // LDS row stride (bytes): 1040 for chunks of 1 KB (or a 656-byte packed
  // superblock), the chunk plus 16 bytes for chunks of 512 bytes or less
  // (rows stay 4 banks apart)
  static constexpr int RSB = CHUNKB > 512 ? 1040 : CHUNKB + 16;
  static constexpr int ROWS = 16 * NT + 2;          // tile rows, weight row, spare row
  static constexpr int BYTES = ROWS * RSB;          // one stage
  static constexpr int NI = (16 * NT + 1 + 3) / 4;  // load instructions per wave per chunk
};

// CHUNKB: bytes of one row per chunk (1024, or one 656-byte packed
// superblock: lanes past it re-read the superblock's first 16 bytes into the
// unused end of the row's slot, so no load leaves the row).
// Short chunks (CHUNKB <= 512: three or more 16-row tiles, or L > 64): one row
// per instruction, only the lanes that cover the row load (so the rows can be
// padded in LDS), and WB bytes of weights; rows of tiles outside `need`
// re-read the chunk's first row (a cached duplicate) so that every wave still
// issues NI loads per chunk.
constexpr int CPOL_NT = 2;   // the non-temporal bit of a load's cache-policy operand (gfx950)

template <int NT, int CHUNKB = 1024, int WB = 512>
__device__ __forceinline__ void stage_issue(char* stage, const char* __restrict__ qrows, int64_t rowb,
                                            const char* __restrict__ wrow, int L, int wave, int lane,
                                            unsigned need = ~0u) {
  using GS = GramStage<NT, CHUNKB>;
  constexpr bool SHORT = CHUNKB <= 512;
#pragma unroll
  for (int i = 0; i < GS::NI; ++i) {
    const int slot = wave + 4 * i;                   // 0 .. 16 NT  (16 NT = weights)
    const char* src;
    int dst;
    if (slot < 16 * NT) {
      int row = slot < L ? slot : L - 1;              // padded rows re-read a real row
      if (!((need >> (slot >> 4)) & 1u)) row = 0;     // tile not needed here
      src = qrows + (int64_t)row * rowb;
      dst = slot;
    } else if (slot == 16 * NT) {
      src = wrow;
      dst = slot;
    } else {
      src = wrow;                                     // spare slot: harmless duplicate
      dst = 16 * NT + 1;
    }
    // blocks are read once: non-temporal (cache policy NT); the weights are
    // read again for every frequency and keep the default policy
    typedef const void __attribute__((address_space(1)))* gptr;
    typedef void __attribute__((address_space(3)))* lptr;
    const lptr ldst = (lptr)(stage + dst * GS::RSB);
    if constexpr (SHORT) {
      const int nl = slot >= 16 * NT ? WB / 16 : CHUNKB / 16;
      if (lane < nl) {
        if (slot < 16 * NT) __builtin_amdgcn_global_load_lds((gptr)(src + 16 * lane), ldst, 16, 0, CPOL_NT);
        else __builtin_amdgcn_global_load_lds((gptr)(src + 16 * lane), ldst, 16, 0, 0);
      }
    } else {
      // the weight row holds 512 bytes: lanes 32..63 re-read the first half
      if (slot < 16 * NT)
        __builtin_amdgcn_global_load_lds((gptr)(src + (16 * lane < CHUNKB ? 16 * lane : 0)), ldst, 16, 0,
                                         CPOL_NT);
      else
        __builtin_amdgcn_global_load_lds((gptr)(src + 16 * (lane & 31)), ldst, 16, 0, 0);
    }
  }
}

// G: the pair group this wave computes; WPG: waves per group (4 / number of
// groups).  With one group (L <= 32) all four waves share the pairs and split
// each chunk's degrees of freedom; with 2 or 4 groups (L <= 48, <= 64) each
// wave runs its group's instantiation over the chunk that all four waves
// loaded, so the rows are read from HBM once per workgroup.  Every
// instantiation executes the same barriers, in the same order.
// PK: qhat in the packed 20-bit layout (one chunk = one superblock of 128
// degrees of freedom per row; ldq = bytes of a packed row; the rows are padded
// with zeros to whole superblocks and the weights to a multiple of 128).
// BIG (L > 64): one contraction step per chunk (GDOF degrees of freedom), one
// wave per pair group (WPG = 1), PGB pairs per group, the groups of a frequency
// spread over several workgroups (grid z); only the tiles in `need` (the
// workgroup's groups) are read.  `write`: false for a wave with no group of its
// own (it repeats another group's work for the barriers and stores nothing).
constexpr int PGB = 6;

// Bytes of one row per LDS chunk (L <= 64): 1 KB for up to two 16-row tiles;
// 512 bytes for three or four, so that the two stages take half the LDS and
// two workgroups share a CU (with 1 KB chunks one workgroup filled it, one
// wavefront per SIMD); one superblock for packed blocks.
template <int NT, bool PK>
__host__ __device__ constexpr int gram_chunk_bytes() {
  return PK ? PK_SB_BYTES : (NT >= 3 ? 512 : 1024);
}

template <int MODE, int NT, int G, int WPG, bool PK = false, bool BIG = false>
__device__ __forceinline__ void gram_body(const typename GramCfg<MODE>::C* __restrict__ qhat,
                                          const typename GramCfg<MODE>::T* __restrict__ sqrtw,
                                          double* __restrict__ part, int64_t M,
                                          int64_t ldq, int L, int S, bool vec, double* red, char* lds,
                                          int s, int k, unsigned need = ~0u, bool write = true) {
  using Cfg = GramCfg<MODE>;
  using T = typename Cfg::T;
  using C = typename Cfg::C;
  using ACC = typename Cfg::ACC;
  constexpr int DPL = Cfg::DPL;
  constexpr int GDOF = 4 * DPL;                             // degrees of freedom per group
  constexpr int CD = BIG ? GDOF : (PK ? PK_SB_DOFS : gram_chunk_bytes<NT, false>() / (int)sizeof(C));
  constexpr int CHUNKB = PK ? PK_SB_BYTES : CD * (int)sizeof(C);   // degrees of freedom, bytes per chunk
  using GS = GramStage<NT, CHUNKB>;
  constexpr int GPW = CD / GDOF / WPG;                      // DOF groups per wave per chunk
  constexpr int D = 16 * NT;
  constexpr int NP = NT * (NT + 1) / 2;
  constexpr int PGX = BIG ? PGB : PG;                       // pairs per group
  constexpr int P0 = G * PGX;
  constexpr int NPG = (NP - P0) < PGX ? (NP - P0) : PGX;
  static_assert(!BIG || (WPG == 1 && !PK), "L > 64: one wave per group, complex blocks");
  constexpr unsigned NEED = tiles_needed<NT, P0, NPG>();
  constexpr bool SPLIT = MODE == G_BF16X4 || MODE == G_FP16X4;
  static_assert(CD * (int)sizeof(T) <= 512, "weights of a chunk must fit the 512-byte weight row");
  static_assert(GPW >= 1, "a chunk must give every wave a group");

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int wsub = wave % WPG;          // this wave's share of the chunk within its group
  const int lane = tid & 63;
  const int r16 = lane & 15;
  const int g4 = lane >> 4;
  static_assert(!PK || (MODE != G_F64 && CD == PK_SB_DOFS), "packed blocks are complex64 superblocks");
  const C* qk = PK ? nullptr : qhat + (int64_t)k * L * ldq;

  // full chunks are split over the S slices; the ragged remainder (or all of
  // it, when 16-byte loads are not possible) goes to the last slice
  const int64_t nchunk = PK ? pk_superblocks(M) : (vec ? M / CD : 0);
  const int64_t c0 = nchunk * s / S, c1 = nchunk * (s + 1) / S;

  constexpr int NACC = MODE == G_F64 ? NPG : 1;
  ACC accR[NACC], accI[NACC];        // FP64 mode: running sums
  ACC accG[NACC];                    // FP64 mode: the third product of the 3-multiplication form
  double sR[NPG][4], sI[NPG][4];     // FP64 sums of the FP32 partials (not FP64 mode)
#pragma unroll
  for (int i = 0; i < NACC; ++i) accG[i] = accR[i] = accI[i] = ACC{0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < NPG; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) sR[i][v] = sI[i][v] = 0.0;
  auto compute = [&](const Raw<MODE, NT>& cur) {
    if constexpr (!SPLIT) {
      // four 4-wide MFMA steps; step t uses element t of every lane's run
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        T fa[NT], fb[NT], fd[NT], fs[NT];
#pragma unroll
        for (int a = 0; a < NT; ++a) {
          const bool live = 16 * a + r16 < L;
          fa[a] = live ? cur.x[a][t].x * cur.w[t] : (T)0;
          fb[a] = live ? cur.x[a][t].y * cur.w[t] : (T)0;
          fd[a] = fa[a] - fb[a];
          fs[a] = fa[a] + fb[a];
        }
        int pi = 0;
#pragma unroll
        for (int a = 0; a < NT; ++a) {
#pragma unroll
          for (int b = a; b < NT; ++b, ++pi) {
            if (pi < P0 || pi >= P0 + NPG) continue;
            const int i = pi - P0;
            if constexpr (MODE == G_F64) {
              // three real products per complex one: T1 = A_a A_b^T,
              // T2 = B_a B_b^T, T3 = (A_a - B_a)(A_b + B_b)^T; at the end
              // Re = T1 + T2 and Im = T3 - T1 + T2 (= A_a B_b^T - B_a A_b^T)
              accR[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fa[b], accR[i], 0, 0, 0);
              accI[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(fb[a], fb[b], accI[i], 0, 0, 0);
              accG[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(fd[a], fs[b], accG[i], 0, 0, 0);
            } else {
              ACC tr = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[a], fa[b], ACC{0, 0, 0, 0}, 0, 0, 0);
              tr = __builtin_amdgcn_mfma_f32_16x16x4f32(fb[a], fb[b], tr, 0, 0, 0);
              ACC ti = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[a], fb[b], ACC{0, 0, 0, 0}, 0, 0, 0);
              ti = __builtin_amdgcn_mfma_f32_16x16x4f32(-fb[a], fa[b], ti, 0, 0, 0);
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                sR[i][v] += (double)tr[v];
                sI[i][v] += (double)ti[v];
              }
            }
          }
        }
      }
    } else {
      using FR = typename std::conditional<MODE == G_BF16X4, v8bf, v8h>::type;
      using T16 = typename std::conditional<MODE == G_BF16X4, __bf16, _Float16>::type;
      constexpr int H = MODE == G_BF16X4 ? 8 : 9;     // bits of the integer part h
      // Rows past L hold a copy of row L - 1 (the staging re-reads it): they
      // only reach rows and columns of the partial Gram past L, which the
      // combination never reads, and they leave the step's maximum unchanged,
      // so they need no masking here.
      float ya[NT][8], yb[NT][8];
      float mx = 0.0f;
#pragma unroll
      for (int a = 0; a < NT; ++a) {
        if (!((NEED >> a) & 1u)) continue;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          ya[a][e] = cur.x[a][e].x * cur.w[e];
          yb[a][e] = cur.x[a][e].y * cur.w[e];
          mx = fmaxf(mx, fmaxf(fabsf(ya[a][e]), fabsf(yb[a][e])));
        }
      }
      // one exponent for the whole step of this wave: mx < 2^ex, so
      // |y| 2^-E < 2^H with E = ex - H (uniform across the wavefront)
      const int E = wave_max_exp(mx) - H;
      const double unit = ldexp(1.0, 2 * E);            // value of one integer product
      FR ah[NT], al[NT], bh[NT], bl[NT];
#pragma unroll
      for (int a = 0; a < NT; ++a) {
        if (!((NEED >> a) & 1u)) continue;
        split_int<T16>(ya[a], E, ah[a], al[a]);
        split_int<T16>(yb[a], E, bh[a], bl[a]);
      }
      int pi = 0;
#pragma unroll
      for (int a = 0; a < NT; ++a) {
#pragma unroll
        for (int b = a; b < NT; ++b, ++pi) {
          if (pi < P0 || pi >= P0 + NPG) continue;
          const int i = pi - P0;
          const FR nbh = negate(bh[a]), nbl = negate(bl[a]);
          ACC tr, ti, cr, ci;
#define SPOD_MFMA(x, y, acc) mfma_split<MODE>((x), (y), (acc))
          const ACC z = ACC{0, 0, 0, 0};
          // exact integer sums: Re h = ha hb^T (re) + ..., Im h = ha_re hb_im^T - ha_im hb_re^T
          tr = SPOD_MFMA(ah[a], ah[b], z);
          tr = SPOD_MFMA(bh[a], bh[b], tr);
          ti = SPOD_MFMA(ah[a], bh[b], z);
          ti = SPOD_MFMA(nbh, ah[b], ti);
          // correction products (rounded FP32 sums, at most 2^-(H-1) of the above)
          cr = SPOD_MFMA(ah[a], al[b], z);
          cr = SPOD_MFMA(al[a], ah[b], cr);
          cr = SPOD_MFMA(al[a], al[b], cr);
          cr = SPOD_MFMA(bh[a], bl[b], cr);
          cr = SPOD_MFMA(bl[a], bh[b], cr);
          cr = SPOD_MFMA(bl[a], bl[b], cr);
          ci = SPOD_MFMA(ah[a], bl[b], z);
          ci = SPOD_MFMA(al[a], bh[b], ci);
          ci = SPOD_MFMA(al[a], bl[b], ci);
          ci = SPOD_MFMA(nbh, al[b], ci);
          ci = SPOD_MFMA(nbl, ah[b], ci);
          ci = SPOD_MFMA(nbl, al[b], ci);
#undef SPOD_MFMA
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            sR[i][v] = fma((double)tr[v], unit, sR[i][v]);
            sR[i][v] = fma((double)cr[v], unit, sR[i][v]);
            sI[i][v] = fma((double)ti[v], unit, sI[i][v]);
            sI[i][v] = fma((double)ci[v], unit, sI[i][v]);
          }
        }
      }
    }
  };

  constexpr int WB = CHUNKB <= 512 ? CD * (int)sizeof(T) : 512;   // weight bytes per chunk
  const char* qb = PK ? reinterpret_cast<const char*>(qhat) + (int64_t)k * L * ldq
                      : reinterpret_cast<const char*>(qk);
  const char* wb = reinterpret_cast<const char*>(sqrtw);
  const int64_t rowb = PK ? ldq : ldq * (int64_t)sizeof(C);
  // the explicit counts below assume that only this unit's loads are in
  // flight (a persistent workgroup may still have its previous unit's stores)
  __builtin_amdgcn_s_waitcnt(0);
  if (c0 < c1)
    stage_issue<NT, CHUNKB, WB>(lds, qb + c0 * CHUNKB, rowb, wb + c0 * CD * (int64_t)sizeof(T), L,
                                wave, lane, need);
#pragma unroll 1
  for (int64_t c = c0; c < c1; ++c) {
    char* cur = lds + ((c - c0) & 1) * GS::BYTES;
    char* nxt = lds + (((c - c0) & 1) ^ 1) * GS::BYTES;
    // prefetch the next chunk (the last one re-reads itself into the free stage)
    const int64_t cn = c + 1 < c1 ? c + 1 : c;
    stage_issue<NT, CHUNKB, WB>(nxt, qb + cn * CHUNKB, rowb, wb + cn * CD * (int64_t)sizeof(T), L,
                                wave, lane, need);
    // wait for this wave's loads of chunk c (the NI of chunk c+1 stay in
    // flight), then for everybody's.  A bare s_barrier: __syncthreads() would
    // add a release fence that drains the prefetch as well.
    __builtin_amdgcn_s_waitcnt((GS::NI & 15) | ((GS::NI >> 4) << 14) | (7 << 4) | (15 << 8));
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int gw = 0; gw < GPW; ++gw) {
      const int base = (wsub * GPW + gw) * GDOF + g4 * DPL;   // this lane's run within the chunk
      Raw<MODE, NT> r;
#pragma unroll
      for (int a = 0; a < NT; ++a) {
        if (!((NEED >> a) & 1u)) continue;
        if constexpr (PK) {
          // decode this lane's DPL degrees of freedom (DPL / 2 pairs of one
          // group): int16 high parts, low nibbles, the group's exponent
          typedef unsigned int v4u __attribute__((ext_vector_type(4)));
          typedef unsigned int v2u __attribute__((ext_vector_type(2)));
          const char* rowp = cur + (16 * a + r16) * GS::RSB;
          const int g = base >> 4, p0 = (base & 15) >> 1;
          const float scale = pk_scale((int)(signed char)rowp[g]);
          const char* grp = rowp + PK_HDR_BYTES + PK_GROUP_BYTES * g;
          uint32_t hw[DPL], nw[DPL / 4 > 0 ? DPL / 4 : 1];
#pragma unroll
          for (int v = 0; v < DPL / 4; ++v) {
            const v4u h = *reinterpret_cast<const v4u*>(grp + 8 * p0 + 16 * v);
            hw[4 * v] = h[0];
            hw[4 * v + 1] = h[1];
            hw[4 * v + 2] = h[2];
            hw[4 * v + 3] = h[3];
          }
          if constexpr (DPL == 8) {
            const v2u n = *reinterpret_cast<const v2u*>(grp + 64 + 2 * p0);
            nw[0] = n[0];
            nw[1] = n[1];
          } else {
            nw[0] = *reinterpret_cast<const uint32_t*>(grp + 64 + 2 * p0);
          }
#pragma unroll
          for (int i = 0; i < DPL / 2; ++i) {
            float v[4];
            pk_decode4(hw[2 * i], hw[2 * i + 1], (nw[i >> 1] >> (16 * (i & 1))) & 0xffffu, scale, v);
            r.x[a][2 * i] = C{v[0], v[1]};
            r.x[a][2 * i + 1] = C{v[2], v[3]};
          }
          continue;
        }
        const v4f* src = reinterpret_cast<const v4f*>(cur + (16 * a + r16) * GS::RSB + base * (int)sizeof(C));
        constexpr int NV = (int)(sizeof(C) * DPL / 16);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const v4f f = src[v];
          if constexpr (sizeof(C) == 8) {
            r.x[a][2 * v] = C{f[0], f[1]};
            r.x[a][2 * v + 1] = C{f[2], f[3]};
          } else {
            double2 d;
            __builtin_memcpy(&d, &f, 16);
            r.x[a][v] = d;
          }
        }
      }
      const v4f* wsrc = reinterpret_cast<const v4f*>(cur + 16 * NT * GS::RSB + base * (int)sizeof(T));
      constexpr int NW = (int)(sizeof(T) * DPL / 16);
#pragma unroll
      for (int v = 0; v < NW; ++v) {
        const v4f f = wsrc[v];
        __builtin_memcpy(&r.w[v * (16 / (int)sizeof(T))], &f, 16);
      }
      compute(r);
    }
    // every wave's LDS reads of `cur` are done before anyone refills it
    __builtin_amdgcn_s_waitcnt(15 | (3 << 14) | (7 << 4) | (0 << 8));
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
  }
  // remaining degrees of freedom (ragged end, or everything when rows are not
  // 16-byte aligned), split over the S slices like the chunks; packed rows are
  // whole superblocks
  if constexpr (!PK) {
    const int64_t m_rem = nchunk * CD;
    const int64_t ng = (M - m_rem + GDOF - 1) / GDOF;
    const int64_t g0 = ng * s / S, g1 = ng * (s + 1) / S;
#pragma unroll 1
    for (int64_t g = g0 + wsub; g < g1; g += WPG) {
      Raw<MODE, NT> r;
      gram_load_any<MODE, NT, NEED>(r, qk, sqrtw, m_rem + g * GDOF + g4 * DPL, M, ldq, L, r16);
      compute(r);
    }
  }
  if constexpr (MODE == G_F64) {
#pragma unroll
    for (int i = 0; i < NPG; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        sR[i][v] = accR[i][v] + accI[i][v];
        sI[i][v] = (accG[i][v] - accR[i][v]) + accI[i][v];
      }
  }

  // element (lane, v) of a 16x16 result tile sits in column lane%16 and row
  // 4*(lane/16)+v for the FP32-accumulating instructions, but row lane/16+4*v
  // for v_mfma_f64_16x16x4f64.  Partials are stored as complex [D][D].
  double2* out = reinterpret_cast<double2*>(part) + ((int64_t)k * S + s) * D * D;
  if constexpr (WPG == 1) {
    // the wave is its group's only contributor: store from the registers
    __builtin_amdgcn_s_waitcnt(0);
    if (write) {
#pragma unroll
      for (int i = 0; i < NPG; ++i) {
        int a = 0, rem = P0 + i;
        while (rem >= NT - a) {
          rem -= NT - a;
          ++a;
        }
        const int b = a + rem;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = (MODE == G_F64) ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v;
          out[(16 * a + r) * D + 16 * b + (lane & 15)] = make_double2(sR[i][v], sI[i][v]);
        }
      }
    }
    return;
  }
  // the stages are reused for the reduction: drain the last (re-read)
  // prefetch of every wave first
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  // sum the group's waves through LDS (each group has its own region), one
  // wave at a time
  double* rg = red + G * (PG * 2 * 4 * 64);
#pragma unroll 1
  for (int w = 0; w < WPG; ++w) {
    if (wsub == w) {
#pragma unroll
      for (int i = 0; i < NPG; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double* rr = &rg[((2 * i) * 4 + v) * 64 + lane];
          double* ri = &rg[((2 * i + 1) * 4 + v) * 64 + lane];
          *rr = (w == 0) ? sR[i][v] : *rr + sR[i][v];
          *ri = (w == 0) ? sI[i][v] : *ri + sI[i][v];
        }
    }
    __syncthreads();
  }
  for (int idx = wsub * 64 + lane; idx < NPG * 4 * 64; idx += 64 * WPG) {
    const int ln = idx & 63;
    const int v = (idx >> 6) & 3;
    const int i = idx >> 8;
    int a = 0, rem = P0 + i;
    while (rem >= NT - a) {
      rem -= NT - a;
      ++a;
    }
    const int b = a + rem;
    const int r = (MODE == G_F64) ? (ln >> 4) + 4 * v : 4 * (ln >> 4) + v;
    out[(16 * a + r) * D + 16 * b + (ln & 15)] =
        make_double2(rg[((2 * i) * 4 + v) * 64 + ln], rg[((2 * i + 1) * 4 + v) * 64 + ln]);
  }
}

// Work unit = (slice s, frequency k), one workgroup each; the pair groups of
// a unit are spread over the workgroup's waves (see gram_body).
template <int MODE, int NT, bool PK = false>
__device__ __forceinline__ void gram_unit(const typename GramCfg<MODE>::C* __restrict__ qhat,
                                          const typename GramCfg<MODE>::T* __restrict__ sqrtw,
                                          double* __restrict__ part,
                                          int64_t M, int64_t ldq, int L, int S, int K, bool vec,
                                          int64_t local, char* lds) {
  constexpr int NP = NT * (NT + 1) / 2;
  constexpr int NG = (NP + PG - 1) / PG;
  static_assert(NG == 1 || NG == 2 || NG == 4, "pair groups must divide the 4 waves");
  constexpr int WPG = 4 / NG;
  if (local >= (int64_t)S * K) return;
  const int s = (int)(local % S);
  const int k = (int)(local / S);
  double* red = reinterpret_cast<double*>(lds);                      // reused after the loop
  const int g = (int)(threadIdx.x >> 6) / WPG;
  switch (g) {
    case 0: gram_body<MODE, NT, 0, WPG, PK>(qhat, sqrtw, part, M, ldq, L, S, vec, red, lds, s, k); break;
    case 1: if constexpr (NG > 1) gram_body<MODE, NT, 1, WPG, PK>(qhat, sqrtw, part, M, ldq, L, S, vec, red, lds, s, k); break;
    case 2: if constexpr (NG > 2) gram_body<MODE, NT, 2, WPG, PK>(qhat, sqrtw, part, M, ldq, L, S, vec, red, lds, s, k); break;
    case 3: if constexpr (NG > 3) gram_body<MODE, NT, 3, WPG, PK>(qhat, sqrtw, part, M, ldq, L, S, vec, red, lds, s, k); break;
    default: break;
  }
}

template <int MODE, int NT, bool PK>
__global__ __launch_bounds__(256, 2) void gram_kernel(const typename GramCfg<MODE>::C* __restrict__ qhat,
                                                      const void* __restrict__ sqrtw_v,
                                                      double* __restrict__ part, int64_t M,
                                                      int64_t ldq, int L, int S, int K, int vec) {
  using T = typename GramCfg<MODE>::T;
  extern __shared__ __attribute__((aligned(16))) char gram_lds[];   // 2 stages
  gram_unit<MODE, NT, PK>(qhat, static_cast<const T*>(sqrtw_v), part, M, ldq, L, S, K, vec != 0,
                          blockIdx.x, gram_lds);
}

// ---------------------------------------------------------------------------
// L > 64: the block pairs in groups of PGB, four groups (one per wave) per
// workgroup; work unit = (group set z, slice s, frequency k)
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int big_groups(int nt) { return (nt * (nt + 1) / 2 + PGB - 1) / PGB; }

// tiles used by pair group g (pairs g PGB .. g PGB + PGB - 1 in (a, b >= a) order)
__host__ __device__ constexpr unsigned big_need(int nt, int g) {
  unsigned mask = 0;
  int pi = 0;
  for (int a = 0; a < nt; ++a)
    for (int b = a; b < nt; ++b, ++pi)
      if (pi >= g * PGB && pi < (g + 1) * PGB) mask |= (1u << a) | (1u << b);
  return mask;
}

template <int MODE, int NT, int G>
__device__ __forceinline__ void gram_big_dispatch(int g, bool write, unsigned need,
                                                  const typename GramCfg<MODE>::C* __restrict__ qhat,
                                                  const typename GramCfg<MODE>::T* __restrict__ sqrtw,
                                                  double* __restrict__ part, int64_t M, int L, int S,
                                                  bool vec, char* lds, int s, int k) {
  if constexpr (G < big_groups(NT)) {
    if (g == G)
      gram_body<MODE, NT, G, 1, false, true>(qhat, sqrtw, part, M, M, L, S, vec, nullptr, lds, s, k,
                                             need, write);
    else
      gram_big_dispatch<MODE, NT, G + 1>(g, write, need, qhat, sqrtw, part, M, L, S, vec, lds, s, k);
  }
}

template <int MODE, int NT>
__global__ __launch_bounds__(256, 1) void gram_big_kernel(const typename GramCfg<MODE>::C* __restrict__ qhat,
                                                          const void* __restrict__ sqrtw_v,
                                                          double* __restrict__ part, int64_t M, int L,
                                                          int S, int K, int vec) {
  using T = typename GramCfg<MODE>::T;
  extern __shared__ __attribute__((aligned(16))) char gram_lds[];
  constexpr int NG = big_groups(NT);
  const int64_t local = blockIdx.x;
  const int z = (int)(local / ((int64_t)S * K));
  const int64_t rem = local - (int64_t)z * S * K;
  const int s = (int)(rem % S), k = (int)(rem / S);
  const int g = 4 * z + (int)(threadIdx.x >> 6);
  const bool write = g < NG;
  unsigned need = 0;
  for (int i = 4 * z; i < 4 * z + 4 && i < NG; ++i) need |= big_need(NT, i);
  gram_big_dispatch<MODE, NT, 0>(write ? g : NG - 1, write, need, qhat, static_cast<const T*>(sqrtw_v),
                                 part, M, L, S, vec != 0, gram_lds, s, k);
}

// Grouped launch over a batch: workgroup b -> item, then the item's local
// index -> work unit as in gram_kernel.
template <int MODE, int NT, bool PERSIST>
__global__ __launch_bounds__(256, 2) void gram_batch_kernel(const GramItem* __restrict__ items, int n,
                                                             int units, int* queue) {
  using T = typename GramCfg<MODE>::T;
  using C = typename GramCfg<MODE>::C;
  extern __shared__ __attribute__((aligned(16))) char gram_lds[];
  __shared__ int slot;
  for (int b = next_unit(PERSIST ? queue : nullptr, &slot, true); b < units;
       b = next_unit(PERSIST ? queue : nullptr, &slot, false)) {
    const GramItem& it = items[find_item(items, n, b)];
    gram_unit<MODE, NT>(static_cast<const C*>(it.qhat), static_cast<const T*>(it.sqrtw), it.part,
                        it.M, it.ldq, it.L, it.S, it.K, it.vec != 0, (int64_t)b - it.start, gram_lds);
    if constexpr (!PERSIST) break;
  }
}

// Sum the S partial Grams in FP64.  Each partial holds the 16 x 16 blocks
// (a, b) with a <= b; an entry (i, j) of a lower block is conj of (j, i).
__device__ __forceinline__ void gram_combine_body(const double2* __restrict__ part,
                                                  double2* __restrict__ gram, int L, int D, int S,
                                                  int k, bool acc) {
  const double2* pk = part + (int64_t)k * S * D * D;
  for (int idx = threadIdx.x; idx < L * L; idx += blockDim.x) {
    const int i = idx / L, j = idx % L;
    const bool up = (i >> 4) <= (j >> 4);
    const int off = up ? i * D + j : j * D + i;
    double re = 0.0, im = 0.0;
    for (int s = 0; s < S; ++s) {
      const double2 v = pk[(int64_t)s * D * D + off];
      re += v.x;
      im += v.y;
    }
    double2* g = gram + ((int64_t)k * L + i) * L + j;
    if (acc) {
      const double2 o = *g;
      *g = make_double2(o.x + re, o.y + (up ? im : -im));
    } else {
      *g = make_double2(re, up ? im : -im);
    }
  }
}

__global__ __launch_bounds__(256) void gram_combine_kernel(const double2* __restrict__ part,
                                                           double2* __restrict__ gram, int L, int D,
                                                           int S, int acc) {
  gram_combine_body(part, gram, L, D, S, blockIdx.x, acc != 0);
}

__global__ __launch_bounds__(256) void gram_combine_batch_kernel(const CombineItem* __restrict__ items,
                                                                 int n) {
  const CombineItem& it = items[find_item(items, n, (int)blockIdx.x)];
  gram_combine_body(static_cast<const double2*>(it.part), static_cast<double2*>(it.gram), it.L,
                    it.D, it.S, (int)blockIdx.x - it.start, false);
}

// ---------------------------------------------------------------------------
size_t csd_workspace(const Plan& p) {
  const size_t D = (size_t)p.gram_dim;
  return sizeof(double2) * (size_t)p.nfreq * (size_t)p.gram_split * D * D;
}

template <int MODE, int NTI>
static void launch_gram_nti(const Plan& p, const void* qhat, const void* sqrtw, double* part,
                            hipStream_t st) {
  using C = typename GramCfg<MODE>::C;
  dim3 grid((unsigned)((int64_t)p.gram_split * p.nfreq));
  const size_t lds = 2 * (size_t)GramStage<NTI, gram_chunk_bytes<NTI, false>()>::BYTES;
  if constexpr (MODE != G_F64) {
    if (p.qhat_packed) {
      const size_t lds_pk = 2 * (size_t)GramStage<NTI, PK_SB_BYTES>::BYTES;
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&gram_kernel<MODE, NTI, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_pk);
      hipLaunchKernelGGL((gram_kernel<MODE, NTI, true>), grid, dim3(256), lds_pk, st,
                         static_cast<const C*>(qhat), sqrtw, part, (int64_t)p.M, pk_row_bytes(p.M),
                         (int)p.nblocks, p.gram_split, (int)p.nfreq, 1);
      return;
    }
  }
  // 16-byte loads need 16-byte aligned rows (an aligned base and, for
  // complex64, an even M) and 16-byte aligned weights
  const bool vec = ((uintptr_t)qhat % 16 == 0) && (sizeof(C) == 16 || p.M % 2 == 0) &&
                   ((uintptr_t)sqrtw % 16 == 0);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&gram_kernel<MODE, NTI, false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((gram_kernel<MODE, NTI, false>), grid, dim3(256), lds, st,
                     static_cast<const C*>(qhat), sqrtw, part, (int64_t)p.M, (int64_t)p.M,
                     (int)p.nblocks, p.gram_split, (int)p.nfreq, (int)vec);
}

template <int MODE, int NTI>
static spod_status launch_gram_big(const Plan& p, const void* qhat, const void* sqrtw, double* part,
                                   hipStream_t st) {
  using C = typename GramCfg<MODE>::C;
  if constexpr (MODE == G_F32) {
    return fail(SPOD_ERR_UNSUPPORTED, "nblocks > 64 needs the fp64, bf16x4 or fp16x4 form");
  } else {
    if (p.qhat_packed) return fail(SPOD_ERR_UNSUPPORTED, "nblocks > 64 needs complex Fourier blocks");
    constexpr int CHUNKB = 4 * GramCfg<MODE>::DPL * (int)sizeof(C);
    const int Z = (big_groups(NTI) + 3) / 4;
    dim3 grid((unsigned)((int64_t)p.gram_split * p.nfreq * Z));
    const bool vec = ((uintptr_t)qhat % 16 == 0) && (sizeof(C) == 16 || p.M % 2 == 0) &&
                     ((uintptr_t)sqrtw % 16 == 0);
    const size_t lds = 2 * (size_t)GramStage<NTI, CHUNKB>::BYTES;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&gram_big_kernel<MODE, NTI>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((gram_big_kernel<MODE, NTI>), grid, dim3(256), lds, st,
                       static_cast<const C*>(qhat), sqrtw, part, (int64_t)p.M, (int)p.nblocks,
                       p.gram_split, (int)p.nfreq, (int)vec);
    return SPOD_OK;
  }
}

template <int MODE>
static spod_status launch_gram_mode(const Plan& p, const void* qhat, const void* sqrtw,
                                    double* part, hipStream_t st) {
  spod_status r = SPOD_OK;
  switch (p.gram_dim / 16) {
    case 1: launch_gram_nti<MODE, 1>(p, qhat, sqrtw, part, st); break;
    case 2: launch_gram_nti<MODE, 2>(p, qhat, sqrtw, part, st); break;
    case 3: launch_gram_nti<MODE, 3>(p, qhat, sqrtw, part, st); break;
    case 4: launch_gram_nti<MODE, 4>(p, qhat, sqrtw, part, st); break;
    case 5: r = launch_gram_big<MODE, 5>(p, qhat, sqrtw, part, st); break;
    case 6: r = launch_gram_big<MODE, 6>(p, qhat, sqrtw, part, st); break;
    case 7: r = launch_gram_big<MODE, 7>(p, qhat, sqrtw, part, st); break;
    case 8: r = launch_gram_big<MODE, 8>(p, qhat, sqrtw, part, st); break;
    case 9: r = launch_gram_big<MODE, 9>(p, qhat, sqrtw, part, st); break;
    case 10: r = launch_gram_big<MODE, 10>(p, qhat, sqrtw, part, st); break;
    default: return fail(SPOD_ERR_UNSUPPORTED, "nblocks > 160");
  }
  if (r != SPOD_OK) return r;
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPOD_OK : hip_fail(e, "gram_kernel");
}

spod_status launch_csd(const Plan& p, const void* qhat, void* gram, void* ws, hipStream_t st,
                       bool accumulate) {
  if (p.nblocks > SPOD_MAX_NBLOCKS) return fail(SPOD_ERR_UNSUPPORTED, "nblocks > 160");
  double* part = static_cast<double*>(ws);
  const size_t D = (size_t)p.gram_dim;
  spod_status s;
  switch (p.prec) {
    case SPOD_PREC_FP64: s = launch_gram_mode<G_F64>(p, qhat, p.d_sqrtw, part, st); break;
    case SPOD_PREC_FP32: s = launch_gram_mode<G_F32>(p, qhat, p.d_sqrtw32, part, st); break;
    case SPOD_PREC_BF16X4: s = launch_gram_mode<G_BF16X4>(p, qhat, p.d_sqrtw32, part, st); break;
    case SPOD_PREC_FP16X4: s = launch_gram_mode<G_FP16X4>(p, qhat, p.d_sqrtw32, part, st); break;
    default: return fail(SPOD_ERR_INVALID_ARG, "precision");
  }
  if (s != SPOD_OK) return s;
  hipLaunchKernelGGL(gram_combine_kernel, dim3((unsigned)p.nfreq), dim3(256), 0, st,
                     reinterpret_cast<const double2*>(part), static_cast<double2*>(gram),
                     (int)p.nblocks, (int)D, p.gram_split, accumulate ? 1 : 0);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPOD_OK : hip_fail(e, "gram_combine_kernel");
}

// ---------------------------------------------------------------------------
// spod_csd without a caller workspace: the Gram partials go to a scratch array
// of the library's own (file scope, one copy per device, held until the
// process ends).  Nothing in it has to start at zero: every slice writes all
// of its upper 16 x 16 blocks and the combination reads only those.  Calls
// that overlap on one device share the array and race.
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[SPOD_CSD_NOALLOC_MAX_BYTES];

constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex scratch_mu;
static void* scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// Device address of `scratch` on device `dev` (the current device): taken
// with hipGetSymbolAddress on the first call per device, then reused.  In host
// code the array's name is not a device address; only this pointer is.
static spod_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES)
    return fail(SPOD_ERR_UNSUPPORTED, "device ordinal above 63");
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(SPOD_ERR_HIP, "hipGetSymbolAddress(scratch) gave NULL");
    scratch_ptr[dev] = ptr;
  }
  *out = scratch_ptr[dev];
  return SPOD_OK;
}

spod_status launch_csd_noalloc(const Plan& p, const void* qhat, void* gram, hipStream_t st) {
  const size_t per_slice = sizeof(double2) * (size_t)p.nfreq * (size_t)p.gram_dim * (size_t)p.gram_dim;
  if (per_slice > SPOD_CSD_NOALLOC_MAX_BYTES)
    return fail(SPOD_ERR_UNSUPPORTED,
                "one slice of Gram partials (nfreq * (16 ceil(nblocks/16))^2 * 16 bytes) exceeds "
                "SPOD_CSD_NOALLOC_MAX_BYTES");
  // the plan's slice count, reduced until the partials fit the scratch array
  const int64_t fit = (int64_t)(SPOD_CSD_NOALLOC_MAX_BYTES / per_slice);
  Plan c = p;
  c.gram_split = (int)std::min<int64_t>(p.gram_split, fit);
  void* ptr = nullptr;
  spod_status s = scratch_address(p.device, &ptr);
  if (s != SPOD_OK) return s;
  return launch_csd(c, qhat, gram, ptr, st);
}

int64_t csd_noalloc_split(const Plan& p) {
  const size_t per_slice = sizeof(double2) * (size_t)p.nfreq * (size_t)p.gram_dim * (size_t)p.gram_dim;
  if (per_slice > SPOD_CSD_NOALLOC_MAX_BYTES) return 0;
  return std::min<int64_t>(p.gram_split, (int64_t)(SPOD_CSD_NOALLOC_MAX_BYTES / per_slice));
}

// ---------------------------------------------------------------------------
// grouped launches for a batch
// ---------------------------------------------------------------------------
int gram_groups(int nt16) {
  const int np = nt16 * (nt16 + 1) / 2;
  return (np + PG - 1) / PG;
}

int64_t gram_group_wgs(int nt16, int64_t S, int64_t K) {
  (void)nt16;
  return S * K;
}

template <int MODE, int NTI>
static spod_status gram_group_nti(const GramItem* d, int n, int wgs, int* queue, hipStream_t st) {
  const size_t lds = 2 * (size_t)GramStage<NTI, gram_chunk_bytes<NTI, false>()>::BYTES;
  if (queue) {
    const void* k = reinterpret_cast<const void*>(&gram_batch_kernel<MODE, NTI, true>);
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((gram_batch_kernel<MODE, NTI, true>), dim3((unsigned)persistent_grid(k, 256, lds, wgs)),
                       dim3(256), lds, st, d, n, wgs, queue);
  } else {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&gram_batch_kernel<MODE, NTI, false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((gram_batch_kernel<MODE, NTI, false>), dim3((unsigned)wgs), dim3(256), lds, st,
                       d, n, wgs, queue);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPOD_OK : hip_fail(e, "gram_batch_kernel");
}

template <int MODE>
static spod_status gram_group_mode(int nt16, const GramItem* d, int n, int wgs, int* queue,
                                   hipStream_t st) {
  switch (nt16) {
    case 1: return gram_group_nti<MODE, 1>(d, n, wgs, queue, st);
    case 2: return gram_group_nti<MODE, 2>(d, n, wgs, queue, st);
    case 3: return gram_group_nti<MODE, 3>(d, n, wgs, queue, st);
    case 4: return gram_group_nti<MODE, 4>(d, n, wgs, queue, st);
  }
  return fail(SPOD_ERR_UNSUPPORTED, "nblocks > 64");
}

spod_status launch_gram_group(spod_precision prec, int nt16, const GramItem* d_items, int n,
                              int wgs, int* queue, hipStream_t st) {
  switch (prec) {
    case SPOD_PREC_FP64: return gram_group_mode<G_F64>(nt16, d_items, n, wgs, queue, st);
    case SPOD_PREC_FP32: return gram_group_mode<G_F32>(nt16, d_items, n, wgs, queue, st);
    case SPOD_PREC_BF16X4: return gram_group_mode<G_BF16X4>(nt16, d_items, n, wgs, queue, st);
    case SPOD_PREC_FP16X4: return gram_group_mode<G_FP16X4>(nt16, d_items, n, wgs, queue, st);
  }
  return fail(SPOD_ERR_INVALID_ARG, "precision");
}

spod_status launch_gram_combine_group(const CombineItem* d_items, int n, int wgs, hipStream_t st) {
  hipLaunchKernelGGL(gram_combine_batch_kernel, dim3((unsigned)wgs), dim3(256), 0, st, d_items, n);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPOD_OK : hip_fail(e, "gram_combine_batch_kernel");
}

}  // namespace spod
