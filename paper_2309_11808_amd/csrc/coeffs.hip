// Expansion coefficients and reconstruction (SPOD for data compression,
// eq. (coeffs) and eq. (SPODrec)):
//
//   Phi_r = [modes of the retained frequencies, by frequency then mode]  (M x R)
//   B     = Phi_r^* W Phi_r                                  (R x R, Hermitian)
//   C     = Phi_r^* W (Q - qbar 1^T)                         (R x N_t)
//   A     = B^{-1} C                       (Cholesky B = L L^*, two solves)
//   Q~    = Re(Phi_r A) + qbar 1^T                           (M x N_t)
//
// B, C and Q~ are long real contractions run on v_mfma_f64_16x16x4f64 in
// 64 x 64 output tiles per workgroup (four waves of 32 x 32): 16- or 32-wide
// blocks of the contraction are staged in LDS as [k][64] so that a wave's 16
// lanes of one k read 16 consecutive doubles.  Complex operands are split into real and
// imaginary planes; complex64 modes and float32 snapshots are widened to FP64
// as they are loaded, so every form of the plan computes in FP64.  B and C
// contract over the M degrees of freedom, split into S slices whose partial
// tiles a second kernel adds in FP64 (the paper's sum over ranks).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"

namespace spod {

typedef double v4d __attribute__((ext_vector_type(4)));

namespace {

constexpr int TILE = 64;   // output tile edge
constexpr int KB = 16;     // contraction block staged in LDS

// Row r of Phi_r^T: mode r % n_r of frequency bins[r / n_r].
struct ModeSel {
  int n_r, n_modes, R;
  int bin[CoeffSel::MAX_BINS];
};

__device__ __forceinline__ int64_t sel_row(const ModeSel& s, int r) {
  return (int64_t)s.bin[r / s.n_r] * s.n_modes + r % s.n_r;
}

__device__ __forceinline__ double2 ld_c(const double2* p) { return *p; }
__device__ __forceinline__ double2 ld_c(const float2* p) {
  const float2 v = *p;
  return make_double2((double)v.x, (double)v.y);
}
__device__ __forceinline__ void st_c(double2* p, double2 v) { *p = v; }
__device__ __forceinline__ void st_c(float2* p, double2 v) {
  *p = make_float2((float)v.x, (float)v.y);
}

__device__ __forceinline__ v4d mfma(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// X = W conj(Phi_r) as two FP64 planes [M][R] (real, imaginary): a tiled
// transpose through LDS, so that the right-hand side reads 16 contiguous rows
// of R values per block instead of 64 mode rows far apart in memory.
// ---------------------------------------------------------------------------
constexpr int GM = 32;     // DOFs per gather tile

template <typename CT>
__global__ __launch_bounds__(256) void gather_weighted_kernel(const CT* __restrict__ phi,
                                                              const double* __restrict__ w,
                                                              ModeSel sel, double* __restrict__ Xr,
                                                              double* __restrict__ Xi, int64_t M) {
  __shared__ double tr[TILE][GM + 1], ti[TILE][GM + 1];
  const int R = sel.R;
  const int Ti = (R + TILE - 1) / TILE;
  const int i0 = (int)(blockIdx.x % Ti) * TILE;
  const int64_t m0 = (int64_t)(blockIdx.x / Ti) * GM;
  const int tid = threadIdx.x;
  // read: 64 mode rows x 32 DOFs, 8 threads x 4 DOFs a row, 32 rows per pass
  for (int rr = tid >> 3; rr < TILE; rr += 32) {
    const int i = i0 + rr;
    const CT* src = phi + (i < R ? sel_row(sel, i) * M : 0);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = (tid & 7) * 4 + u;
      const int64_t m = m0 + c;
      const double2 v = (i < R && m < M) ? ld_c(src + m) : make_double2(0.0, 0.0);
      const double wm = m < M ? w[m] : 0.0;
      tr[rr][c] = wm * v.x;
      ti[rr][c] = -wm * v.y;
    }
  }
  __syncthreads();
  // write: 32 DOF rows x 64 modes, 16 threads x 4 modes a row, 16 rows per pass
  for (int cc = tid >> 4; cc < GM; cc += 16) {
    const int64_t m = m0 + cc;
    if (m >= M) continue;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = (tid & 15) * 4 + u;
      if (i0 + r < R) {
        Xr[m * R + i0 + r] = tr[r][cc];
        Xi[m * R + i0 + r] = ti[r][cc];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// C = X^T (Q - qbar) with X = W conj(Phi_r): partial tile of slice s.  Grid:
// i tiles fastest, then t tiles, then slices (the i tiles of one t tile share
// its Q rows).  16-wide blocks of the contraction; the next block is loaded
// into registers while the current one is multiplied from LDS.
// ---------------------------------------------------------------------------
constexpr int KR = 16;               // contraction block of the right-hand side

template <typename QT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void coeff_rhs_kernel(
    const double* __restrict__ Xr, const double* __restrict__ Xi, const QT* __restrict__ q,
    const double* __restrict__ mean, double2* __restrict__ out, int R, int64_t M, int64_t nt,
    int S) {
  __shared__ double Ar[KR][TILE], Ai[KR][TILE], Bq[KR][TILE];
  const int Ti = (R + TILE - 1) / TILE;
  const int64_t Tt = (nt + TILE - 1) / TILE;
  const int64_t b = blockIdx.x;
  const int ti = (int)(b % Ti);
  const int64_t tt = (b / Ti) % Tt;
  const int s = (int)(b / Ti / Tt);
  const int i0 = ti * TILE;
  const int64_t t0 = tt * TILE;
  const int64_t m_beg = M * s / S, m_end = M * (s + 1) / S;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;

  // loaders (16 threads per row of 64): row k = tid/16, four consecutive columns
  const int ld_k = tid >> 4, ld_c4 = (tid & 15) * 4;
  const bool i_full = i0 + TILE <= R, t_full = t0 + TILE <= nt;

  double ra[4], rai[4], rb[4];
  auto fetch = [&](int64_t m0) {
    const int64_t m = m0 + ld_k;
    const bool ml = m < m_end;
    const double* xr = Xr + (ml ? m : 0) * R + i0 + ld_c4;
    const double* xi = Xi + (ml ? m : 0) * R + i0 + ld_c4;
    const double mu = ml ? mean[m] : 0.0;
    const QT* qr = q + (ml ? m : 0) * nt + t0 + ld_c4;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool il = ml && (i_full || i0 + ld_c4 + u < R);
      ra[u] = il ? xr[u] : 0.0;
      rai[u] = il ? xi[u] : 0.0;
      rb[u] = (ml && (t_full || t0 + ld_c4 + u < nt)) ? (double)qr[u] - mu : 0.0;
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      Ar[ld_k][ld_c4 + u] = ra[u];
      Ai[ld_k][ld_c4 + u] = rai[u];
      Bq[ld_k][ld_c4 + u] = rb[u];
    }
  };

  v4d accR[2][2], accI[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) accR[x][y] = accI[x][y] = v4d{0, 0, 0, 0};

  if (m_beg < m_end) fetch(m_beg);
  for (int64_t m0 = m_beg; m0 < m_end; m0 += KR) {
    __syncthreads();                 // every wave is done with the previous block
    stage();
    __syncthreads();
    if (m0 + KR < m_end) fetch(m0 + KR);
#pragma unroll
    for (int ks = 0; ks < KR / 4; ++ks) {
      const int kk = 4 * ks + (lane >> 4);
      double ar[2], ai[2], bq[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        ar[x] = Ar[kk][32 * wr + 16 * x + (lane & 15)];
        ai[x] = Ai[kk][32 * wr + 16 * x + (lane & 15)];
        bq[x] = Bq[kk][32 * wc + 16 * x + (lane & 15)];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          accR[x][y] = mfma(ar[x], bq[y], accR[x][y]);
          accI[x][y] = mfma(ai[x], bq[y], accI[x][y]);
        }
    }
  }
  double2* o = out + (int64_t)s * R * nt;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + 32 * wr + 16 * x + (lane >> 4) + 4 * v;
        const int64_t t = t0 + 32 * wc + 16 * y + (lane & 15);
        if (i < R && t < nt) o[(int64_t)i * nt + t] = make_double2(accR[x][y][v], accI[x][y][v]);
      }
}

// out[e] = sum over S slices of part[s][e], e < n
__global__ __launch_bounds__(256) void coeff_sum_kernel(const double2* __restrict__ part,
                                                        double2* __restrict__ out, int64_t n,
                                                        int S) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    double re = 0.0, im = 0.0;
    for (int s = 0; s < S; ++s) {
      const double2 v = part[(int64_t)s * n + e];
      re += v.x;
      im += v.y;
    }
    out[e] = make_double2(re, im);
  }
}

// ---------------------------------------------------------------------------
// B = Phi_r^* W Phi_r: partial 64 x 64 tile (ta, tb), ta <= tb, of slice s.
// Grid: tile pairs fastest, then slices.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void pair_of(int p, int T, int* ta, int* tb) {
  int a = 0;
  while (p >= T - a) {
    p -= T - a;
    ++a;
  }
  *ta = a;
  *tb = a + p;
}

template <typename CT>
__global__ __launch_bounds__(256) void mode_gram_kernel(const CT* __restrict__ phi,
                                                        const double* __restrict__ w, ModeSel sel,
                                                        double2* __restrict__ part, int64_t M,
                                                        int S) {
  __shared__ double Ar[KB][TILE], Ai[KB][TILE], Br[KB][TILE], Bi[KB][TILE];
  const int R = sel.R;
  const int T = (R + TILE - 1) / TILE;
  const int P = T * (T + 1) / 2;
  const int pr = (int)(blockIdx.x % P), s = (int)(blockIdx.x / P);
  int ta, tb;
  pair_of(pr, T, &ta, &tb);
  const int64_t m_beg = M * s / S, m_end = M * (s + 1) / S;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int ld_row = tid >> 2, ld_m = (tid & 3) * 4;
  const bool a_live = ta * TILE + ld_row < R, b_live = tb * TILE + ld_row < R;
  const CT* a_src = phi + (a_live ? sel_row(sel, ta * TILE + ld_row) * M : 0);
  const CT* b_src = phi + (b_live ? sel_row(sel, tb * TILE + ld_row) * M : 0);

  v4d accR[2][2], accI[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) accR[x][y] = accI[x][y] = v4d{0, 0, 0, 0};

  for (int64_t m0 = m_beg; m0 < m_end; m0 += KB) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t m = m0 + ld_m + u;
      const bool ml = m < m_end;
      const double wm = ml ? w[m] : 0.0;
      const double2 va = (a_live && ml) ? ld_c(a_src + m) : make_double2(0.0, 0.0);
      const double2 vb = (b_live && ml) ? ld_c(b_src + m) : make_double2(0.0, 0.0);
      Ar[ld_m + u][ld_row] = wm * va.x;
      Ai[ld_m + u][ld_row] = wm * va.y;
      Br[ld_m + u][ld_row] = vb.x;
      Bi[ld_m + u][ld_row] = vb.y;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < KB / 4; ++ks) {
      const int kk = 4 * ks + (lane >> 4);
      double ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        ar[x] = Ar[kk][32 * wr + 16 * x + (lane & 15)];
        ai[x] = Ai[kk][32 * wr + 16 * x + (lane & 15)];
        br[x] = Br[kk][32 * wc + 16 * x + (lane & 15)];
        bi[x] = Bi[kk][32 * wc + 16 * x + (lane & 15)];
      }
      // conj(a) b = (ar br + ai bi) + i (ar bi - ai br)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          accR[x][y] = mfma(ar[x], br[y], accR[x][y]);
          accR[x][y] = mfma(ai[x], bi[y], accR[x][y]);
          accI[x][y] = mfma(ar[x], bi[y], accI[x][y]);
          accI[x][y] = mfma(-ai[x], br[y], accI[x][y]);
        }
    }
    __syncthreads();
  }
  double2* o = part + ((int64_t)s * P + pr) * TILE * TILE;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 32 * wr + 16 * x + (lane >> 4) + 4 * v;
        const int c = 32 * wc + 16 * y + (lane & 15);
        o[r * TILE + c] = make_double2(accR[x][y][v], accI[x][y][v]);
      }
}

// B[i][j] from the partial tiles: tile (ta, tb) with ta <= tb holds rows of
// ta and columns of tb; the lower half is its conjugate transpose.
__global__ __launch_bounds__(256) void mode_gram_sum_kernel(const double2* __restrict__ part,
                                                            double2* __restrict__ B, int R, int S) {
  const int T = (R + TILE - 1) / TILE;
  const int P = T * (T + 1) / 2;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < (int64_t)P * TILE * TILE;
       e += (int64_t)gridDim.x * 256) {
    const int pr = (int)(e / (TILE * TILE)), rc = (int)(e % (TILE * TILE));
    int ta, tb;
    pair_of(pr, T, &ta, &tb);
    const int i = ta * TILE + rc / TILE, j = tb * TILE + rc % TILE;
    if (i >= R || j >= R) continue;
    double re = 0.0, im = 0.0;
    for (int s = 0; s < S; ++s) {
      const double2 v = part[((int64_t)s * P + pr) * TILE * TILE + rc];
      re += v.x;
      im += v.y;
    }
    B[(int64_t)i * R + j] = make_double2(re, im);
    if (ta != tb) B[(int64_t)j * R + i] = make_double2(re, -im);
  }
}

// ---------------------------------------------------------------------------
// Cholesky B = L L^* in place (lower triangle), one workgroup.  info = 0, or
// j + 1 when pivot j is not positive (the factorisation stops there).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void cholesky_kernel(double2* __restrict__ B, int R,
                                                        int32_t* __restrict__ info) {
  const int tid = threadIdx.x;
  for (int j = 0; j < R; ++j) {
    __syncthreads();
    const double d = B[(int64_t)j * R + j].x;
    if (!(d > 0.0)) {                       // the same value in every thread
      if (tid == 0) *info = j + 1;
      return;
    }
    const double l = sqrt(d), inv = 1.0 / l;
    for (int i = j + 1 + tid; i < R; i += blockDim.x) {
      double2* p = &B[(int64_t)i * R + j];
      *p = make_double2(p->x * inv, p->y * inv);
    }
    __syncthreads();
    if (tid == 0) B[(int64_t)j * R + j] = make_double2(l, 0.0);
    const int n = R - j - 1;
    for (int64_t e = tid; e < (int64_t)n * n; e += blockDim.x) {
      const int i = j + 1 + (int)(e / n), k = j + 1 + (int)(e % n);
      if (k > i) continue;
      const double2 a = B[(int64_t)i * R + j], c = B[(int64_t)k * R + j];
      // B[i][k] -= L[i][j] conj(L[k][j])
      double2* p = &B[(int64_t)i * R + k];
      *p = make_double2(p->x - (a.x * c.x + a.y * c.y), p->y - (a.y * c.x - a.x * c.y));
    }
  }
  __syncthreads();
  // U = L^* in the strictly upper triangle, so the back substitution reads rows
  for (int64_t e = tid; e < (int64_t)R * R; e += blockDim.x) {
    const int i = (int)(e / R), k = (int)(e % R);
    if (k > i) {
      const double2 l = B[(int64_t)k * R + i];
      B[e] = make_double2(l.x, -l.y);
    }
  }
  if (tid == 0) *info = 0;
}

// A = L^{-*} L^{-1} C.  One workgroup per SOLVE_COLS columns of C, whose
// unknowns live in LDS; 32 lanes share the dot product of every row (strided
// over k, summed by shuffles).  L is read by rows: the lower triangle for the
// forward pass, U = L^* (stored above the diagonal) for the backward pass.
// With info != 0 the columns of A are zero.
constexpr int SOLVE_COLS = 8;

template <typename CT>
__global__ __launch_bounds__(256) void coeff_solve_kernel(const double2* __restrict__ L,
                                                          const double2* __restrict__ C,
                                                          CT* __restrict__ A, int R, int64_t nt,
                                                          const int32_t* __restrict__ info) {
  extern __shared__ double2 y[];            // [R][SOLVE_COLS]
  const int tid = threadIdx.x, col = tid >> 5, sub = tid & 31;
  const int64_t t = (int64_t)blockIdx.x * SOLVE_COLS + col;
  const bool live = t < nt;
  if (*info != 0) {
    if (live)
      for (int i = sub; i < R; i += 32) st_c(&A[(int64_t)i * nt + t], make_double2(0.0, 0.0));
    return;
  }
  for (int i = sub; i < R; i += 32)
    y[i * SOLVE_COLS + col] = live ? C[(int64_t)i * nt + t] : make_double2(0.0, 0.0);
  __syncthreads();
  for (int i = 0; i < R; ++i) {             // L y = c
    const double2* Li = L + (int64_t)i * R;
    double re = 0.0, im = 0.0;
    for (int k = sub; k < i; k += 32) {
      const double2 l = Li[k], v = y[k * SOLVE_COLS + col];
      re += l.x * v.x - l.y * v.y;
      im += l.x * v.y + l.y * v.x;
    }
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) {
      re += __shfl_xor(re, off, 32);
      im += __shfl_xor(im, off, 32);
    }
    if (sub == 0) {
      const double d = 1.0 / Li[i].x;
      const double2 c = y[i * SOLVE_COLS + col];
      y[i * SOLVE_COLS + col] = make_double2((c.x - re) * d, (c.y - im) * d);
    }
    __syncthreads();
  }
  for (int i = R - 1; i >= 0; --i) {        // L^* a = y, U = L^* row by row
    const double2* Ui = L + (int64_t)i * R;
    double re = 0.0, im = 0.0;
    for (int k = i + 1 + sub; k < R; k += 32) {
      const double2 u = Ui[k], v = y[k * SOLVE_COLS + col];
      re += u.x * v.x - u.y * v.y;
      im += u.x * v.y + u.y * v.x;
    }
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) {
      re += __shfl_xor(re, off, 32);
      im += __shfl_xor(im, off, 32);
    }
    if (sub == 0) {
      const double d = 1.0 / Ui[i].x;
      const double2 c = y[i * SOLVE_COLS + col];
      y[i * SOLVE_COLS + col] = make_double2((c.x - re) * d, (c.y - im) * d);
    }
    __syncthreads();
  }
  if (live)
    for (int i = sub; i < R; i += 32) st_c(&A[(int64_t)i * nt + t], y[i * SOLVE_COLS + col]);
}

// ---------------------------------------------------------------------------
// Q~[m][t] = sum_r Re(phi_r[m] A[r][t]) + qbar[m].  Grid: t tiles fastest,
// then m tiles (consecutive workgroups share the modes of one m tile).
// ---------------------------------------------------------------------------
template <typename CT, typename QT>
__global__ __launch_bounds__(256) void reconstruct_kernel(const CT* __restrict__ phi,
                                                          const CT* __restrict__ A,
                                                          const double* __restrict__ mean,
                                                          ModeSel sel, QT* __restrict__ qrec,
                                                          int64_t M, int64_t nt) {
  __shared__ double Pr[KB][TILE], Pi[KB][TILE], Xr[KB][TILE], Xi[KB][TILE];
  const int R = sel.R;
  const int64_t Tt = (nt + TILE - 1) / TILE;
  const int64_t tt = blockIdx.x % Tt, tm = blockIdx.x / Tt;
  const int64_t m0 = tm * TILE, t0 = tt * TILE;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int ld_k = tid >> 4, ld_x = (tid & 15) * 4;   // row k of the block, four columns

  v4d acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = v4d{0, 0, 0, 0};

  for (int r0 = 0; r0 < R; r0 += KB) {
    const int r = r0 + ld_k;
    const bool rl = r < R;
    const CT* prow = phi + (rl ? sel_row(sel, r) * M : 0);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t m = m0 + ld_x + u, t = t0 + ld_x + u;
      const double2 p = (rl && m < M) ? ld_c(prow + m) : make_double2(0.0, 0.0);
      const double2 a = (rl && t < nt) ? ld_c(A + (int64_t)r * nt + t) : make_double2(0.0, 0.0);
      Pr[ld_k][ld_x + u] = p.x;
      Pi[ld_k][ld_x + u] = -p.y;          // Re(p a) = p.x a.x - p.y a.y
      Xr[ld_k][ld_x + u] = a.x;
      Xi[ld_k][ld_x + u] = a.y;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < KB / 4; ++ks) {
      const int kk = 4 * ks + (lane >> 4);
      double pr[2], pi[2], xr[2], xi[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        pr[x] = Pr[kk][32 * wr + 16 * x + (lane & 15)];
        pi[x] = Pi[kk][32 * wr + 16 * x + (lane & 15)];
        xr[x] = Xr[kk][32 * wc + 16 * x + (lane & 15)];
        xi[x] = Xi[kk][32 * wc + 16 * x + (lane & 15)];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          acc[x][y] = mfma(pr[x], xr[y], acc[x][y]);
          acc[x][y] = mfma(pi[x], xi[y], acc[x][y]);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t m = m0 + 32 * wr + 16 * x + (lane >> 4) + 4 * v;
      if (m >= M) continue;
      const double mu = mean[m];
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const int64_t t = t0 + 32 * wc + 16 * y + (lane & 15);
        if (t < nt) qrec[m * nt + t] = (QT)(acc[x][y][v] + mu);
      }
    }
}

ModeSel make_sel(const CoeffSel& cs) {
  ModeSel s;
  s.n_r = cs.n_r;
  s.n_modes = cs.n_modes;
  s.R = cs.n_bins * cs.n_r;
  for (int i = 0; i < CoeffSel::MAX_BINS; ++i) s.bin[i] = i < cs.n_bins ? cs.bin[i] : 0;
  return s;
}

}  // namespace

CoeffLayout coeff_layout(const Plan& p, int R) {
  CoeffLayout c;
  c.R = R;
  const int Ti = (R + TILE - 1) / TILE;
  const int64_t Tt = (p.nt + TILE - 1) / TILE;
  const int64_t tiles = (int64_t)Ti * Tt;
  // about 8192 workgroups for the right-hand side, slices of >= 4096 DOFs
  int64_t s = (8192 + tiles - 1) / tiles;
  s = std::min<int64_t>(s, std::max<int64_t>(1, p.M / 4096));
  c.S_rhs = (int)std::max<int64_t>(1, s);
  const int P = Ti * (Ti + 1) / 2;
  int64_t sb = (2048 + P - 1) / P;
  sb = std::min<int64_t>(sb, std::max<int64_t>(1, p.M / 1024));
  c.S_gram = (int)std::max<int64_t>(1, sb);
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t rhs_part = c.S_rhs > 1 ? sizeof(double2) * (size_t)c.S_rhs * R * p.nt : 0;
  const size_t gram_part = sizeof(double2) * (size_t)c.S_gram * P * TILE * TILE;
  c.off_B = 0;
  c.off_C = up(sizeof(double2) * (size_t)R * R);
  c.off_part = c.off_C + up(sizeof(double2) * (size_t)R * p.nt);
  c.off_X = c.off_part + up(std::max(rhs_part, gram_part));
  c.bytes = c.off_X + 2 * up(sizeof(double) * (size_t)p.M * R);
  return c;
}

spod_status launch_coeffs(const Plan& p, const void* q, spod_dtype dtype, const double* mean,
                          const void* phi, const CoeffSel& cs, void* a, int32_t* info, void* ws,
                          hipStream_t st) {
  const ModeSel sel = make_sel(cs);
  const int R = sel.R;
  const CoeffLayout c = coeff_layout(p, R);
  char* base = static_cast<char*>(ws);
  double2* B = reinterpret_cast<double2*>(base + c.off_B);
  double2* Cm = reinterpret_cast<double2*>(base + c.off_C);
  double2* part = reinterpret_cast<double2*>(base + c.off_part);
  const bool c128 = is_complex128(p);
  const int Ti = (R + TILE - 1) / TILE;
  const int P = Ti * (Ti + 1) / 2;
  const int64_t Tt = (p.nt + TILE - 1) / TILE;

  // B = Phi^* W Phi
  if (c128)
    hipLaunchKernelGGL(mode_gram_kernel<double2>, dim3((unsigned)(P * c.S_gram)), dim3(256), 0, st,
                       static_cast<const double2*>(phi), p.d_weights, sel, part, p.M, c.S_gram);
  else
    hipLaunchKernelGGL(mode_gram_kernel<float2>, dim3((unsigned)(P * c.S_gram)), dim3(256), 0, st,
                       static_cast<const float2*>(phi), p.d_weights, sel, part, p.M, c.S_gram);
  const int64_t nb = (int64_t)P * TILE * TILE;
  hipLaunchKernelGGL(mode_gram_sum_kernel, dim3((unsigned)std::min<int64_t>((nb + 255) / 256, 4096)),
                     dim3(256), 0, st, part, B, R, c.S_gram);
  hipLaunchKernelGGL(cholesky_kernel, dim3(1), dim3(1024), 0, st, B, R, info);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "mode_gram / cholesky");

  // X = W conj(Phi_r) as [M][R] planes, then C = X^T (Q - qbar)
  double* Xr = reinterpret_cast<double*>(base + c.off_X);
  double* Xi = Xr + ((sizeof(double) * (size_t)p.M * R + 255) / 256 * 256) / sizeof(double);
  const int64_t Tm = (p.M + GM - 1) / GM;
  if (c128)
    hipLaunchKernelGGL(gather_weighted_kernel<double2>, dim3((unsigned)(Ti * Tm)), dim3(256), 0, st,
                       static_cast<const double2*>(phi), p.d_weights, sel, Xr, Xi, p.M);
  else
    hipLaunchKernelGGL(gather_weighted_kernel<float2>, dim3((unsigned)(Ti * Tm)), dim3(256), 0, st,
                       static_cast<const float2*>(phi), p.d_weights, sel, Xr, Xi, p.M);
  double2* rhs = c.S_rhs > 1 ? part : Cm;
  const unsigned grid = (unsigned)((int64_t)Ti * Tt * c.S_rhs);
  if (dtype == SPOD_F32)
    hipLaunchKernelGGL(coeff_rhs_kernel<float>, dim3(grid), dim3(256), 0, st, Xr, Xi,
                       static_cast<const float*>(q), mean, rhs, R, p.M, p.nt, c.S_rhs);
  else
    hipLaunchKernelGGL(coeff_rhs_kernel<double>, dim3(grid), dim3(256), 0, st, Xr, Xi,
                       static_cast<const double*>(q), mean, rhs, R, p.M, p.nt, c.S_rhs);
  if (c.S_rhs > 1) {
    const int64_t n = (int64_t)R * p.nt;
    hipLaunchKernelGGL(coeff_sum_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 8192)),
                       dim3(256), 0, st, part, Cm, n, c.S_rhs);
  }
  const unsigned sg = (unsigned)((p.nt + SOLVE_COLS - 1) / SOLVE_COLS);
  const size_t lds = sizeof(double2) * (size_t)R * SOLVE_COLS;   // <= 128 KiB (R <= 1024)
  if (c128) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&coeff_solve_kernel<double2>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(coeff_solve_kernel<double2>, dim3(sg), dim3(256), lds, st, B, Cm,
                       static_cast<double2*>(a), R, p.nt, info);
  } else {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&coeff_solve_kernel<float2>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(coeff_solve_kernel<float2>, dim3(sg), dim3(256), lds, st, B, Cm,
                       static_cast<float2*>(a), R, p.nt, info);
  }
  e = hipGetLastError();
  return e == hipSuccess ? SPOD_OK : hip_fail(e, "coeff_rhs / solve");
}

spod_status launch_reconstruct(const Plan& p, const void* phi, const CoeffSel& cs, const void* a,
                               const double* mean, void* qrec, spod_dtype dtype, hipStream_t st) {
  const ModeSel sel = make_sel(cs);
  const int64_t Tt = (p.nt + TILE - 1) / TILE, Tm = (p.M + TILE - 1) / TILE;
  const int64_t wgs = Tt * Tm;
  if (wgs > 0x7fffffffLL) return fail(SPOD_ERR_UNSUPPORTED, "reconstruction grid too large");
  const dim3 grid((unsigned)wgs);
#define SPOD_REC(CT, QT)                                                                          \
  hipLaunchKernelGGL((reconstruct_kernel<CT, QT>), grid, dim3(256), 0, st,                       \
                     static_cast<const CT*>(phi), static_cast<const CT*>(a), mean, sel,           \
                     static_cast<QT*>(qrec), p.M, p.nt)
  const bool c128 = is_complex128(p);
  if (c128 && dtype == SPOD_F32) SPOD_REC(double2, float);
  else if (c128) SPOD_REC(double2, double);
  else if (dtype == SPOD_F32) SPOD_REC(float2, float);
  else SPOD_REC(float2, double);
#undef SPOD_REC
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPOD_OK : hip_fail(e, "reconstruct_kernel");
}

}  // namespace spod
