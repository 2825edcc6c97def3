// Adjoint of the SPOD path (the paper does not differentiate SPOD; this is the
// reverse mode of the forward definition of Sec. 2.3).
//
// For a real loss E and complex z the gradient is g_z = dE/dRe z + i dE/dIm z.
// Per selected frequency k, with Qhat_k the M x L block matrix, M_k =
// Qhat_k^H W Qhat_k = Psi Lambda Psi^H and Phi_k = Qhat_k C, C = Psi_n
// Lambda_n^{-1/2} (n leading modes):
//
//   A  R = Qhat_k^H g_Phi                          (L x n, reduction over M)
//   B  g_C = R; g_Psi = R Lambda^{-1/2}; g_lambda_j += -1/2 lambda_j^{-3/2}
//      Re(psi_j^H R_j); the phase convention psi_j[p] > 0 (p = entry of
//      largest modulus) adds -i Im(psi_j^H g_psi_j) / |psi_j[p]| at entry p;
//      X = Psi^H g_Psi, K = diag(g_lambda) + F o (X - X^H)/2 with
//      F_ij = 1 / (lambda_j - lambda_i); G = Psi K Psi^H (Hermitian).
//   C  g_Qhat_k = g_Phi C^H + 2 W Qhat_k G
//   D  g_x[l s + n] += kappa w[n] Re sum_k g_Qhat[k][l] e^{+2 pi i k n / N}
//      (one-sided sum), then g_q = g_x - mean_t(g_x) (mean removal).
//
// D runs the sum as a length-N complex FFT: the one-sided spectra of two
// degrees of freedom a, b are extended Hermitian-wise (H[0] = 2 Re g_0,
// H[N/2] = 2 Re g_{N/2}, H[N-k] = conj g_k), packed as Z = H_a + i H_b, and
// y_a + i y_b = 1/2 conj(DFT(conj Z)).  The blocks are overlap-added in
// registers (the hop is 2, 4 or 8 lane strides), and the mean adjoint
// sum_t g_x = kappa sum_l Re sum_k g_Qhat[k][l] conj(What_k) only needs the
// bins where the window's DFT What_k is non-zero, so g_q is written once.
#include <hip/hip_runtime.h>

#include <vector>

#include "fft_core.h"
#include "internal.h"

namespace spod {

constexpr int BWD_MAXL = 64;
constexpr int BWD_MAXK = 513;      // nfft / 2 + 1 for nfft <= 1024
constexpr int BWD_TM = 64;         // degrees of freedom per LDS tile of pass A
constexpr int BWD_TMP = BWD_TM + 1; // its padded row (rows l of one column fall in different banks)
constexpr int BWD_PARTS = 2048;    // partial sums of pass A over all selected bins

// Selected frequencies (row s of the per-bin arrays holds frequency k[s]) and
// the inverse map (slot[k] = s, or -1), passed by value.
struct BinTable {
  int n;
  int16_t k[BWD_MAXK];
  int16_t slot[BWD_MAXK];
};

// Bins with What_k != 0 for the mean adjoint: slots and the window's DFT.  n < 0:
// use every selected bin with the plan's What table.
struct MeanList {
  int n;
  int slot[Plan::SPOD_MAX_MEAN_BINS];
  double wr[Plan::SPOD_MAX_MEAN_BINS], wi[Plan::SPOD_MAX_MEAN_BINS];
};

__global__ void write_sel_kernel(BinTable bt, int* __restrict__ dst) {
  for (int i = threadIdx.x; i < bt.n; i += blockDim.x) dst[i] = bt.k[i];
}

// ---------------------------------------------------------------------------
// pass A: R[s][part][l][j] = sum_m conj(qhat[k][l][m]) g_phi[s][j][m] over the
// part's range of m, accumulated in FP64.  Rows l and j of a tile of 64
// degrees of freedom are staged in LDS; thread t owns outputs o = t (+256..)
// and, when there are fewer than 128 outputs, a residue class of the tile's
// columns (the column partial sums are added in a fixed order at the end).
// ---------------------------------------------------------------------------
template <typename TC>
__global__ __launch_bounds__(256) void bwd_r_kernel(const cpx_t<TC>* qrows, int q_by_k,
                                                    const cpx_t<TC>* __restrict__ g_phi,
                                                    double2* __restrict__ rpart, BinTable bt,
                                                    int64_t M, int L, int n, int S, int64_t per) {
  using C = cpx_t<TC>;
  extern __shared__ char r_lds[];
  C* tile = reinterpret_cast<C*>(r_lds);                                   // [L + n][TMP]
  double2* red = reinterpret_cast<double2*>(r_lds + sizeof(C) * ((L + n) * BWD_TMP + 1) / 16 * 16);
  const int s = blockIdx.y;
  const int k = bt.k[s];
  const int tid = threadIdx.x;
  const C* qk = qrows + (int64_t)(q_by_k ? k : s) * L * M;
  const C* gk = g_phi + (int64_t)s * n * M;
  const int NO = L * n;
  const int RP = NO >= 128 ? 1 : (256 / NO < 8 ? 256 / NO : 8);
  const int opt = (NO + 255) / 256;
  const int o0 = RP > 1 ? tid % NO : tid;
  const int part = RP > 1 ? tid / NO : 0;
  const bool active = part < RP;

  double2 acc[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) acc[u] = make_double2(0.0, 0.0);

  const int64_t mb = (int64_t)blockIdx.x * per;
  const int64_t me = mb + per < M ? mb + per : M;
  for (int64_t m0 = mb; m0 < me; m0 += BWD_TM) {
    for (int idx = tid; idx < (L + n) * BWD_TM; idx += 256) {
      const int row = idx / BWD_TM, c = idx % BWD_TM;
      const int64_t m = m0 + c;
      C v{0, 0};
      if (m < me) v = row < L ? qk[(int64_t)row * M + m] : gk[(int64_t)(row - L) * M + m];
      tile[row * BWD_TMP + c] = v;
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int o = o0 + u * 256;
        if (u < opt && o < NO) {
          const int l = o / n, j = o % n;
          const C* a = tile + l * BWD_TMP;
          const C* b = tile + (L + j) * BWD_TMP;
          double sr = 0.0, si = 0.0;
          for (int c = part; c < BWD_TM; c += RP) {
            const double ar = a[c].x, ai = a[c].y, br = b[c].x, bi = b[c].y;
            sr += ar * br + ai * bi;     // conj(a) b
            si += ar * bi - ai * br;
          }
          acc[u].x += sr;
          acc[u].y += si;
        }
      }
    }
    __syncthreads();
  }
  double2* out = rpart + ((int64_t)s * S + blockIdx.x) * NO;
  if (RP == 1) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int o = tid + u * 256;
      if (u < opt && o < NO) out[o] = acc[u];
    }
  } else {
    red[tid] = acc[0];
    __syncthreads();
    if (tid < NO) {
      double2 r = red[tid];
      for (int pp = 1; pp < RP; ++pp) {
        r.x += red[tid + pp * NO].x;
        r.y += red[tid + pp * NO].y;
      }
      out[tid] = r;
    }
  }
}

// ---------------------------------------------------------------------------
// pass B: eigen adjoint of one frequency, FP64, matrices in LDS (Psi is read
// from global memory, where it stays in cache).  Writes G2 = 2 G [L][L] and
// CC = conj(C) [L][n] for pass C.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void bwd_eig_kernel(const double* __restrict__ lam,
                                                      const double2* __restrict__ psi,
                                                      const double* __restrict__ g_lam,
                                                      const double2* __restrict__ rpart, int S,
                                                      double2* __restrict__ g2,
                                                      double2* __restrict__ cc, BinTable bt,
                                                      int L, int n, double eps, double gap) {
  extern __shared__ double2 e_lds[];
  const int LD = L + 1;
  double2* A = e_lds;            // g_Psi, then K
  double2* B = A + L * LD;       // X, then Psi K
  __shared__ double lm[BWD_MAXL], sc[BWD_MAXL], gl[BWD_MAXL], dg[BWD_MAXL];
  __shared__ int piv[BWD_MAXL];
  const int s = blockIdx.x;
  const int k = bt.k[s];
  const int tid = threadIdx.x;
  const double* lk = lam + (int64_t)k * L;
  const double2* Pk = psi + (int64_t)k * L * L;      // Pk[l * L + j] = psi_j[l]

  for (int i = tid; i < L; i += blockDim.x) lm[i] = lk[i];
  __syncthreads();
  const double l0 = lm[0];
  for (int j = tid; j < L; j += blockDim.x) {
    const bool valid = j < n && l0 > 0.0 && lm[j] > eps * l0;
    sc[j] = valid ? 1.0 / sqrt(lm[j]) : 0.0;
    gl[j] = g_lam ? g_lam[(int64_t)s * L + j] : 0.0;
  }
  // R summed over the partials in a fixed order (A[l][j], j < n; zero elsewhere)
  for (int idx = tid; idx < L * L; idx += blockDim.x) {
    const int l = idx / L, j = idx % L;
    double2 r = make_double2(0.0, 0.0);
    if (j < n && rpart) {
      const double2* rp = rpart + (int64_t)s * S * L * n + l * n + j;
      for (int pp = 0; pp < S; ++pp) {
        r.x += rp[(int64_t)pp * L * n].x;
        r.y += rp[(int64_t)pp * L * n].y;
      }
    }
    A[l * LD + j] = r;
  }
  __syncthreads();
  // eigenvalue gradient of the Lambda^{-1/2} scaling, and the pivots
  for (int j = tid; j < L; j += blockDim.x) {
    if (sc[j] > 0.0) {
      double re = 0.0;
      for (int l = 0; l < L; ++l) {
        const double2 p = Pk[l * L + j], r = A[l * LD + j];
        re += p.x * r.x + p.y * r.y;
      }
      gl[j] += -0.5 * sc[j] * sc[j] * sc[j] * re;
    }
    int pv = 0;
    double best = -1.0;
    for (int l = 0; l < L; ++l) {
      const double2 p = Pk[l * L + j];
      const double m2 = p.x * p.x + p.y * p.y;
      if (m2 > best) {
        best = m2;
        pv = l;
      }
    }
    piv[j] = pv;
  }
  __syncthreads();
  for (int idx = tid; idx < L * L; idx += blockDim.x) {
    const int l = idx / L, j = idx % L;
    A[l * LD + j].x *= sc[j];
    A[l * LD + j].y *= sc[j];
  }
  __syncthreads();
  // derivative of the phase convention
  for (int j = tid; j < L; j += blockDim.x) {
    double im = 0.0;
    for (int l = 0; l < L; ++l) {
      const double2 p = Pk[l * L + j], g = A[l * LD + j];
      im += p.x * g.y - p.y * g.x;
    }
    const double2 pp = Pk[piv[j] * L + j];
    const double r = sqrt(pp.x * pp.x + pp.y * pp.y);
    dg[j] = r > 0.0 ? im / r : 0.0;
  }
  __syncthreads();
  for (int j = tid; j < L; j += blockDim.x) A[piv[j] * LD + j].y -= dg[j];
  __syncthreads();
  // X = Psi^H g_Psi
  for (int idx = tid; idx < L * L; idx += blockDim.x) {
    const int i = idx / L, j = idx % L;
    double xr = 0.0, xi = 0.0;
    for (int l = 0; l < L; ++l) {
      const double2 p = Pk[l * L + i], g = A[l * LD + j];
      xr += p.x * g.x + p.y * g.y;
      xi += p.x * g.y - p.y * g.x;
    }
    B[i * LD + j] = make_double2(xr, xi);
  }
  __syncthreads();
  // K = diag(g_lambda) + F o (X - X^H) / 2
  const double gthr = gap * fabs(l0);
  for (int idx = tid; idx < L * L; idx += blockDim.x) {
    const int i = idx / L, j = idx % L;
    double2 kv;
    if (i == j) {
      kv = make_double2(gl[i], 0.0);
    } else {
      const double dl = lm[j] - lm[i];
      const double f = fabs(dl) > gthr ? 1.0 / dl : 0.0;
      const double2 x = B[i * LD + j], y = B[j * LD + i];
      kv = make_double2(0.5 * f * (x.x - y.x), 0.5 * f * (x.y + y.y));
    }
    A[i * LD + j] = kv;
  }
  __syncthreads();
  // Psi K
  for (int idx = tid; idx < L * L; idx += blockDim.x) {
    const int a = idx / L, c = idx % L;
    double tr = 0.0, ti = 0.0;
    for (int b = 0; b < L; ++b) {
      const double2 p = Pk[a * L + b], kv = A[b * LD + c];
      tr += p.x * kv.x - p.y * kv.y;
      ti += p.x * kv.y + p.y * kv.x;
    }
    B[a * LD + c] = make_double2(tr, ti);
  }
  __syncthreads();
  // G2 = 2 (Psi K) Psi^H
  double2* g2k = g2 + (int64_t)s * L * L;
  for (int idx = tid; idx < L * L; idx += blockDim.x) {
    const int a = idx / L, d = idx % L;
    double gr = 0.0, gi = 0.0;
    for (int c = 0; c < L; ++c) {
      const double2 t = B[a * LD + c], p = Pk[d * L + c];
      gr += t.x * p.x + t.y * p.y;
      gi += t.y * p.x - t.x * p.y;
    }
    g2k[idx] = make_double2(2.0 * gr, 2.0 * gi);
  }
  if (n > 0) {
    double2* cck = cc + (int64_t)s * L * n;
    for (int idx = tid; idx < L * n; idx += blockDim.x) {
      const int l = idx / n, j = idx % n;
      const double2 p = Pk[l * L + j];
      cck[idx] = make_double2(p.x * sc[j], -p.y * sc[j]);
    }
  }
}

// ---------------------------------------------------------------------------
// pass C: g_qhat[s][l][m] = sum_j CC[l][j] g_phi[s][j][m]
//                          + W_m sum_i G2[i][l] qhat[k][i][m]
// One thread per degree of freedom holds its Z = L + n inputs in registers
// (ZB >= Z), so qhat may be overwritten in place; the coefficients are read
// from LDS (the same address across the wavefront).
// ---------------------------------------------------------------------------
template <typename TC, int ZB>
__global__ __launch_bounds__(256) void bwd_gq_kernel(const cpx_t<TC>* qrows, int q_by_k,
                                                     const cpx_t<TC>* __restrict__ g_phi,
                                                     const double2* __restrict__ g2,
                                                     const double2* __restrict__ cc,
                                                     const double* __restrict__ weights,
                                                     cpx_t<TC>* g_qhat, BinTable bt, int64_t M,
                                                     int L, int n) {
  using C = cpx_t<TC>;
  extern __shared__ char c_lds[];
  C* coef = reinterpret_cast<C*>(c_lds);    // [L + n][L]
  const int s = blockIdx.y;
  const int k = bt.k[s];
  const int tid = threadIdx.x;
  const int Z = L + n;
  for (int idx = tid; idx < Z * L; idx += blockDim.x) {
    const int r = idx / L, l = idx % L;
    const double2 v = r < L ? g2[((int64_t)s * L + r) * L + l] : cc[((int64_t)s * L + l) * n + (r - L)];
    coef[idx] = C{(TC)v.x, (TC)v.y};
  }
  __syncthreads();
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + tid;
  if (m >= M) return;
  const C* qk = qrows + (int64_t)(q_by_k ? k : s) * L * M + m;
  const C* gk = g_phi ? g_phi + (int64_t)s * n * M + m : nullptr;
  C* out = g_qhat + (int64_t)s * L * M + m;
  const TC wm = (TC)weights[m];
  {
    C z[ZB];
#pragma unroll
    for (int i = 0; i < ZB; ++i) {
      C v{0, 0};
      if (i < L) {
        const C x = qk[(int64_t)i * M];
        v = C{x.x * wm, x.y * wm};
      } else if (i < Z) {
        v = gk[(int64_t)(i - L) * M];
      }
      z[i] = v;
    }
    for (int l = 0; l < L; ++l) {
      TC ar = 0, ai = 0;
#pragma unroll
      for (int i = 0; i < ZB; ++i) {
        if (i < Z) {
          const C c = coef[i * L + l];
          ar += c.x * z[i].x - c.y * z[i].y;
          ai += c.x * z[i].y + c.y * z[i].x;
        }
      }
      out[(int64_t)l * M] = C{ar, ai};
    }
  }
}

// ---------------------------------------------------------------------------
// pass D: adjoint of the windowed one-sided DFT, overlap-add and mean removal.
// Same tiling as the forward transform: a workgroup owns T = 2 NPAIR degrees
// of freedom and runs all L blocks in order.
// ---------------------------------------------------------------------------
template <int SH, typename T>
__device__ __forceinline__ void shift_down(T (&a)[8]) {
#pragma unroll
  for (int r = 0; r < 8; ++r) a[r] = r + SH < 8 ? a[r + SH] : (T)0;
}

template <int NF, typename TC, typename TOUT, int NPAIR>
__global__ __launch_bounds__(NPAIR*(NF / 8)) void bwd_fft_kernel(
    const cpx_t<TC>* __restrict__ gqh, const double* __restrict__ window,
    const cpx_t<TC>* __restrict__ tw, const double2* __restrict__ what, TOUT* __restrict__ g_q,
    BinTable bt, MeanList ml, int64_t M, int64_t nt, int step, int L, double kappa) {
  using C = cpx_t<TC>;
  constexpr int P = NF / 8;
  constexpr int T = 2 * NPAIR;
  constexpr int NTH = NPAIR * P;
  constexpr int G = NTH / T;              // P / 2 lanes share one degree of freedom below
  constexpr int LDP = NF + NF / 8 + 1;
  constexpr int K = NF / 2 + 1;
  constexpr bool TWL = sizeof(TC) == 4;
  static_assert(P >= 2, "the adjoint transform needs nfft >= 16");
  __shared__ C lds[NPAIR * LDP];
  __shared__ C twl[TWL ? NF : 1];
  __shared__ int16_t sl[K];
  __shared__ double red[NTH];
  __shared__ double cmean[T];

  const int tid = threadIdx.x;
  const int f = tid / P;
  const int j = tid % P;
  const int64_t m0 = (int64_t)blockIdx.x * T;
  const int64_t ma = m0 + 2 * f, mb = ma + 1;
  const bool va = ma < M, vb = mb < M;
  C* buf = lds + f * LDP;

  TC w[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) w[r] = (TC)(0.5 * kappa * window[j + r * P]);
  const C* twp = tw;
  if constexpr (TWL) {
    for (int i = tid; i < NF; i += NTH) twl[i] = tw[i];
    twp = twl;
  }
  for (int i = tid; i < K; i += NTH) sl[i] = bt.slot[i];
  __syncthreads();

  // mean adjoint: cmean[d] = (kappa / nt) sum_l sum_k Re(g[k][l][m0 + d] conj(What_k))
  {
    const int d = tid % T, g = tid / T;
    const int64_t m = m0 + d;
    const int nb = ml.n >= 0 ? ml.n : bt.n;
    double acc = 0.0;
    if (m < M) {
      for (int it = g; it < nb * L; it += G) {
        const int b = it / L, l = it % L;
        int sk;
        double wr, wi;
        if (ml.n >= 0) {
          sk = ml.slot[b];
          wr = ml.wr[b];
          wi = ml.wi[b];
        } else {
          sk = b;
          const double2 wv = what[bt.k[b]];
          wr = wv.x;
          wi = wv.y;
        }
        const C v = gqh[((int64_t)sk * L + l) * M + m];
        acc += (double)v.x * wr + (double)v.y * wi;
      }
    }
    red[tid] = acc;
    __syncthreads();
    if (tid < T) {
      double c = 0.0;
      for (int gg = 0; gg < G; ++gg) c += red[tid + gg * T];
      cmean[tid] = c * kappa / (double)nt;
    }
    __syncthreads();
  }
  const TC ca = (TC)cmean[2 * f], cb = (TC)cmean[2 * f + 1];

  TOUT* ra = g_q + (va ? ma : 0) * nt;
  TOUT* rb = g_q + (vb ? mb : 0) * nt;
  TC acca[8], accb[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) acca[r] = accb[r] = (TC)0;
  const int shift = step / P;

  for (int l = 0; l < L; ++l) {
    // conj(Z) of every pair of the tile; frequencies outside the selection are zero
    for (int idx = tid; idx < K * NPAIR; idx += NTH) {
      const int k = idx / NPAIR, ff = idx % NPAIR;
      const int sk = sl[k];
      C ga{0, 0}, gb{0, 0};
      const int64_t mA = m0 + 2 * ff;
      if (sk >= 0) {
        const C* src = gqh + ((int64_t)sk * L + l) * M;
        if (mA < M) ga = src[mA];
        if (mA + 1 < M) gb = src[mA + 1];
      }
      C* row = lds + ff * LDP;
      if (k == 0 || k == NF / 2) {
        row[pad8(k)] = C{(TC)2 * ga.x, (TC)-2 * gb.x};
      } else {
        row[pad8(k)] = C{ga.x - gb.y, -ga.y - gb.x};
        row[pad8(NF - k)] = C{ga.x + gb.y, ga.y - gb.x};
      }
    }
    __syncthreads();
    C v[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = buf[pad8(j + r * P)];
    xbarrier<(P <= 64)>();
    stockham<NF, 1>(v, buf, j, twp);
    // g_x = kappa w (1/2 Re V) for a, kappa w (-1/2 Im V) for b
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      acca[r] += w[r] * v[r].x;
      accb[r] -= w[r] * v[r].y;
    }
    // samples that no later block touches are final
    const int nw = l == L - 1 ? 8 : shift;
    const int64_t t0 = (int64_t)l * step + j;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      if (r < nw) {
        const int64_t t = t0 + r * P;
        if (va) ra[t] = (TOUT)(acca[r] - ca);
        if (vb) rb[t] = (TOUT)(accb[r] - cb);
      }
    }
    if (shift == 2) {
      shift_down<2>(acca);
      shift_down<2>(accb);
    } else if (shift == 4) {
      shift_down<4>(acca);
      shift_down<4>(accb);
    } else {
      shift_down<8>(acca);
      shift_down<8>(accb);
    }
    __syncthreads();
  }
  // samples after the last block only enter through the mean
  for (int64_t t = (int64_t)(L - 1) * step + NF + j; t < nt; t += P) {
    if (va) ra[t] = (TOUT)(-ca);
    if (vb) rb[t] = (TOUT)(-cb);
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace {

struct BwdLayout {
  size_t mean = 0, sel = 0, rpart = 0, g2 = 0, cc = 0, total = 0;
};

size_t round256(size_t x) { return (x + 255) / 256 * 256; }

BwdLayout bwd_layout(const Plan& p) {
  const size_t L = (size_t)p.nblocks, K = (size_t)p.nfreq;
  const size_t parts = K > (size_t)BWD_PARTS ? K : (size_t)BWD_PARTS;
  BwdLayout b;
  b.mean = 0;
  b.sel = round256(sizeof(double) * (size_t)p.M);
  b.rpart = b.sel + round256(sizeof(int) * K);
  b.g2 = b.rpart + round256(sizeof(double2) * parts * L * L);
  b.cc = b.g2 + round256(sizeof(double2) * K * L * L);
  b.total = b.cc + round256(sizeof(double2) * K * L * L);
  return b;
}

template <int NF, typename TC, typename TOUT>
spod_status launch_bwd_fft_nf(const Plan& p, const void* gqh, void* g_q, const BinTable& bt,
                              const MeanList& ml, hipStream_t st) {
  // complex64: 32 degrees of freedom per tile, so every frequency row is read
  // in runs of 256 bytes (as the forward transform writes them)
  using S = FftShape<NF, sizeof(TC) == 4 ? 16 : 8>;
  using C = cpx_t<TC>;
  const int64_t ntiles = (p.M + S::T - 1) / S::T;
  if (ntiles > 0x7fffffff) return fail(SPOD_ERR_UNSUPPORTED, "too many tiles");
  const void* tw = sizeof(TC) == 4 ? (const void*)p.d_tw32 : (const void*)p.d_tw64;
  hipLaunchKernelGGL((bwd_fft_kernel<NF, TC, TOUT, S::NPAIR>), dim3((unsigned)ntiles),
                     dim3(S::NPAIR * S::P), 0, st, static_cast<const C*>(gqh), p.d_window,
                     static_cast<const C*>(tw), p.d_what, static_cast<TOUT*>(g_q), bt, ml,
                     (int64_t)p.M, (int64_t)p.nt, (int)p.step, (int)p.nblocks, p.kappa);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPOD_OK : hip_fail(e, "bwd_fft_kernel");
}

template <typename TC, typename TOUT>
spod_status launch_bwd_fft(const Plan& p, const void* gqh, void* g_q, const BinTable& bt,
                           const MeanList& ml, hipStream_t st) {
  switch (p.nfft) {
    case 16: return launch_bwd_fft_nf<16, TC, TOUT>(p, gqh, g_q, bt, ml, st);
    case 32: return launch_bwd_fft_nf<32, TC, TOUT>(p, gqh, g_q, bt, ml, st);
    case 64: return launch_bwd_fft_nf<64, TC, TOUT>(p, gqh, g_q, bt, ml, st);
    case 128: return launch_bwd_fft_nf<128, TC, TOUT>(p, gqh, g_q, bt, ml, st);
    case 256: return launch_bwd_fft_nf<256, TC, TOUT>(p, gqh, g_q, bt, ml, st);
    case 512: return launch_bwd_fft_nf<512, TC, TOUT>(p, gqh, g_q, bt, ml, st);
    case 1024: return launch_bwd_fft_nf<1024, TC, TOUT>(p, gqh, g_q, bt, ml, st);
  }
  return fail(SPOD_ERR_UNSUPPORTED, "nfft");
}

template <typename TC>
spod_status launch_bwd_t(const Plan& p, spod_dtype dtype, const void* qrows, int q_by_k,
                         const double* lam, const void* psi, const double* g_lam,
                         const void* g_phi, int n, void* g_qhat, void* g_q, char* ws,
                         const BinTable& bt, const MeanList& ml, hipStream_t st) {
  using C = cpx_t<TC>;
  const BwdLayout lay = bwd_layout(p);
  const int L = (int)p.nblocks, nb = bt.n;
  double2* rpart = reinterpret_cast<double2*>(ws + lay.rpart);
  double2* g2 = reinterpret_cast<double2*>(ws + lay.g2);
  double2* cc = reinterpret_cast<double2*>(ws + lay.cc);
  hipError_t e;

  // A
  int S = 0;
  if (g_phi) {
    const int64_t parts = p.nfreq > BWD_PARTS ? p.nfreq : BWD_PARTS;
    int64_t s = parts / nb;
    const int64_t cap = (p.M + 1023) / 1024;
    if (s > cap) s = cap;
    if (s < 1) s = 1;
    int64_t per = (p.M + s - 1) / s;
    per = (per + BWD_TM - 1) / BWD_TM * BWD_TM;
    S = (int)((p.M + per - 1) / per);
    const size_t lds = (sizeof(C) * ((size_t)(L + n) * BWD_TMP + 1) / 16 * 16) + sizeof(double2) * 256;
    e = hipFuncSetAttribute((const void*)bwd_r_kernel<TC>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
    hipLaunchKernelGGL(bwd_r_kernel<TC>, dim3((unsigned)S, (unsigned)nb), dim3(256), lds, st,
                       static_cast<const C*>(qrows), q_by_k, static_cast<const C*>(g_phi), rpart,
                       bt, (int64_t)p.M, L, n, S, per);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "bwd_r_kernel");
  }
  // B
  {
    const size_t lds = sizeof(double2) * 2 * (size_t)L * (L + 1);
    e = hipFuncSetAttribute((const void*)bwd_eig_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
    hipLaunchKernelGGL(bwd_eig_kernel, dim3((unsigned)nb), dim3(256), lds, st, lam,
                       static_cast<const double2*>(psi), g_lam, g_phi ? rpart : nullptr, S, g2,
                       cc, bt, L, n, is_complex128(p) ? 1e-12 : 1e-6, 1e-12);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "bwd_eig_kernel");
  }
  // C
  {
    const int Z = L + n;
    const size_t lds = sizeof(C) * (size_t)Z * L;
    dim3 grid((unsigned)((p.M + 255) / 256), (unsigned)nb);
    const C* qr = static_cast<const C*>(qrows);
    const C* gp = static_cast<const C*>(g_phi);
    C* out = static_cast<C*>(g_qhat);
    auto go = [&](auto kern) -> spod_status {
      hipError_t e2 = hipFuncSetAttribute((const void*)kern,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e2 != hipSuccess) return hip_fail(e2, "hipFuncSetAttribute");
      hipLaunchKernelGGL(kern, grid, dim3(256), lds, st, qr, q_by_k, gp, g2, cc, p.d_weights,
                         out, bt, (int64_t)p.M, L, n);
      e2 = hipGetLastError();
      return e2 == hipSuccess ? SPOD_OK : hip_fail(e2, "bwd_gq_kernel");
    };
    spod_status r;
    if (Z <= 16) r = go(bwd_gq_kernel<TC, 16>);
    else if (Z <= 24) r = go(bwd_gq_kernel<TC, 24>);
    else if (Z <= 32) r = go(bwd_gq_kernel<TC, 32>);
    else if (Z <= 40) r = go(bwd_gq_kernel<TC, 40>);
    else if (Z <= 48) r = go(bwd_gq_kernel<TC, 48>);
    else if (Z <= 64) r = go(bwd_gq_kernel<TC, 64>);
    else r = go(bwd_gq_kernel<TC, 128>);
    if (r != SPOD_OK) return r;
  }
  // D
  if (p.general) {
    // any block length: the adjoint of the mixed-radix transform
    GenAdjBins gb;
    gb.n = bt.n;
    for (int i = 0; i < bt.n; ++i) gb.k[i] = bt.k[i];
    GenAdjMean gm{};
    gm.n = ml.n;
    for (int i = 0; i < ml.n; ++i) {
      gm.slot[i] = ml.slot[i];
      gm.wr[i] = ml.wr[i];
      gm.wi[i] = ml.wi[i];
    }
    return launch_general_adjoint(p, g_qhat, dtype, g_q, gb, gm, st);
  }
  return dtype == SPOD_F32 ? launch_bwd_fft<TC, float>(p, g_qhat, g_q, bt, ml, st)
                           : launch_bwd_fft<TC, double>(p, g_qhat, g_q, bt, ml, st);
}

}  // namespace

size_t backward_workspace(const Plan& p) { return bwd_layout(p).total; }

spod_status launch_backward(const Plan& p, const void* q, spod_dtype dtype, const void* qhat,
                            const double* lam, const void* psi, const double* g_lam,
                            const void* g_phi, int n_modes, const int32_t* bins, int n_bins,
                            void* g_qhat, void* g_q, void* ws, hipStream_t st) {
  const int K = (int)p.nfreq;
  // a power-of-two transform keeps its K <= 513 bins in the table's inverse
  // map; any other block length takes at most 513 selected bins (the inverse
  // map is then not used)
  if ((!p.general && K > BWD_MAXK) || p.nblocks > BWD_MAXL) return fail(SPOD_ERR_UNSUPPORTED, "shape");
  if (n_bins > BWD_MAXK)
    return fail(SPOD_ERR_UNSUPPORTED, "at most 513 bins: pass a selection (bins) for nfft above 1024");
  if (p.general && !qhat)
    return fail(SPOD_ERR_UNSUPPORTED,
                "pass the Fourier blocks (qhat) for a block length other than a power of two <= 1024");
  BinTable bt;
  bt.n = n_bins;
  for (int k = 0; k < BWD_MAXK; ++k) bt.slot[k] = -1;
  for (int s = 0; s < n_bins; ++s) {
    const int k = bins ? bins[s] : s;
    bt.k[s] = (int16_t)k;
    if (k < BWD_MAXK) bt.slot[k] = (int16_t)s;
  }
  // the selected bins where the window's DFT is not zero
  auto slot_of = [&](int k) {
    for (int s = 0; s < n_bins; ++s)
      if (bt.k[s] == k) return s;
    return -1;
  };
  MeanList ml{};
  if (p.n_mean_bins >= 0) {
    ml.n = 0;
    for (int i = 0; i < p.n_mean_bins; ++i) {
      const int s = slot_of(p.mean_bin[i]);
      if (s < 0) continue;
      ml.slot[ml.n] = s;
      ml.wr[ml.n] = p.what_re[i];
      ml.wi[ml.n] = p.what_im[i];
      ++ml.n;
    }
  } else {
    ml.n = -1;
  }
  char* w = static_cast<char*>(ws);
  const BwdLayout lay = bwd_layout(p);
  const void* qrows = qhat;
  int q_by_k = 1;
  if (!qhat) {
    // recompute the Fourier blocks of the selected bins into g_qhat
    FftSel fs;
    std::vector<int> slot(K);
    for (int k = 0; k < K; ++k) slot[k] = bt.slot[k];
    if (bins) {
      int* d_sel = reinterpret_cast<int*>(w + lay.sel);
      hipLaunchKernelGGL(write_sel_kernel, dim3(1), dim3(256), 0, st, bt, d_sel);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return hip_fail(e, "write_sel_kernel");
      fs.d_sel = d_sel;
      fs.nsel = n_bins;
      fs.h_slot = slot.data();
    }
    spod_status r = launch_blocks_fft(p, q, dtype, g_qhat, nullptr, ws, st, fs);
    if (r != SPOD_OK) return r;
    qrows = g_qhat;
    q_by_k = 0;
  }
  if (is_complex128(p))
    return launch_bwd_t<double>(p, dtype, qrows, q_by_k, lam, psi, g_lam, g_phi, n_modes, g_qhat,
                                g_q, w, bt, ml, st);
  return launch_bwd_t<float>(p, dtype, qrows, q_by_k, lam, psi, g_lam, g_phi, n_modes, g_qhat,
                             g_q, w, bt, ml, st);
}

}  // namespace spod
