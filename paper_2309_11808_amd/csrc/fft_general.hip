// Steps 1-2 of SPOD for any block length N_f (eq. (blocks), (blocks-ft),
// (blocks-k)): Welch blocks, window and one-sided DFT in time, where N_f is
// not a power of two or is above the register-resident transform's 1024 (the
// paper's hourly data use N_f = 8760 = 2^3 3 5 73).
//
// One workgroup of 1024 threads owns one pair of degrees of freedom: the two
// real rows are packed as a + i c, transformed once, and split
// with the two-for-one identity.  The transform is a self-sorting mixed-radix
// one (decimation in frequency) held in LDS: for N = r_0 r_1 ... the stage of
// radix r with current length n and stride s maps
//   y[q + s (r p + k)] = W_n^{p k} sum_j x[q + s (p + j n / r)] W_r^{j k},
// every output a direct radix-r sum (so a prime factor such as 73 needs no
// special case).  W_n^{p k} = W_N^{(N / n) p k} is read from the plan's table
// W_N^t (p k < n, so no reduction mod N).  For an odd radix the outputs k and
// r - k come from (r - 1) / 2 terms of the symmetric sums, a quarter of the
// multiplications; a work item takes up to 6 such pairs of one butterfly,
// all lanes of a wavefront the same pairs, so their W_r^{jk} come from the
// plan's per-stage table through scalar loads.  With two LDS buffers a stage
// reads one and writes the other; with one, a thread computes its outputs of
// a stage into registers, the workgroup synchronises, and the outputs
// overwrite the inputs.  The mean comes from the FP64
// mean pass.  A workgroup takes the blocks of its pair in turn, loading the
// next block while it transforms the current one.  Consecutive workgroups of
// one XCD take consecutive pairs, so their 16-byte stores of neighbouring
// degrees of freedom meet in that XCD's L2.
#include <hip/hip_runtime.h>

#include <numeric>

#include <algorithm>

#include "fft_core.h"
#include "internal.h"

namespace spod {
namespace {

constexpr int GEN_THREADS = 1024;

template <typename TC>
__device__ __forceinline__ cpx_t<TC> mk(TC x, TC y) {
  cpx_t<TC> c;
  c.x = x;
  c.y = y;
  return c;
}

// Workgroup barrier for LDS traffic only: every wave's LDS reads and writes
// are complete, while its global loads (the next block's samples) may still
// be in flight (__syncthreads would wait for those too).  The compiler fences
// keep LDS accesses from moving across it.
__device__ __forceinline__ void lds_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(15 | (3 << 14) | (7 << 4) | (0 << 8));   // lgkmcnt(0) only
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_sched_barrier(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// W_N^t from two tables in LDS, t = 64 a + b: hi[a] = W_N^{64 a} and
// lo[b] = W_N^b, so one complex product (a rounding of the working precision)
// replaces a load from the N-entry table in global memory.  Stages that read
// their twiddles this way wait on no global memory operation, so the stores of
// the previous block stay in flight under them.
template <typename TC>
struct TwSplit {
  const cpx_t<TC>* hi;
  const cpx_t<TC>* lo;
  __device__ __forceinline__ cpx_t<TC> operator[](int t) const {
    const cpx_t<TC> a = hi[t >> 6], b = lo[t & 63];
    return mk<TC>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
  }
};

// Quotient and remainder of a / d for 0 <= a < 2^24 and 1 <= d, from the
// precomputed float reciprocal inv = 1/d: the product is within one of the
// true quotient, and one correction step makes it exact.
struct DivMod {
  int q, r;
};
__device__ __forceinline__ DivMod divmod(int a, int d, float inv) {
  int q = (int)((float)a * inv);
  int r = a - q * d;
  if (r < 0) {
    --q;
    r += d;
  } else if (r >= d) {
    ++q;
    r -= d;
  }
  return {q, r};
}

// One output of an even-radix stage: y[o] = W_n^{p k} sum_j x[q + s(p + j m)] W_r^{j k}
// (four independent partial sums, t = j k mod r).
template <typename TC, typename TW>
__device__ __forceinline__ cpx_t<TC> even_output(const cpx_t<TC>* __restrict__ X,
                                                 const cpx_t<TC>* __restrict__ Wr,
                                                 const TW tw, int o, int r,
                                                 int s, int m, int wn, int N, float inv_s,
                                                 float inv_r) {
  using C = cpx_t<TC>;
  const DivMod a = divmod(o, s, inv_s);       // o = qq + s * rest
  const DivMod b = divmod(a.q, r, inv_r);     // rest = k + r * pp
  const int qq = a.r, k = b.r, pp = b.q;
  const int base = qq + s * pp, js = s * m;
  TC ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
  int j = 0, t = 0;
  for (; j + 4 <= r; j += 4) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const C xv = X[base + (j + v) * js];
      const C wv = Wr[t];
      ar[v] += xv.x * wv.x - xv.y * wv.y;
      ai[v] += xv.x * wv.y + xv.y * wv.x;
      t += k;
      if (t >= r) t -= r;
    }
  }
  for (; j < r; ++j) {
    const C xv = X[base + j * js];
    const C wv = Wr[t];
    ar[0] += xv.x * wv.x - xv.y * wv.y;
    ai[0] += xv.x * wv.y + xv.y * wv.x;
    t += k;
    if (t >= r) t -= r;
  }
  const TC sr = (ar[0] + ar[1]) + (ar[2] + ar[3]), si = (ai[0] + ai[1]) + (ai[2] + ai[3]);
  const C t2 = tw[wn * pp * k];
  return mk<TC>(sr * t2.x - si * t2.y, sr * t2.y + si * t2.x);
}

// Work item it of an odd-radix stage: with a_j = x_j + x_{r-j}, b_j =
// x_j - x_{r-j} and W_r^{jk} = c - i s, the outputs k and r - k share the sums
// A = sum_{j <= (r-1)/2} a_j c and B = sum b_j s:  y_k = x_0 + A - i B,
// y_{r-k} = x_0 + A + i B (then W_n^{p k}, W_n^{p(r-k)}).  kk = it / NB in
// [0, (r-1)/2]; consecutive items are consecutive butterflies.
template <typename TC, typename TW>
__device__ __forceinline__ void odd_pair(const cpx_t<TC>* __restrict__ X,
                                         const cpx_t<TC>* __restrict__ Wr,
                                         const TW tw, int it, int NB, int r,
                                         int s, int m, int wn, int N, cpx_t<TC>& y0,
                                         cpx_t<TC>& y1, int& o0, int& o1) {
  using C = cpx_t<TC>;
  const int kk = it / NB, bf = it - kk * NB;
  const int qq = bf % s, pp = bf / s;
  const int base = qq + s * pp, js = s * m;
  const C x0 = X[base];
  TC Ar = 0, Ai = 0, Br = 0, Bi = 0;
  int t = 0;
  for (int j = 1; 2 * j < r; ++j) {
    t += kk;
    if (t >= r) t -= r;
    const C xa = X[base + j * js], xb = X[base + (r - j) * js];
    const C w = Wr[t];
    const TC c = w.x, sn = -w.y;
    Ar += (xa.x + xb.x) * c;
    Ai += (xa.y + xb.y) * c;
    Br += (xa.x - xb.x) * sn;
    Bi += (xa.y - xb.y) * sn;
  }
  const TC ykr = x0.x + Ar + Bi, yki = x0.y + Ai - Br;
  const TC yrr = x0.x + Ar - Bi, yri = x0.y + Ai + Br;
  const C t0 = tw[wn * pp * kk];
  const C t1 = tw[wn * pp * (r - kk)];
  y0 = mk<TC>(ykr * t0.x - yki * t0.y, ykr * t0.y + yki * t0.x);
  y1 = mk<TC>(yrr * t1.x - yri * t1.y, yrr * t1.y + yri * t1.x);
  o0 = qq + s * (r * pp + kk);
  o1 = kk > 0 ? qq + s * (r * pp + r - kk) : -1;
}

// One butterfly of a radix-2, 4 or 8 stage: the RS inputs x[q + s(p + j m)]
// through the in-register DFT, output k times W_n^{p k}, stored at
// y[q + s(RS p + k)].
template <int RS, typename TC, typename TW>
__device__ __forceinline__ void even_butterfly(const cpx_t<TC>* __restrict__ X,
                                               const TW tw,
                                               cpx_t<TC>* __restrict__ Y, int bf, int s, int m,
                                               int wn, int N, float inv_s) {
  using C = cpx_t<TC>;
  const DivMod a = divmod(bf, s, inv_s);      // bf = qq + s * pp
  const int qq = a.r, pp = a.q;
  const int base = qq + s * pp, js = s * m;
  C x[RS];
#pragma unroll
  for (int j = 0; j < RS; ++j) x[j] = X[base + j * js];
  dft_r<RS>(x);
  const int step = wn * pp;   // W_n^{p k} = W_N^{k step}, k step < N
  int t = 0;
  const int out = qq + s * RS * pp;
  Y[out] = x[0];
#pragma unroll
  for (int k = 1; k < RS; ++k) {
    t += step;
    const C w = tw[t];
    Y[out + s * k] = mk<TC>(x[k].x * w.x - x[k].y * w.y, x[k].x * w.y + x[k].y * w.x);
  }
}

// Work item of an odd-radix stage: the output pairs k_c = g + c G, c < KPT,
// of butterfly bf, with the symmetric sums of odd_pair.  The loads of x_j and
// x_{r-j} and their sum and difference are shared by the KPT pairs.  g is
// the same for every lane of the wavefront (the butterflies of one g are
// padded to a multiple of 64 work items), so the stage's table Tg[j][c] =
// W_r^{(j + 1) k_c} (row g of the plan's odd-stage table) is read at
// wave-uniform addresses, into scalar registers, with no index arithmetic.
// Pairs with k_c >= h = (r + 1) / 2 use the last pair's values and store
// nothing.
template <int KPT, typename TC, typename TW>
__device__ __forceinline__ void odd_uniform(const cpx_t<TC>* __restrict__ X,
                                            const cpx_t<TC>* __restrict__ Tg,
                                            const TW tw,
                                            cpx_t<TC>* __restrict__ Y, int bf, int g, int G, int r,
                                            int s, int m, int wn, float inv_s) {
  using C = cpx_t<TC>;
  const int h = (r + 1) / 2, hm = h - 1;
  const DivMod b = divmod(bf, s, inv_s);      // bf = qq + s * pp
  const int qq = b.r, pp = b.q;
  const int base = qq + s * pp, js = s * m;
  const C x0 = X[base];
  TC ar[KPT], ai[KPT], br[KPT], bi[KPT];
#pragma unroll
  for (int c = 0; c < KPT; ++c) ar[c] = ai[c] = br[c] = bi[c] = 0;
  const C* pa = X + base + js;
  const C* pb = X + base + (r - 1) * js;
  for (int j = 0; j < hm; ++j, pa += js, pb -= js) {
    const C xa = *pa, xb = *pb;
    const TC sr = xa.x + xb.x, si = xa.y + xb.y, dr = xa.x - xb.x, di = xa.y - xb.y;
    const C* w = Tg + j * KPT;
#pragma unroll
    for (int c = 0; c < KPT; ++c) {
      const C wc = w[c];
      ar[c] += sr * wc.x;
      ai[c] += si * wc.x;
      br[c] -= dr * wc.y;
      bi[c] -= di * wc.y;
    }
  }
  // y_k = x0 + A - iB, y_{r-k} = x0 + A + iB, then W_n^{p k}, W_n^{p (r-k)}
  const int wp = wn * pp;
#pragma unroll
  for (int c = 0; c < KPT; ++c) {
    const int k = g + c * G;
    if (k < h) {
      const TC ykr = x0.x + ar[c] + bi[c], yki = x0.y + ai[c] - br[c];
      const C t0 = tw[wp * k];
      Y[qq + s * (r * pp + k)] = mk<TC>(ykr * t0.x - yki * t0.y, ykr * t0.y + yki * t0.x);
      if (k > 0) {
        const TC yrr = x0.x + ar[c] - bi[c], yri = x0.y + ai[c] + br[c];
        const C t1 = tw[wp * (r - k)];
        Y[qq + s * (r * pp + r - k)] = mk<TC>(yrr * t1.x - yri * t1.y, yrr * t1.y + yri * t1.x);
      }
    }
  }
}

// An odd stage of the two-buffer kernel: work items (g, bf) with bf padded to
// NBp, a multiple of 64, so every wavefront has one g.
template <int KPT, typename TC, typename TW>
__device__ __forceinline__ void odd_stage(const cpx_t<TC>* __restrict__ X,
                                          const cpx_t<TC>* __restrict__ T,
                                          const TW tw,
                                          cpx_t<TC>* __restrict__ Y, int tid, int NB, int r, int s,
                                          int m, int wn) {
  const int h = (r + 1) / 2, hm = h - 1, G = (h + KPT - 1) / KPT;
  const int NBp = (NB + 63) & ~63;
  const float inv_nbp = 1.0f / (float)NBp, inv_s = 1.0f / (float)s;
  for (int it = tid; it < NBp * G; it += GEN_THREADS) {
    // NBp G is a multiple of 64: whole wavefronts run this body
    const int g = __builtin_amdgcn_readfirstlane(divmod(it, NBp, inv_nbp).q);
    const int bf = it - g * NBp;
    if (bf < NB)
      odd_uniform<KPT, TC>(X, T + (size_t)g * hm * KPT, tw, Y, bf, g, G, r, s, m, wn, inv_s);
  }
}

// One stage of the two-buffer kernel, X -> Y (W_n^{p k} = tw[wn p k], wn = N / n).
template <typename TC, typename TW>
__device__ __forceinline__ void pp_stage(const cpx_t<TC>* __restrict__ X,
                                         cpx_t<TC>* __restrict__ Y,
                                         const TW tw,
                                         const cpx_t<TC>* __restrict__ Wr,
                                         const cpx_t<TC>* __restrict__ oddw, const Radices& rad,
                                         int st, int tid, int N, int r, int s, int m, int wn) {
  if (r % 2 == 1) {
    const int NB = N / r;
    const cpx_t<TC>* T = oddw + rad.toff[st];
    switch (rad.kpt[st]) {
      case 1: odd_stage<1, TC>(X, T, tw, Y, tid, NB, r, s, m, wn); break;
      case 2: odd_stage<2, TC>(X, T, tw, Y, tid, NB, r, s, m, wn); break;
      case 3: odd_stage<3, TC>(X, T, tw, Y, tid, NB, r, s, m, wn); break;
      case 4: odd_stage<4, TC>(X, T, tw, Y, tid, NB, r, s, m, wn); break;
      case 5: odd_stage<5, TC>(X, T, tw, Y, tid, NB, r, s, m, wn); break;
      default: odd_stage<6, TC>(X, T, tw, Y, tid, NB, r, s, m, wn); break;
    }
    static_assert(GENERAL_MAX_KPT == 6, "one case per output-pair count");
  } else if (r == 8 || r == 4 || r == 2) {
    const float inv_s = 1.0f / (float)s;
    const int NB = N / r;
    for (int bf = tid; bf < NB; bf += GEN_THREADS) {
      if (r == 8) even_butterfly<8, TC>(X, tw, Y, bf, s, m, wn, N, inv_s);
      else if (r == 4) even_butterfly<4, TC>(X, tw, Y, bf, s, m, wn, N, inv_s);
      else even_butterfly<2, TC>(X, tw, Y, bf, s, m, wn, N, inv_s);
    }
  } else {
    const float inv_s = 1.0f / (float)s, inv_r = 1.0f / (float)r;
    for (int o = tid; o < N; o += GEN_THREADS)
      Y[o] = even_output<TC>(X, Wr, tw, o, r, s, m, wn, N, inv_s, inv_r);
  }
}

// The stages of the transform on X (in LDS, natural order in and out); with
// PP the stages alternate between X and Y.  Returns the buffer that holds the
// result.  The caller has synchronised the workgroup after writing X.
template <typename TC, bool PP, int MAXU, int MAXI, typename TW>
__device__ __forceinline__ cpx_t<TC>* dft_stages(cpx_t<TC>* X, cpx_t<TC>* Y,
                                                 const cpx_t<TC>* __restrict__ Wt,
                                                 const TW tw,
                                                 const cpx_t<TC>* __restrict__ oddw,
                                                 const Radices& rad, int tid, int N) {
  using C = cpx_t<TC>;
  int n = N, s = 1, off = 0;
  for (int st = 0; st < rad.n; ++st) {
    const int r = rad.r[st];
    const int m = n / r;
    const int wn = N / n;          // W_n = W_N^(N/n)
    const C* Wr = Wt + off;
    if constexpr (PP) {
      pp_stage<TC>(X, Y, tw, Wr, oddw, rad, st, tid, N, r, s, m, wn);
      lds_barrier();
      C* tmp = X;
      X = Y;
      Y = tmp;
    } else {
      if (r % 2 == 1) {
        const int NB = N / r, items = NB * ((r + 1) / 2);
        C y0[MAXI], y1[MAXI];
        int o0[MAXI], o1[MAXI];
#pragma unroll
        for (int u = 0; u < MAXI; ++u) {
          const int it = tid + u * GEN_THREADS;
          o0[u] = -1;
          if (it < items)
            odd_pair<TC>(X, Wr, tw, it, NB, r, s, m, wn, N, y0[u], y1[u], o0[u], o1[u]);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < MAXI; ++u) {
          if (o0[u] >= 0) {
            X[o0[u]] = y0[u];
            if (o1[u] >= 0) X[o1[u]] = y1[u];
          }
        }
      } else {
        C y[MAXU];
#pragma unroll
        for (int u = 0; u < MAXU; ++u) {
          const int o = tid + u * GEN_THREADS;
          if (o < N)
            y[u] = even_output<TC>(X, Wr, tw, o, r, s, m, wn, N, 1.0f / (float)s, 1.0f / (float)r);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < MAXU; ++u) {
          const int o = tid + u * GEN_THREADS;
          if (o < N) X[o] = y[u];
        }
      }
      __syncthreads();
    }
    n = m;
    s *= r;
    off += r;
  }
  return X;
}

// PP: two LDS buffers, every stage reads one and writes the other (no
// staging registers).  Otherwise one buffer: a thread computes its outputs of
// a stage into registers (MAXU outputs of an even-radix stage, MAXI pairs of
// an odd one, (N / r)(r + 1) / 2 <= 2N / 3 items), the workgroup synchronises,
// and the outputs overwrite the inputs.  A workgroup takes every block of its
// pair in turn; with PP the samples of the next block are loaded into
// registers (MAXR per thread and row) while the current one is transformed.
template <typename TC, typename TIN, bool PP, int MAXU, int MAXI = (2 * MAXU + 2) / 3,
          int MAXR = PP ? MAXU : 1>
__global__ __launch_bounds__(GEN_THREADS) void blocks_dft_general_kernel(
    const TIN* __restrict__ q, const double* __restrict__ mean, const double* __restrict__ window,
    const cpx_t<TC>* __restrict__ tw, cpx_t<TC>* __restrict__ qhat, int64_t M, int64_t nt, int N,
    int step, int L, int K, TC kappa, Radices rad, int64_t per_xcd,
    const cpx_t<TC>* __restrict__ oddw) {
  using C = cpx_t<TC>;
  extern __shared__ unsigned char smem[];
  C* const B0 = reinterpret_cast<C*>(smem);
  C* const B1 = PP ? B0 + N : B0;
  C* Wt = B0 + (PP ? 2 * N : N);  // per stage: W_r^t, t < r, stage after stage
  const int64_t b = blockIdx.x;
  const int64_t pair = (b & 7) * per_xcd + (b >> 3);   // consecutive pairs on one XCD
  const int64_t P = (M + 1) / 2;
  if (pair >= P) return;                       // the same for every thread
  const int64_t m0 = 2 * pair;
  const bool two = m0 + 1 < M;
  const int tid = threadIdx.x;

  int woff = 0;
  for (int st = 0; st < rad.n; ++st) {
    const int r = rad.r[st];
    for (int t = tid; t < r; t += GEN_THREADS) Wt[woff + t] = tw[(N / r) * t];
    woff += r;
  }
  // PP: W_N^t as the product of two short tables after the per-stage ones
  C* const Th = Wt + woff;
  C* const Tl = Th + ((N + 63) >> 6);
  if constexpr (PP) {
    for (int a = tid; 64 * a < N; a += GEN_THREADS) Th[a] = tw[64 * a];
    for (int b = tid; b < 64 && b < N; b += GEN_THREADS) Tl[b] = tw[b];
  }
  const double mu0 = mean[m0], mu1 = two ? mean[m0 + 1] : 0.0;
  const TIN* r0 = q + m0 * nt;
  const TIN* r1 = q + (two ? m0 + 1 : m0) * nt;
  TIN pa[MAXR], pb[MAXR];                      // the next block's samples (PP)
  double wr[MAXR];                             // this thread's window samples (PP)
  if constexpr (PP) {
#pragma unroll
    for (int u = 0; u < MAXR; ++u) {
      const int n = tid + u * GEN_THREADS;
      pa[u] = n < N ? r0[n] : (TIN)0;
      pb[u] = n < N ? r1[n] : (TIN)0;
      wr[u] = n < N ? window[n] : 0.0;
    }
  }
  const TC h = (TC)0.5 * kappa;
  const bool vec = two && (M % 2 == 0);        // 16-byte aligned pair (m0 even)

  for (int l = 0; l < L; ++l) {
    C* X = B0;
    C* Y = B1;
    // windowed, mean-free samples of both rows as one complex sequence
    if constexpr (PP) {
#pragma unroll
      for (int u = 0; u < MAXR; ++u) {
        const int n = tid + u * GEN_THREADS;
        if (n < N) {
          const double w = wr[u];
          X[n] = mk<TC>((TC)(((double)pa[u] - mu0) * w),
                        (TC)(two ? ((double)pb[u] - mu1) * w : 0.0));
        }
      }
      if (l + 1 < L) {
        const int64_t o = (int64_t)(l + 1) * step;
#pragma unroll
        for (int u = 0; u < MAXR; ++u) {
          const int n = tid + u * GEN_THREADS;
          pa[u] = n < N ? r0[o + n] : (TIN)0;
          pb[u] = n < N ? r1[o + n] : (TIN)0;
        }
      }
    } else {
      const int64_t o = (int64_t)l * step;
      for (int n = tid; n < N; n += GEN_THREADS) {
        const double w = window[n];
        const double a = ((double)r0[o + n] - mu0) * w;
        const double c = two ? ((double)r1[o + n] - mu1) * w : 0.0;
        X[n] = mk<TC>((TC)a, (TC)c);
      }
    }
    if constexpr (PP) lds_barrier();
    else __syncthreads();

    if constexpr (PP) {
      X = dft_stages<TC, PP, MAXU, MAXI>(X, Y, Wt, TwSplit<TC>{Th, Tl}, oddw, rad, tid, N);
      // an empty asm that reads the next block's samples takes the wait for
      // them (and for this thread's earlier stores) here, after the stages,
      // so the stores of the previous block drain under the window and stages
      if (l + 1 < L) {
#pragma unroll
        for (int u = 0; u < MAXR; ++u) asm volatile("" ::"v"(pa[u]), "v"(pb[u]));
      }
    } else {
      X = dft_stages<TC, PP, MAXU, MAXI>(X, Y, Wt, tw, oddw, rad, tid, N);
    }

    // two-for-one split: A = (Z_k + conj Z_{N-k}) / 2, C = (Z_k - conj Z_{N-k}) / 2i
    const C* Z = X;
    for (int k = tid; k < K; k += GEN_THREADS) {
      const C z = Z[k], zc = Z[k == 0 ? 0 : N - k];
      const C a = mk<TC>(h * (z.x + zc.x), h * (z.y - zc.y));
      const C c = mk<TC>(h * (z.y + zc.y), h * (zc.x - z.x));
      C* dst = qhat + ((int64_t)k * L + l) * M + m0;
      if constexpr (sizeof(TC) == 4) {
        if (vec) {
          *reinterpret_cast<float4*>(dst) = make_float4(a.x, a.y, c.x, c.y);
          continue;
        }
      }
      dst[0] = a;
      if (two) dst[1] = c;
    }
    // Z is read before the next block writes B0
    if constexpr (PP) lds_barrier();
    else __syncthreads();
  }
}

template <typename TC, typename TIN, bool PP, int MAXU>
spod_status launch_general_pp(const Plan& p, const TIN* q, const double* mean, void* qhat,
                              size_t lds, hipStream_t st) {
  using C = cpx_t<TC>;
  const void* fn = reinterpret_cast<const void*>(&blocks_dft_general_kernel<TC, TIN, PP, MAXU>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
  const int64_t P = (p.M + 1) / 2;
  const int64_t per_xcd = (P + 7) / 8;
  const int64_t wgs = 8 * per_xcd;
  if (wgs > 0x7fffffffLL) return fail(SPOD_ERR_UNSUPPORTED, "general transform grid too large");
  const C* tw = static_cast<const C*>(sizeof(TC) == 8 ? (const void*)p.d_tw64 : (const void*)p.d_tw32);
  hipLaunchKernelGGL((blocks_dft_general_kernel<TC, TIN, PP, MAXU>), dim3((unsigned)wgs),
                     dim3(GEN_THREADS), lds, st, q, mean, p.d_window, tw, static_cast<C*>(qhat),
                     (int64_t)p.M, (int64_t)p.nt, (int)p.nfft, (int)p.step, (int)p.nblocks,
                     (int)p.nfreq, (TC)p.kappa, p.radices, per_xcd,
                     static_cast<const C*>(sizeof(TC) == 8 ? (const void*)p.d_oddw64
                                                           : (const void*)p.d_oddw32));
  e = hipGetLastError();
  return e == hipSuccess ? SPOD_OK : hip_fail(e, "blocks_dft_general_kernel");
}

template <typename TC, typename TIN, int MAXU>
spod_status launch_general_t(const Plan& p, const TIN* q, const double* mean, void* qhat,
                             hipStream_t st) {
  using C = cpx_t<TC>;
  int sum_r = 0;
  for (int i = 0; i < p.radices.n; ++i) sum_r += p.radices.r[i];
  constexpr size_t LDS_MAX = 160 * 1024;
  const size_t two_buf =
      sizeof(C) * (2 * (size_t)p.nfft + (size_t)sum_r + ((size_t)p.nfft + 63) / 64 + 64);
  // two buffers and the twiddle tables: complex64 N <= ~10080, complex128
  // <= ~5000, so at most ceil(10240 / 1024) samples per thread and row to
  // prefetch
  if (two_buf <= LDS_MAX)
    return launch_general_pp<TC, TIN, true, (sizeof(C) == 8 ? 10 : 5)>(p, q, mean, qhat, two_buf, st);
  const size_t one_buf = sizeof(C) * ((size_t)p.nfft + (size_t)sum_r);
  if (one_buf > LDS_MAX)
    return fail(SPOD_ERR_UNSUPPORTED, "block and twiddles exceed the 160 KiB of LDS");
  return launch_general_pp<TC, TIN, false, MAXU>(p, q, mean, qhat, one_buf, st);
}

// Adjoint of the general transform for the selected bins (not in the paper;
// the reverse of eq. (blocks-ft) and of the mean removal).  With
// Qhat_k = kappa sum_n w[n] x[n] W_N^{kn} on the one-sided bins, and
// g = dE/dRe + i dE/dIm,
//   dE/dx[n] = kappa w[n] Re sum_k g_k W_N^{-kn} = kappa w[n] (1/2) sum_k H_k W_N^{-kn}
// over all N bins with H_0 = 2 Re g_0, H_{N/2} = 2 Re g_{N/2} (N even),
// H_k = g_k and H_{N-k} = conj g_k.  Two rows a, c are packed as
// Z = H_a + i H_c; the same forward stages give D = DFT(conj Z), and
// (1/2) conj D carries row a in its real part and row c in its imaginary part.
// The blocks are added into g_q in turn (the workgroup owns both rows, so no
// other workgroup writes them).  The mean removal x - mean(x) adds
// -(1/nt) sum_t dE/dx[t] to every sample; that sum is
// kappa sum_l Re sum_k g_{k,l} conj(What_k), taken from the bins where the
// window's DFT is not zero before the blocks, so every row starts at that
// constant and the blocks accumulate onto it.
template <typename TC, typename TOUT, bool PP, int MAXU, int MAXI = (2 * MAXU + 2) / 3>
__global__ __launch_bounds__(GEN_THREADS) void general_adjoint_kernel(
    const cpx_t<TC>* __restrict__ gqh, TOUT* __restrict__ g_q, const double* __restrict__ window,
    const cpx_t<TC>* __restrict__ tw, const double2* __restrict__ what, int64_t M, int64_t nt,
    int N, int step, int L, double kappa, Radices rad, int64_t per_xcd,
    const cpx_t<TC>* __restrict__ oddw, GenAdjBins bins, GenAdjMean gm) {
  using C = cpx_t<TC>;
  extern __shared__ unsigned char smem[];
  C* const B0 = reinterpret_cast<C*>(smem);
  C* const B1 = PP ? B0 + N : B0;
  C* Wt = B0 + (PP ? 2 * N : N);
  const int64_t b = blockIdx.x;
  const int64_t pair = (b & 7) * per_xcd + (b >> 3);
  const int64_t P = (M + 1) / 2;
  if (pair >= P) return;                       // the same for every thread
  const int64_t m0 = 2 * pair;
  const bool two = m0 + 1 < M;
  const int tid = threadIdx.x;

  // sum_t dE/dx[t] of both rows, in FP64 (reduced in the first 16 KiB of LDS,
  // before the twiddles and the blocks take it)
  double sa = 0.0, sc = 0.0;
  const int nmb = gm.n >= 0 ? gm.n : bins.n;
  for (int it = tid; it < nmb * L; it += GEN_THREADS) {
    const int i = it / L, l = it - i * L;
    const int slot = gm.n >= 0 ? gm.slot[i] : i;
    double wr, wi;
    if (gm.n >= 0) {
      wr = gm.wr[i];
      wi = gm.wi[i];
    } else {
      const double2 wv = what[bins.k[i]];
      wr = wv.x;
      wi = wv.y;
    }
    const C* src = gqh + ((int64_t)slot * L + l) * M + m0;
    const C ga = src[0];
    sa += (double)ga.x * wr + (double)ga.y * wi;
    if (two) {
      const C gc = src[1];
      sc += (double)gc.x * wr + (double)gc.y * wi;
    }
  }
  double* red = reinterpret_cast<double*>(B0);   // before the first block uses B0
  red[tid] = sa;
  red[GEN_THREADS + tid] = sc;
  __syncthreads();
  for (int h = GEN_THREADS / 2; h > 0; h >>= 1) {
    if (tid < h) {
      red[tid] += red[tid + h];
      red[GEN_THREADS + tid] += red[GEN_THREADS + tid + h];
    }
    __syncthreads();
  }
  const double ca = -kappa * red[0] / (double)nt, cc = -kappa * red[GEN_THREADS] / (double)nt;
  __syncthreads();
  {
    int off = 0;
    for (int st = 0; st < rad.n; ++st) {
      const int r = rad.r[st];
      for (int t = tid; t < r; t += GEN_THREADS) Wt[off + t] = tw[(N / r) * t];
      off += r;
    }
  }
  TOUT* ra = g_q + m0 * nt;
  TOUT* rc = g_q + (two ? m0 + 1 : m0) * nt;
  for (int64_t t = tid; t < nt; t += GEN_THREADS) {
    ra[t] = (TOUT)ca;
    if (two) rc[t] = (TOUT)cc;
  }
  __syncthreads();

  const TC hk = (TC)(0.5 * kappa);
  for (int l = 0; l < L; ++l) {
    C* X = B0;
    C* Y = B1;
    // conj Z: zero, then the selected bins and their mirrors
    for (int n = tid; n < N; n += GEN_THREADS) X[n] = mk<TC>((TC)0, (TC)0);
    __syncthreads();
    for (int i = tid; i < bins.n; i += GEN_THREADS) {
      const int k = bins.k[i];
      const C* src = gqh + ((int64_t)i * L + l) * M + m0;
      const C ga = src[0];
      const C gc = two ? src[1] : mk<TC>((TC)0, (TC)0);
      if (k == 0 || 2 * k == N) {
        X[k] = mk<TC>((TC)2 * ga.x, (TC)-2 * gc.x);
      } else {
        X[k] = mk<TC>(ga.x - gc.y, -ga.y - gc.x);
        X[N - k] = mk<TC>(ga.x + gc.y, ga.y - gc.x);
      }
    }
    __syncthreads();
    const C* D = dft_stages<TC, PP, MAXU, MAXI>(X, Y, Wt, tw, oddw, rad, tid, N);
    // (1/2) conj D, times kappa w[n], added into the block's samples
    const int64_t o = (int64_t)l * step;
    for (int n = tid; n < N; n += GEN_THREADS) {
      const TC w = (TC)window[n] * hk;
      const C d = D[n];
      ra[o + n] = (TOUT)((TC)ra[o + n] + w * d.x);
      if (two) rc[o + n] = (TOUT)((TC)rc[o + n] - w * d.y);
    }
    // the next block reads these samples and rewrites the buffers
    __syncthreads();
  }
}

template <typename TC, typename TOUT, bool PP, int MAXU>
spod_status launch_adjoint_pp(const Plan& p, const void* g_qhat, void* g_q, const GenAdjBins& bins,
                              const GenAdjMean& gm, size_t lds, hipStream_t st) {
  using C = cpx_t<TC>;
  const void* fn = reinterpret_cast<const void*>(&general_adjoint_kernel<TC, TOUT, PP, MAXU>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
  const int64_t P = (p.M + 1) / 2;
  const int64_t per_xcd = (P + 7) / 8;
  const int64_t wgs = 8 * per_xcd;
  if (wgs > 0x7fffffffLL) return fail(SPOD_ERR_UNSUPPORTED, "general transform grid too large");
  const C* tw = static_cast<const C*>(sizeof(TC) == 8 ? (const void*)p.d_tw64 : (const void*)p.d_tw32);
  hipLaunchKernelGGL((general_adjoint_kernel<TC, TOUT, PP, MAXU>), dim3((unsigned)wgs),
                     dim3(GEN_THREADS), lds, st, static_cast<const C*>(g_qhat),
                     static_cast<TOUT*>(g_q), p.d_window, tw, p.d_what, (int64_t)p.M, (int64_t)p.nt,
                     (int)p.nfft, (int)p.step, (int)p.nblocks, p.kappa, p.radices, per_xcd,
                     static_cast<const C*>(sizeof(TC) == 8 ? (const void*)p.d_oddw64
                                                           : (const void*)p.d_oddw32),
                     bins, gm);
  e = hipGetLastError();
  return e == hipSuccess ? SPOD_OK : hip_fail(e, "general_adjoint_kernel");
}

template <typename TC, typename TOUT, int MAXU>
spod_status launch_adjoint_t(const Plan& p, const void* g_qhat, void* g_q, const GenAdjBins& bins,
                             const GenAdjMean& gm, hipStream_t st) {
  using C = cpx_t<TC>;
  int sum_r = 0;
  for (int i = 0; i < p.radices.n; ++i) sum_r += p.radices.r[i];
  constexpr size_t LDS_MAX = 160 * 1024;
  // at least 16 KiB: the FP64 reduction of the mean term comes first
  const size_t two_buf = std::max<size_t>(sizeof(C) * (2 * (size_t)p.nfft + (size_t)sum_r),
                                          2 * GEN_THREADS * sizeof(double));
  if (two_buf <= LDS_MAX)
    return launch_adjoint_pp<TC, TOUT, true, (sizeof(C) == 8 ? 10 : 5)>(p, g_qhat, g_q, bins, gm,
                                                                          two_buf, st);
  const size_t one_buf = std::max<size_t>(sizeof(C) * ((size_t)p.nfft + (size_t)sum_r),
                                          2 * GEN_THREADS * sizeof(double));
  if (one_buf > LDS_MAX)
    return fail(SPOD_ERR_UNSUPPORTED, "block and twiddles exceed the 160 KiB of LDS");
  return launch_adjoint_pp<TC, TOUT, false, MAXU>(p, g_qhat, g_q, bins, gm, one_buf, st);
}

// ---------------------------------------------------------------------------
// two-pass transform for blocks beyond one workgroup's LDS: N = A B
// ---------------------------------------------------------------------------
// A stage over G sequences of length n stored one after another in X (and
// Y): the butterflies of every sequence in one loop.  In an odd stage the
// work items are ordered by output-pair group g first, then by sequence and
// butterfly (padded to a multiple of 64 once per g, not per sequence, since
// a short sequence has few butterflies), so g stays wavefront-uniform and
// its row of the stage's table is read through scalar loads as in odd_stage.
template <int KPT, typename TC>
__device__ __forceinline__ void odd_stage_batched(const cpx_t<TC>* __restrict__ X,
                                                  const cpx_t<TC>* __restrict__ T,
                                                  const cpx_t<TC>* __restrict__ tw,
                                                  cpx_t<TC>* __restrict__ Y, int tid, int n, int G,
                                                  int r, int s, int m, int wn) {
  const int NB = n / r;
  const int h = (r + 1) / 2, hm = h - 1, GG = (h + KPT - 1) / KPT;
  const int per = G * NB;                     // butterflies of all sequences
  const int perp = (per + 63) & ~63;
  const float inv_perp = 1.0f / (float)perp, inv_nb = 1.0f / (float)NB, inv_s = 1.0f / (float)s;
  for (int it = tid; it < GG * perp; it += GEN_THREADS) {
    const DivMod a = divmod(it, perp, inv_perp);
    const int g = __builtin_amdgcn_readfirstlane(a.q);
    if (a.r < per) {
      const DivMod b = divmod(a.r, NB, inv_nb);      // (sequence, butterfly)
      odd_uniform<KPT, TC>(X + (size_t)b.q * n, T + (size_t)g * hm * KPT, tw, Y + (size_t)b.q * n,
                           b.r, g, GG, r, s, m, wn, inv_s);
    }
  }
}

template <typename TC>
__device__ __forceinline__ void stage_batched(const cpx_t<TC>* __restrict__ X, cpx_t<TC>* __restrict__ Y,
                                              const cpx_t<TC>* __restrict__ tw,
                                              const cpx_t<TC>* __restrict__ oddw, const Radices& rad,
                                              int st, int tid, int n, int G, int r, int s, int m, int wn) {
  if (r % 2 == 1) {
    const cpx_t<TC>* T = oddw + rad.toff[st];
    switch (rad.kpt[st]) {
      case 1: odd_stage_batched<1, TC>(X, T, tw, Y, tid, n, G, r, s, m, wn); break;
      case 2: odd_stage_batched<2, TC>(X, T, tw, Y, tid, n, G, r, s, m, wn); break;
      case 3: odd_stage_batched<3, TC>(X, T, tw, Y, tid, n, G, r, s, m, wn); break;
      case 4: odd_stage_batched<4, TC>(X, T, tw, Y, tid, n, G, r, s, m, wn); break;
      case 5: odd_stage_batched<5, TC>(X, T, tw, Y, tid, n, G, r, s, m, wn); break;
      default: odd_stage_batched<6, TC>(X, T, tw, Y, tid, n, G, r, s, m, wn); break;
    }
  } else {
    // the factorisation gives even radices 8, 4 and 2 only
    const int NB = n / r;
    const float inv_nb = 1.0f / (float)NB, inv_s = 1.0f / (float)s;
    for (int it = tid; it < G * NB; it += GEN_THREADS) {
      const DivMod a = divmod(it, NB, inv_nb);
      const cpx_t<TC>* x = X + (size_t)a.q * n;
      cpx_t<TC>* y = Y + (size_t)a.q * n;
      if (r == 8) even_butterfly<8, TC>(x, tw, y, a.r, s, m, wn, n, inv_s);
      else if (r == 4) even_butterfly<4, TC>(x, tw, y, a.r, s, m, wn, n, inv_s);
      else even_butterfly<2, TC>(x, tw, y, a.r, s, m, wn, n, inv_s);
    }
  }
}

// G transforms of length n (tw = W_n^t), ping-pong between X and Y; returns
// the buffer with the results.  The caller has synchronised after writing X.
template <typename TC>
__device__ __forceinline__ cpx_t<TC>* dft_batched(cpx_t<TC>* X, cpx_t<TC>* Y,
                                                  const cpx_t<TC>* __restrict__ tw,
                                                  const cpx_t<TC>* __restrict__ oddw,
                                                  const Radices& rad, int tid, int n, int G) {
  int nn = n, s = 1;
  for (int st = 0; st < rad.n; ++st) {
    const int r = rad.r[st];
    const int m = nn / r;
    stage_batched<TC>(X, Y, tw, oddw, rad, st, tid, n, G, r, s, m, n / nn);
    __syncthreads();
    cpx_t<TC>* tmp = X;
    X = Y;
    Y = tmp;
    nn = m;
    s *= r;
  }
  return X;
}

// Loads per thread issued together when a batch is brought into LDS.
constexpr int LONG_U = 4;

// One workgroup per CU, taking (tile of up to P pairs of DOFs, block) items in
// turn.  With n = B j + c (j < A, c < B) and k = k1 + A k2:
//   pass 1: for every pair p and column c, Y_p[k1][c] = W_N^{c k1}
//           sum_j x_p[B j + c] W_A^{j k1} (GA sequences of length A per LDS
//           batch; Y in this workgroup's workspace slot, [P][A][B]);
//   pass 2: for the rows k1, X_p[k1 + A k2] = sum_c Y_p[k1][c] W_B^{c k2}, the
//           rows k1 and (A - k1) mod A of every pair side by side (NU of
//           these units per batch), so that Z_k and Z_{N-k} of the
//           two-for-one split are both in LDS, and the P pairs' values of one
//           frequency row are stored by neighbouring lanes: P * 16 bytes
//           contiguous (a whole 128-byte line at P = 8) instead of 16.
// The two rows of a pair are packed as a + i c; the window carries kappa.
template <typename TC, typename TIN>
__global__ __launch_bounds__(GEN_THREADS) void blocks_dft_long_kernel(
    const TIN* __restrict__ q, const double* __restrict__ mean, const double* __restrict__ window,
    const cpx_t<TC>* __restrict__ tw_n, const cpx_t<TC>* __restrict__ tw_a,
    const cpx_t<TC>* __restrict__ oddw_a, Radices rad_a, const cpx_t<TC>* __restrict__ tw_b,
    const cpx_t<TC>* __restrict__ oddw_b, Radices rad_b, int A, int B, int GA, int NU, int P,
    int SB, cpx_t<TC>* __restrict__ scratch, cpx_t<TC>* __restrict__ qhat, int64_t M, int64_t nt,
    int step, int L, int K, double kappa) {
  using C = cpx_t<TC>;
  extern __shared__ unsigned char smem[];
  const int N = A * B;
  const int cap = max(GA * A, 2 * NU * P * B);
  C* const B0 = reinterpret_cast<C*>(smem);
  C* const B1 = B0 + cap;
  // W_N^t = hi[t / SB] lo[t % SB] (SB about sqrt N): the pass-1 twiddles from
  // LDS instead of a gather from the N-entry table
  C* const Thi = B1 + cap;
  C* const Tlo = Thi + (N + SB - 1) / SB;
  for (int a = (int)threadIdx.x; a * SB < N; a += GEN_THREADS) Thi[a] = tw_n[a * SB];
  for (int b = (int)threadIdx.x; b < SB; b += GEN_THREADS) Tlo[b] = tw_n[b];
  const float inv_sb = 1.0f / (float)SB;
  // the stages' W_A^t and W_B^t tables, also in LDS
  C* const Ta = Tlo + SB;
  C* const Tb = Ta + A;
  for (int t = (int)threadIdx.x; t < A; t += GEN_THREADS) Ta[t] = tw_a[t];
  for (int t = (int)threadIdx.x; t < B; t += GEN_THREADS) Tb[t] = tw_b[t];
  C* const Yg = scratch + (size_t)blockIdx.x * P * N;       // [P][A][B]
  const int64_t npair = (M + 1) / 2;
  const int64_t ntile = (npair + P - 1) / P;
  const int tid = threadIdx.x;
  const TC h = (TC)0.5;
  const bool aligned = (M % 2 == 0);
  // quotients by the batch shapes through float reciprocals (every dividend
  // here is below 2^24: a batch holds at most 160 KiB of LDS)
  const float inv_b = 1.0f / (float)B;
  for (int64_t item = blockIdx.x; item < ntile * L; item += gridDim.x) {
    const int64_t tile = item / L;
    const int l = (int)(item - tile * L);
    const int64_t pair0 = tile * P;
    const int np = (int)min((int64_t)P, npair - pair0);
    const float inv_np = 1.0f / (float)np;

    // pass 1: sequences s = p B + c of length A, GA per batch
    for (int s0 = 0; s0 < np * B; s0 += GA) {
      const int gs = min(GA, np * B - s0);
      const float inv_gs = 1.0f / (float)gs;
      // LONG_U loads per thread in flight, then their LDS writes
      for (int i0 = tid; i0 < gs * A; i0 += LONG_U * GEN_THREADS) {
        TIN va[LONG_U], vc[LONG_U];
        double vw[LONG_U], mu[LONG_U], mc[LONG_U];
        bool tw2[LONG_U];
        int dst[LONG_U];
#pragma unroll
        for (int u = 0; u < LONG_U; ++u) {
          const int idx = i0 + u * GEN_THREADS;
          if (idx < gs * A) {
            const DivMod jg = divmod(idx, gs, inv_gs);     // g fastest: consecutive samples
            const int j = jg.q, g = jg.r;
            const DivMod pc = divmod(s0 + g, B, inv_b);
            const int pp = pc.q, c = pc.r;
            const int64_t m0 = 2 * (pair0 + pp);
            const bool two = m0 + 1 < M;
            const int64_t n = (int64_t)l * step + B * j + c;
            va[u] = q[m0 * nt + n];
            vc[u] = q[(two ? m0 + 1 : m0) * nt + n];
            vw[u] = window[B * j + c];
            mu[u] = mean[m0];
            mc[u] = two ? mean[m0 + 1] : 0.0;
            tw2[u] = two;
            dst[u] = g * A + j;
          }
        }
#pragma unroll
        for (int u = 0; u < LONG_U; ++u) {
          const int idx = i0 + u * GEN_THREADS;
          if (idx < gs * A) {
            const double w = vw[u] * kappa;
            B0[dst[u]] = mk<TC>((TC)(((double)va[u] - mu[u]) * w),
                                (TC)(tw2[u] ? ((double)vc[u] - mc[u]) * w : 0.0));
          }
        }
      }
      __syncthreads();
      const C* R = dft_batched<TC>(B0, B1, Ta, oddw_a, rad_a, tid, A, gs);
      for (int idx = tid; idx < gs * A; idx += GEN_THREADS) {
        const DivMod kg = divmod(idx, gs, inv_gs);
        const int k1 = kg.q, g = kg.r;
        const DivMod pc = divmod(s0 + g, B, inv_b);
        const int pp = pc.q, c = pc.r;
        const C v = R[g * A + k1];
        const DivMod tt = divmod(c * k1, SB, inv_sb);         // c k1 < N
        const C th = Thi[tt.q], tl = Tlo[tt.r];
        const C t = mk<TC>(th.x * tl.x - th.y * tl.y, th.x * tl.y + th.y * tl.x);
        Yg[(size_t)pp * N + (size_t)k1 * B + c] = mk<TC>(v.x * t.x - v.y * t.y, v.x * t.y + v.y * t.x);
      }
      // Y written (global, this workgroup only) and the LDS free again
      __syncthreads();
    }

    // pass 2: units u = 0 .. A/2, rows u and (A - u) mod A; sequence
    // (slot, pair) = slot np + p, slot 2i the row u of unit u0 + i, slot 2i + 1
    // its partner
    const int U = A / 2 + 1;
    for (int u0 = 0; u0 < U; u0 += NU) {
      const int nu = min(NU, U - u0), nseq = 2 * nu * np;
      for (int i0 = tid; i0 < nseq * B; i0 += LONG_U * GEN_THREADS) {
        C vy[LONG_U];
#pragma unroll
        for (int v = 0; v < LONG_U; ++v) {
          const int idx = i0 + v * GEN_THREADS;
          if (idx < nseq * B) {
            const DivMod sc = divmod(idx, B, inv_b);
            const int sq = sc.q, c = sc.r;
            const DivMod sp = divmod(sq, np, inv_np);
            const int slot = sp.q, pp = sp.r;
            const int u = u0 + (slot >> 1);
            const int row = ((slot & 1) && u > 0) ? A - u : u;    // (A - u) mod A
            vy[v] = Yg[(size_t)pp * N + (size_t)row * B + c];
          }
        }
#pragma unroll
        for (int v = 0; v < LONG_U; ++v) {
          const int idx = i0 + v * GEN_THREADS;
          if (idx < nseq * B) B0[idx] = vy[v];
        }
      }
      __syncthreads();
      const C* R = dft_batched<TC>(B0, B1, Tb, oddw_b, rad_b, tid, B, nseq);
      // split and store: pairs fastest, so neighbouring lanes write one
      // frequency row's consecutive DOFs
      for (int idx = tid; idx < 2 * nu * B * np; idx += GEN_THREADS) {
        const DivMod rp = divmod(idx, np, inv_np);
        const int pp = rp.r, rest = rp.q;
        const DivMod sk = divmod(rest, B, inv_b);
        const int k2 = sk.r, slot = sk.q;
        const int u = u0 + (slot >> 1);
        const bool second = slot & 1;
        if (second && (u == 0 || 2 * u == A)) continue;     // the same row as slot 2i
        const int k1 = second ? A - u : u;
        const int64_t k = (int64_t)k1 + (int64_t)A * k2;
        if (k >= K) continue;
        // Z_{N-k}: row (A - k1) mod A = the other slot of this unit (the same
        // slot for u = 0 and u = A/2), column (B - k2) mod B for k1 = 0, else
        // B - 1 - k2
        const int pslot = (u == 0 || 2 * u == A) ? slot : (slot ^ 1);
        const int pk2 = (k1 == 0) ? (k2 == 0 ? 0 : B - k2) : B - 1 - k2;
        const C z = R[(slot * np + pp) * B + k2], zc = R[(pslot * np + pp) * B + pk2];
        const C a = mk<TC>(h * (z.x + zc.x), h * (z.y - zc.y));
        const C cc = mk<TC>(h * (z.y + zc.y), h * (zc.x - z.x));
        const int64_t m0 = 2 * (pair0 + pp);
        const bool two = m0 + 1 < M;
        C* dst = qhat + (k * L + l) * M + m0;
        if constexpr (sizeof(TC) == 4) {
          if (two && aligned) {
            *reinterpret_cast<float4*>(dst) = make_float4(a.x, a.y, cc.x, cc.y);
            continue;
          }
        }
        dst[0] = a;
        if (two) dst[1] = cc;
      }
      __syncthreads();
    }
  }
}

// Workgroups per CU of the two-pass transform (measured with one pair per
// item: one with all the LDS, 184 ms on the ten-year workload, against 212
// ms for two with half).
constexpr int LONG_WG_PER_CU = 1;

// Launch shape of the two-pass transform: P pairs per item (8, fewer when
// the pass-2 batch or the scratch, at most 2 GiB, does not allow it), GA
// sequences per pass-1 batch, NU units per pass-2 batch.
struct LongShape {
  int P = 0, GA = 0, NU = 0, SB = 0;
  size_t lds = 0, scratch = 0;
};

LongShape long_shape(const Plan& p) {
  LongShape sh;
  const size_t csz = is_complex128(p) ? 16 : 8;
  // after the two buffers: the split twiddle table W_N^{SB a}, W_N^b (SB =
  // ceil(sqrt N)) and the stages' W_A^t, W_B^t
  int sb = 1;
  while ((int64_t)sb * sb < p.nfft) ++sb;
  const int64_t ntab = (p.nfft + sb - 1) / sb + sb + p.long_a + p.long_b;
  const int64_t cap =
      (int64_t)(160 * 1024 / LONG_WG_PER_CU - ntab * (int64_t)csz) / 2 / (int64_t)csz;   // per buffer
  const int A = p.long_a, B = p.long_b;
  const int64_t grid = (int64_t)p.long_grid * LONG_WG_PER_CU;
  int P = (int)std::min<int64_t>(8, cap / B / 2);
  while (P > 1 && grid * P * p.nfft * (int64_t)csz > (int64_t(2) << 30)) --P;
  if (P < 1 || cap / A < 1) return sh;
  sh.P = P;
  sh.GA = (int)std::min<int64_t>((int64_t)P * B, cap / A);
  // an odd stage pads the butterflies of a batch to whole wavefronts: a batch
  // of GA sequences with GA (A / r) a multiple of 64 for every odd radix r of
  // A idles none of its lanes (A = 292 = 4 73: 32 sequences of 4 butterflies
  // instead of 35, whose 140 fill 192 lanes)
  int align = 1;
  for (int i = 0; i < p.rad_a.n; ++i) {
    const int r = p.rad_a.r[i];
    if (r % 2 == 0) continue;
    align = std::lcm(align, 64 / std::gcd(64, A / r));
  }
  if (align <= sh.GA) sh.GA -= sh.GA % align;
  sh.NU = (int)std::max<int64_t>(1, cap / B / (2 * P));
  sh.SB = sb;
  sh.lds = csz * (2 * (size_t)std::max<int64_t>((int64_t)sh.GA * A, 2LL * sh.NU * P * B) + (size_t)ntab);
  sh.scratch = csz * (size_t)grid * (size_t)P * (size_t)p.nfft;
  return sh;
}

template <typename TC, typename TIN>
spod_status launch_long_t(const Plan& p, const TIN* q, const double* mean, void* qhat, void* scratch,
                          hipStream_t st) {
  using C = cpx_t<TC>;
  const LongShape sh = long_shape(p);
  if (sh.P < 1) return fail(SPOD_ERR_UNSUPPORTED, "two-pass transform: a factor does not fit the LDS");
  const void* fn = reinterpret_cast<const void*>(&blocks_dft_long_kernel<TC, TIN>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds);
  if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
  const bool c8 = sizeof(TC) == 8;
  hipLaunchKernelGGL((blocks_dft_long_kernel<TC, TIN>), dim3((unsigned)(p.long_grid * LONG_WG_PER_CU)),
                     dim3(GEN_THREADS), sh.lds, st, q, mean, p.d_window,
                     static_cast<const C*>(c8 ? (const void*)p.d_tw64 : (const void*)p.d_tw32),
                     static_cast<const C*>(c8 ? (const void*)p.d_tw_a64 : (const void*)p.d_tw_a32),
                     static_cast<const C*>(c8 ? (const void*)p.d_oddw_a64 : (const void*)p.d_oddw_a32),
                     p.rad_a,
                     static_cast<const C*>(c8 ? (const void*)p.d_tw_b64 : (const void*)p.d_tw_b32),
                     static_cast<const C*>(c8 ? (const void*)p.d_oddw_b64 : (const void*)p.d_oddw_b32),
                     p.rad_b, p.long_a, p.long_b, sh.GA, sh.NU, sh.P, sh.SB, static_cast<C*>(scratch),
                     static_cast<C*>(qhat), (int64_t)p.M, (int64_t)p.nt, (int)p.step, (int)p.nblocks,
                     (int)p.nfreq, p.kappa);
  e = hipGetLastError();
  return e == hipSuccess ? SPOD_OK : hip_fail(e, "blocks_dft_long_kernel");
}

}  // namespace

int general_odd_entries(int r, int kpt) {
  const int hm = (r - 1) / 2, G = (hm + kpt) / kpt;
  return G * hm * kpt;
}

int general_odd_kpt(int r, int nb) {
  // instructions of one work item: per term a shared load, sum and difference
  // (about 6) plus 4 multiply-adds per pair; per pair about 30 to finish and
  // store.  A stage costs the work items of the busiest SIMD (the wavefronts
  // of a workgroup spread over its 4 SIMDs).
  const int hm = (r - 1) / 2, h = hm + 1;
  const int64_t nbp = (nb + 63) / 64 * 64;
  int best = 1;
  int64_t best_cost = -1;
  for (int kpt = 1; kpt <= GENERAL_MAX_KPT; ++kpt) {
    const int64_t G = (h + kpt - 1) / kpt;
    const int64_t waves = nbp / 64 * G;
    const int64_t cost = (waves + 3) / 4 * ((int64_t)hm * (6 + 4 * kpt) + 30 * kpt);
    if (best_cost < 0 || cost < best_cost) {
      best = kpt;
      best_cost = cost;
    }
  }
  return best;
}

spod_status launch_blocks_dft_general(const Plan& p, const void* q, spod_dtype dtype,
                                      const double* mean, void* qhat, hipStream_t st) {
  const bool c128 = is_complex128(p);
  if (p.nfft > (c128 ? SPOD_GENERAL_MAX_NFFT / 2 : SPOD_GENERAL_MAX_NFFT))
    return fail(SPOD_ERR_UNSUPPORTED, c128 ? "nfft above 10240 with complex128 blocks"
                                           : "nfft above 20480");
  if (p.radices.n <= 0) return fail(SPOD_ERR_UNSUPPORTED, "nfft has no radix factorisation");
  for (int i = 0; i < p.radices.n; ++i)
    if (p.radices.r[i] > 1024)
      return fail(SPOD_ERR_UNSUPPORTED, "nfft has a prime factor above 1024");
  constexpr int UF = (SPOD_GENERAL_MAX_NFFT + GEN_THREADS - 1) / GEN_THREADS;
  constexpr int UD = (SPOD_GENERAL_MAX_NFFT / 2 + GEN_THREADS - 1) / GEN_THREADS;
  if (dtype == SPOD_F32)
    return c128 ? launch_general_t<double, float, UD>(p, static_cast<const float*>(q), mean, qhat, st)
                : launch_general_t<float, float, UF>(p, static_cast<const float*>(q), mean, qhat, st);
  return c128 ? launch_general_t<double, double, UD>(p, static_cast<const double*>(q), mean, qhat, st)
              : launch_general_t<float, double, UF>(p, static_cast<const double*>(q), mean, qhat, st);
}

}  // namespace spod

namespace spod {

spod_status launch_general_adjoint(const Plan& p, const void* g_qhat, spod_dtype dtype, void* g_q,
                                   const GenAdjBins& bins, const GenAdjMean& mean, hipStream_t st) {
  const bool c128 = is_complex128(p);
  if (p.nfft > (c128 ? SPOD_GENERAL_MAX_NFFT / 2 : SPOD_GENERAL_MAX_NFFT))
    return fail(SPOD_ERR_UNSUPPORTED, "nfft too large for the general transform");
  if (p.radices.n <= 0) return fail(SPOD_ERR_UNSUPPORTED, "nfft has no radix factorisation");
  constexpr int UF = (SPOD_GENERAL_MAX_NFFT + GEN_THREADS - 1) / GEN_THREADS;
  constexpr int UD = (SPOD_GENERAL_MAX_NFFT / 2 + GEN_THREADS - 1) / GEN_THREADS;
  if (dtype == SPOD_F32)
    return c128 ? launch_adjoint_t<double, float, UD>(p, g_qhat, g_q, bins, mean, st)
                : launch_adjoint_t<float, float, UF>(p, g_qhat, g_q, bins, mean, st);
  return c128 ? launch_adjoint_t<double, double, UD>(p, g_qhat, g_q, bins, mean, st)
              : launch_adjoint_t<float, double, UF>(p, g_qhat, g_q, bins, mean, st);
}

}  // namespace spod

namespace spod {

// whether a plan's transform takes the two-pass path (precision dependent)
static bool use_long(const Plan& p) {
  if (!p.long_dft || p.general_passes == 1) return false;
  return p.general_passes == 2 ||
         p.nfft > (is_complex128(p) ? SPOD_GENERAL_MAX_NFFT / 2 : SPOD_GENERAL_MAX_NFFT);
}

size_t long_scratch_bytes(const Plan& p) {
  if (!use_long(p)) return 0;
  return long_shape(p).scratch;
}

spod_status launch_blocks_dft_long(const Plan& p, const void* q, spod_dtype dtype,
                                   const double* mean, void* qhat, void* scratch, hipStream_t st) {
  const bool c128 = is_complex128(p);
  if (dtype == SPOD_F32)
    return c128 ? launch_long_t<double, float>(p, static_cast<const float*>(q), mean, qhat, scratch, st)
                : launch_long_t<float, float>(p, static_cast<const float*>(q), mean, qhat, scratch, st);
  return c128 ? launch_long_t<double, double>(p, static_cast<const double*>(q), mean, qhat, scratch, st)
              : launch_long_t<float, double>(p, static_cast<const double*>(q), mean, qhat, scratch, st);
}

}  // namespace spod
