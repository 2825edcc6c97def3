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
// special case), the W_r^t of every stage copied from the plan's table W_N^t
// into LDS (at most the sum of the radices, 89 values for 8760).  For an odd
// radix one work item yields the outputs k and r - k from (r - 1) / 2 terms
// of the symmetric sums, a quarter of the multiplications.  A thread
// computes its outputs of a stage into registers, the workgroup synchronises,
// and the outputs overwrite the inputs in LDS.  The mean comes from the FP64
// mean pass.  A workgroup takes the blocks of its pair in turn, loading the
// next block while it transforms the current one.  Consecutive workgroups of
// one XCD take consecutive pairs, so their 16-byte stores of neighbouring
// degrees of freedom meet in that XCD's L2.
#include <hip/hip_runtime.h>

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
template <typename TC>
__device__ __forceinline__ cpx_t<TC> even_output(const cpx_t<TC>* __restrict__ X,
                                                 const cpx_t<TC>* __restrict__ Wr,
                                                 const cpx_t<TC>* __restrict__ tw, int o, int r,
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
  const C t2 = tw[(int)(((int64_t)wn * pp * k) % N)];
  return mk<TC>(sr * t2.x - si * t2.y, sr * t2.y + si * t2.x);
}

// Work item it of an odd-radix stage: with a_j = x_j + x_{r-j}, b_j =
// x_j - x_{r-j} and W_r^{jk} = c - i s, the outputs k and r - k share the sums
// A = sum_{j <= (r-1)/2} a_j c and B = sum b_j s:  y_k = x_0 + A - i B,
// y_{r-k} = x_0 + A + i B (then W_n^{p k}, W_n^{p(r-k)}).  kk = it / NB in
// [0, (r-1)/2]; consecutive items are consecutive butterflies.
template <typename TC>
__device__ __forceinline__ void odd_pair(const cpx_t<TC>* __restrict__ X,
                                         const cpx_t<TC>* __restrict__ Wr,
                                         const cpx_t<TC>* __restrict__ tw, int it, int NB, int r,
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
  const C t0 = tw[(int)(((int64_t)wn * pp * kk) % N)];
  const C t1 = tw[(int)(((int64_t)wn * pp * (r - kk)) % N)];
  y0 = mk<TC>(ykr * t0.x - yki * t0.y, ykr * t0.y + yki * t0.x);
  y1 = mk<TC>(yrr * t1.x - yri * t1.y, yrr * t1.y + yri * t1.x);
  o0 = qq + s * (r * pp + kk);
  o1 = kk > 0 ? qq + s * (r * pp + r - kk) : -1;
}

// One butterfly of a radix-2, 4 or 8 stage: the RS inputs x[q + s(p + j m)]
// through the in-register DFT, output k times W_n^{p k}, stored at
// y[q + s(RS p + k)].
template <int RS, typename TC>
__device__ __forceinline__ void even_butterfly(const cpx_t<TC>* __restrict__ X,
                                               const cpx_t<TC>* __restrict__ tw,
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
  const int step = (int)(((int64_t)wn * pp) % N);   // W_n^{p k} = W_N^{k step}
  int t = 0;
  const int out = qq + s * RS * pp;
  Y[out] = x[0];
#pragma unroll
  for (int k = 1; k < RS; ++k) {
    t += step;
    if (t >= N) t -= N;
    const C w = tw[t];
    Y[out + s * k] = mk<TC>(x[k].x * w.x - x[k].y * w.y, x[k].x * w.y + x[k].y * w.x);
  }
}

// Two work items of an odd-radix stage in one pass: the outputs k1 = g and
// k2 = g + hh (when k2 < h = (r + 1) / 2), with their partners r - k, for
// butterfly bf.  The loads of x_j and x_{r-j} and their sum and difference are
// shared by both; writes every output it owns straight to Y.
template <typename TC>
__device__ __forceinline__ void odd_two(const cpx_t<TC>* __restrict__ X, const cpx_t<TC>* __restrict__ Wr,
                                        const cpx_t<TC>* __restrict__ tw, cpx_t<TC>* __restrict__ Y,
                                        int it, int NB, int hh, int r, int s, int m, int wn, int N,
                                        float inv_nb, float inv_s) {
  using C = cpx_t<TC>;
  const int h = (r + 1) / 2;
  const DivMod a = divmod(it, NB, inv_nb);    // it = bf + NB * g
  const int g = a.q, bf = a.r;
  const int k1 = g, k2 = g + hh;
  const DivMod b = divmod(bf, s, inv_s);      // bf = qq + s * pp
  const int qq = b.r, pp = b.q;
  const int base = qq + s * pp, js = s * m;
  const C x0 = X[base];
  TC a1r = 0, a1i = 0, b1r = 0, b1i = 0, a2r = 0, a2i = 0, b2r = 0, b2i = 0;
  int t1 = 0, t2 = 0;
  const C* pa = X + base + js;
  const C* pb = X + base + (r - 1) * js;
  for (int j = 1; 2 * j < r; ++j, pa += js, pb -= js) {
    t1 += k1;
    if (t1 >= r) t1 -= r;
    t2 += k2;
    if (t2 >= r) t2 -= r;
    const C xa = *pa, xb = *pb;
    const TC sr = xa.x + xb.x, si = xa.y + xb.y, dr = xa.x - xb.x, di = xa.y - xb.y;
    const C w1 = Wr[t1], w2 = Wr[t2];
    a1r += sr * w1.x;
    a1i += si * w1.x;
    b1r -= dr * w1.y;
    b1i -= di * w1.y;
    a2r += sr * w2.x;
    a2i += si * w2.x;
    b2r -= dr * w2.y;
    b2i -= di * w2.y;
  }
  auto put = [&](int k, TC ar, TC ai, TC br, TC bi) {
    // y_k = x0 + A - iB, y_{r-k} = x0 + A + iB, then W_n^{p k}, W_n^{p (r-k)}
    const TC ykr = x0.x + ar + bi, yki = x0.y + ai - br;
    const C t0 = tw[(int)(((int64_t)wn * pp * k) % N)];
    Y[qq + s * (r * pp + k)] = mk<TC>(ykr * t0.x - yki * t0.y, ykr * t0.y + yki * t0.x);
    if (k > 0) {
      const TC yrr = x0.x + ar - bi, yri = x0.y + ai + br;
      const C t1w = tw[(int)(((int64_t)wn * pp * (r - k)) % N)];
      Y[qq + s * (r * pp + r - k)] = mk<TC>(yrr * t1w.x - yri * t1w.y, yrr * t1w.y + yri * t1w.x);
    }
  };
  put(k1, a1r, a1i, b1r, b1i);
  if (k2 < h) put(k2, a2r, a2i, b2r, b2i);
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
    int step, int L, int K, TC kappa, Radices rad, int64_t per_xcd) {
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

  {
    int off = 0;
    for (int st = 0; st < rad.n; ++st) {
      const int r = rad.r[st];
      for (int t = tid; t < r; t += GEN_THREADS) Wt[off + t] = tw[(N / r) * t];
      off += r;
    }
  }
  const double mu0 = mean[m0], mu1 = two ? mean[m0 + 1] : 0.0;
  const TIN* r0 = q + m0 * nt;
  const TIN* r1 = q + (two ? m0 + 1 : m0) * nt;
  TIN pa[MAXR], pb[MAXR];                      // the next block's samples (PP)
  if constexpr (PP) {
#pragma unroll
    for (int u = 0; u < MAXR; ++u) {
      const int n = tid + u * GEN_THREADS;
      pa[u] = n < N ? r0[n] : (TIN)0;
      pb[u] = n < N ? r1[n] : (TIN)0;
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
          const double w = window[n];
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

    int n = N, s = 1, off = 0;
    for (int st = 0; st < rad.n; ++st) {
      const int r = rad.r[st];
      const int m = n / r;
      const int wn = N / n;          // W_n = W_N^(N/n)
      const C* Wr = Wt + off;
      if constexpr (PP) {
        if (r % 2 == 1) {
          const int NB = N / r, hh = ((r + 1) / 2 + 1) / 2;
          const float inv_nb = 1.0f / (float)NB, inv_s = 1.0f / (float)s;
          for (int it = tid; it < NB * hh; it += GEN_THREADS)
            odd_two<TC>(X, Wr, tw, Y, it, NB, hh, r, s, m, wn, N, inv_nb, inv_s);
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
                     (int)p.nfreq, (TC)p.kappa, p.radices, per_xcd);
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
  const size_t two_buf = sizeof(C) * (2 * (size_t)p.nfft + (size_t)sum_r);
  // two buffers: complex64 N <= ~10200, complex128 <= ~5100, so at most
  // ceil(10240 / 1024) samples per thread and row to prefetch
  if (two_buf <= LDS_MAX)
    return launch_general_pp<TC, TIN, true, (sizeof(C) == 8 ? 10 : 5)>(p, q, mean, qhat, two_buf, st);
  const size_t one_buf = sizeof(C) * ((size_t)p.nfft + (size_t)sum_r);
  if (one_buf > LDS_MAX)
    return fail(SPOD_ERR_UNSUPPORTED, "block and twiddles exceed the 160 KiB of LDS");
  return launch_general_pp<TC, TIN, false, MAXU>(p, q, mean, qhat, one_buf, st);
}

}  // namespace

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
