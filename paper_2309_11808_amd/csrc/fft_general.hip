// Steps 1-2 of SPOD for any block length N_f (eq. (blocks), (blocks-ft),
// (blocks-k)): Welch blocks, window and one-sided DFT in time, where N_f is
// not a power of two or is above the register-resident transform's 1024 (the
// paper's hourly data use N_f = 8760 = 2^3 3 5 73).
//
// One workgroup of 1024 threads owns one pair of degrees of freedom and one
// block: the two real rows are packed as a + i c, transformed once, and split
// with the two-for-one identity.  The transform is a self-sorting mixed-radix
// one (decimation in frequency) held in LDS: for N = r_0 r_1 ... the stage of
// radix r with current length n and stride s maps
//   y[q + s (r p + k)] = W_n^{p k} sum_j x[q + s (p + j n / r)] W_r^{j k},
// every output a direct radix-r sum (so a prime factor such as 73 needs no
// special case), all twiddles taken from the plan's table W_N^t.  A thread
// computes its outputs of a stage into registers, the workgroup synchronises,
// and the outputs overwrite the inputs in LDS.  The mean comes from the FP64
// mean pass.  Consecutive workgroups of one XCD take consecutive pairs of the
// same block, so their 16-byte stores of neighbouring degrees of freedom
// meet in that XCD's L2.
#include <hip/hip_runtime.h>

#include <algorithm>

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

template <typename TC, typename TIN, int MAXU>
__global__ __launch_bounds__(GEN_THREADS) void blocks_dft_general_kernel(
    const TIN* __restrict__ q, const double* __restrict__ mean, const double* __restrict__ window,
    const cpx_t<TC>* __restrict__ tw, cpx_t<TC>* __restrict__ qhat, int64_t M, int64_t nt, int N,
    int step, int L, int K, TC kappa, Radices rad, int64_t per_xcd) {
  using C = cpx_t<TC>;
  extern __shared__ unsigned char smem[];
  C* T = reinterpret_cast<C*>(smem);
  const int64_t b = blockIdx.x;
  const int64_t x = b >> 3, xcd = b & 7;
  const int64_t l = x / per_xcd;
  const int64_t pair = xcd * per_xcd + x % per_xcd;
  const int64_t P = (M + 1) / 2;
  if (pair >= P || l >= L) return;             // the same for every thread
  const int64_t m0 = 2 * pair;
  const bool two = m0 + 1 < M;
  const int tid = threadIdx.x;

  // windowed, mean-free samples of both rows as one complex sequence
  {
    const double mu0 = mean[m0], mu1 = two ? mean[m0 + 1] : 0.0;
    const TIN* r0 = q + m0 * nt + l * step;
    const TIN* r1 = q + (two ? m0 + 1 : m0) * nt + l * step;
    for (int n = tid; n < N; n += GEN_THREADS) {
      const double w = window[n];
      const double a = ((double)r0[n] - mu0) * w;
      const double c = two ? ((double)r1[n] - mu1) * w : 0.0;
      T[n] = mk<TC>((TC)a, (TC)c);
    }
  }
  __syncthreads();

  int n = N, s = 1;
  for (int st = 0; st < rad.n; ++st) {
    const int r = rad.r[st];
    const int m = n / r;
    const int wr = N / r;          // W_r = W_N^(N/r)
    const int wn = N / n;          // W_n = W_N^(N/n)
    C y[MAXU];
#pragma unroll
    for (int u = 0; u < MAXU; ++u) {
      const int o = tid + u * GEN_THREADS;
      if (o < N) {
        const int qq = o % s, rest = o / s;
        const int k = rest % r, pp = rest / r;
        const int base = qq + s * pp, js = s * m;
        const int wstep = (int)(((int64_t)wr * k) % N);
        TC ar = 0, ai = 0;
        int wi = 0;
        for (int j = 0; j < r; ++j) {
          const C xv = T[base + j * js];
          const C wv = tw[wi];
          ar += xv.x * wv.x - xv.y * wv.y;
          ai += xv.x * wv.y + xv.y * wv.x;
          wi += wstep;
          if (wi >= N) wi -= N;
        }
        const C t2 = tw[(int)(((int64_t)wn * pp * k) % N)];
        y[u] = mk<TC>(ar * t2.x - ai * t2.y, ar * t2.y + ai * t2.x);
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MAXU; ++u) {
      const int o = tid + u * GEN_THREADS;
      if (o < N) T[o] = y[u];
    }
    __syncthreads();
    n = m;
    s *= r;
  }

  // two-for-one split: A = (Z_k + conj Z_{N-k}) / 2, C = (Z_k - conj Z_{N-k}) / 2i
  const TC h = (TC)0.5 * kappa;
  const bool vec = two && (M % 2 == 0);        // 16-byte aligned pair (m0 even)
  for (int k = tid; k < K; k += GEN_THREADS) {
    const C z = T[k], zc = T[k == 0 ? 0 : N - k];
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
}

template <typename TC, typename TIN, int MAXU>
spod_status launch_general_t(const Plan& p, const TIN* q, const double* mean, void* qhat,
                             hipStream_t st) {
  using C = cpx_t<TC>;
  const size_t lds = sizeof(C) * (size_t)p.nfft;
  const void* fn = reinterpret_cast<const void*>(&blocks_dft_general_kernel<TC, TIN, MAXU>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
  const int64_t P = (p.M + 1) / 2;
  const int64_t per_xcd = (P + 7) / 8;
  const int64_t wgs = 8 * per_xcd * p.nblocks;
  if (wgs > 0x7fffffffLL) return fail(SPOD_ERR_UNSUPPORTED, "general transform grid too large");
  const C* tw = static_cast<const C*>(sizeof(TC) == 8 ? (const void*)p.d_tw64 : (const void*)p.d_tw32);
  hipLaunchKernelGGL((blocks_dft_general_kernel<TC, TIN, MAXU>), dim3((unsigned)wgs),
                     dim3(GEN_THREADS), lds, st, q, mean, p.d_window, tw, static_cast<C*>(qhat),
                     (int64_t)p.M, (int64_t)p.nt, (int)p.nfft, (int)p.step, (int)p.nblocks,
                     (int)p.nfreq, (TC)p.kappa, p.radices, per_xcd);
  e = hipGetLastError();
  return e == hipSuccess ? SPOD_OK : hip_fail(e, "blocks_dft_general_kernel");
}

}  // namespace

spod_status launch_blocks_dft_general(const Plan& p, const void* q, spod_dtype dtype,
                                      const double* mean, void* qhat, hipStream_t st) {
  const bool c128 = is_complex128(p);
  if (p.nfft > (c128 ? SPOD_GENERAL_MAX_NFFT / 2 : SPOD_GENERAL_MAX_NFFT))
    return fail(SPOD_ERR_UNSUPPORTED, c128 ? "nfft above 10240 with complex128 blocks"
                                           : "nfft above 20480");
  if (p.radices.n <= 0) return fail(SPOD_ERR_UNSUPPORTED, "nfft has no radix factorisation");
  constexpr int UF = (SPOD_GENERAL_MAX_NFFT + GEN_THREADS - 1) / GEN_THREADS;
  constexpr int UD = (SPOD_GENERAL_MAX_NFFT / 2 + GEN_THREADS - 1) / GEN_THREADS;
  if (dtype == SPOD_F32)
    return c128 ? launch_general_t<double, float, UD>(p, static_cast<const float*>(q), mean, qhat, st)
                : launch_general_t<float, float, UF>(p, static_cast<const float*>(q), mean, qhat, st);
  return c128 ? launch_general_t<double, double, UD>(p, static_cast<const double*>(q), mean, qhat, st)
              : launch_general_t<float, double, UF>(p, static_cast<const double*>(q), mean, qhat, st);
}

}  // namespace spod
