// Steps 1-2 of SPOD (Sec. 2.3): long-time mean, Welch blocks (eq. (blocks)),
// windowed DFT of every block in time (eq. (blocks-ft)), stored per frequency
// (eq. (blocks-k)) as qhat[k][l][m].
//
// Work split (the paper's spatial decomposition of Sec. 3.1 mapped onto one
// GPU): a workgroup owns a tile of T consecutive degrees of freedom and a run
// of blocks, so every transform is workgroup-local and time is never split.
//
// Transform: two real rows a, b of a tile are packed into one complex sequence
// z = x_a + i x_b and transformed by a length-N_f Stockham autosort FFT
// (radix 8 in registers, exchanges through LDS).  Lane j of the P = N_f/8
// lanes of a transform holds elements j + r*P, r = 0..7.  The two spectra are
// separated with X_a[k] = (Z[k] + conj Z[N-k]) / 2 and
// X_b[k] = (Z[k] - conj Z[N-k]) / (2i) while the spectra are read back from
// LDS in [k][m] order, so every frequency row is written as one contiguous run
// of T complex values.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace spod {

// ---------------------------------------------------------------------------
// temporal mean, accumulated in FP64: one 64-lane wavefront per row
// ---------------------------------------------------------------------------
template <typename TIN>
__global__ __launch_bounds__(256) void mean_kernel(const TIN* __restrict__ q, double* __restrict__ mean,
                                                   int64_t M, int64_t nt) {
  const int lane = threadIdx.x & 63;
  const int64_t m = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (m >= M) return;
  const TIN* row = q + m * nt;
  double s = 0.0;
  for (int64_t t = lane; t < nt; t += 64) s += (double)row[t];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) mean[m] = s / (double)nt;
}

// ---------------------------------------------------------------------------
// in-register DFTs of size 2, 4 and 8 (natural order in and out)
// ---------------------------------------------------------------------------
template <typename C>
__device__ __forceinline__ void dft2(C* x) {
  C a = x[0], b = x[1];
  x[0] = cadd(a, b);
  x[1] = csub(a, b);
}

template <typename C>
__device__ __forceinline__ void dft4(C* x) {
  C c0 = cadd(x[0], x[2]), d0 = csub(x[0], x[2]);
  C c1 = cadd(x[1], x[3]), d1 = cmul_mi(csub(x[1], x[3]));
  x[0] = cadd(c0, c1);
  x[2] = csub(c0, c1);
  x[1] = cadd(d0, d1);
  x[3] = csub(d0, d1);
}

template <typename C>
__device__ __forceinline__ void dft8(C* x) {
  using T = decltype(x[0].x);
  const T h = (T)0.70710678118654752440084436210484903928;
  // decimation in frequency: a = x[q] + x[q+4], b = (x[q] - x[q+4]) w8^q
  C a[4], b[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    a[q] = cadd(x[q], x[q + 4]);
    b[q] = csub(x[q], x[q + 4]);
  }
  b[1] = C{h * (b[1].x + b[1].y), h * (b[1].y - b[1].x)};    // * (1 - i)/sqrt2
  b[2] = cmul_mi(b[2]);                                      // * -i
  b[3] = C{h * (b[3].y - b[3].x), -h * (b[3].x + b[3].y)};   // * (-1 - i)/sqrt2
  dft4(a);
  dft4(b);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    x[2 * k] = a[k];
    x[2 * k + 1] = b[k];
  }
}

template <int RS, typename C>
__device__ __forceinline__ void dft_r(C* x) {
  if constexpr (RS == 2) dft2(x);
  else if constexpr (RS == 4) dft4(x);
  else dft8(x);
}

// One Stockham stage of radix RS after NS points have been combined.  Lane j
// handles butterflies b = j + u*P (u < 8/RS) over elements b + q*(NF/RS).
template <int NF, int NS, int RS, typename C>
__device__ __forceinline__ void stockham_stage(C (&v)[8], C* buf, int j, const C* __restrict__ tw) {
  constexpr int P = NF / 8;
  constexpr int U = 8 / RS;
  constexpr bool LAST = (NS * RS == NF);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int b = j + u * P;
    const int kk = b % NS;
    C x[RS];
#pragma unroll
    for (int q = 0; q < RS; ++q) x[q] = v[q * U + u];
    if constexpr (NS > 1) {
#pragma unroll
      for (int q = 1; q < RS; ++q) x[q] = cmul(x[q], tw[q * kk * (NF / (NS * RS))]);
    }
    dft_r<RS>(x);
    if constexpr (LAST) {
#pragma unroll
      for (int q = 0; q < RS; ++q) v[q * U + u] = x[q];
    } else {
      const int base = (b / NS) * NS * RS + kk;
#pragma unroll
      for (int q = 0; q < RS; ++q) buf[base + q * NS] = x[q];
    }
  }
  if constexpr (!LAST) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = buf[j + r * P];
    __syncthreads();
  }
}

template <int NF, int NS, typename C>
__device__ __forceinline__ void stockham(C (&v)[8], C* buf, int j, const C* __restrict__ tw) {
  if constexpr (NS < NF) {
    constexpr int REM = NF / NS;
    constexpr int RS = REM >= 8 ? 8 : REM;
    stockham_stage<NF, NS, RS>(v, buf, j, tw);
    stockham<NF, NS * RS>(v, buf, j, tw);
  }
}

// ---------------------------------------------------------------------------
// windowed block transform
// ---------------------------------------------------------------------------
// SHIFT = hop / P when the hop between blocks is a whole number of lane
// strides (e.g. 4 for 50% overlap): the raw samples of elements SHIFT..7 of
// block l are elements 0..7-SHIFT of block l+1 and stay in registers.
// SHIFT = 8 reloads every block.
template <int NF, typename TC, typename TIN, int NPAIR, int SHIFT>
__global__ __launch_bounds__(NPAIR*(NF / 8)) void blocks_fft_kernel(
    const TIN* __restrict__ q, const double* __restrict__ mean, const double* __restrict__ window,
    const cpx_t<TC>* __restrict__ tw, cpx_t<TC>* __restrict__ qhat, int64_t M, int64_t nt,
    int step, int L, int bpw, TC kappa) {
  using C = cpx_t<TC>;
  constexpr int P = NF / 8;              // lanes per transform
  constexpr int T = 2 * NPAIR;           // degrees of freedom per tile
  constexpr int NTH = NPAIR * P;
  constexpr int LD = NF + 1;             // padded LDS row (bank spread for the [k][m] reads)
  constexpr int K = NF / 2 + 1;
  __shared__ C lds[NPAIR * LD];

  const int tid = threadIdx.x;
  const int f = tid / P;                 // transform (pair) index in the tile
  const int j = tid % P;                 // lane within the transform
  const int64_t m0 = (int64_t)blockIdx.x * T;
  const int64_t ma = m0 + 2 * f, mb = ma + 1;
  const bool va = ma < M, vb = mb < M;
  const double mua = va ? mean[ma] : 0.0, mub = vb ? mean[mb] : 0.0;
  const TIN* ra = q + (va ? ma : 0) * nt;
  const TIN* rb = q + (vb ? mb : 0) * nt;
  C* buf = lds + f * LD;

  TC w[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) w[r] = (TC)window[j + r * P];

  const int l0 = blockIdx.y * bpw;
  const int l1 = min(L, l0 + bpw);
  TIN xa[8], xb[8];
  for (int l = l0; l < l1; ++l) {
    const int64_t t0 = (int64_t)l * step;
    const bool first = (l == l0);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      if (!first && r + SHIFT < 8) {
        xa[r] = xa[r + SHIFT];
        xb[r] = xb[r + SHIFT];
      } else {
        const int64_t t = t0 + j + r * P;
        xa[r] = va ? ra[t] : (TIN)0;
        xb[r] = vb ? rb[t] : (TIN)0;
      }
    }

    C v[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const TC a = (TC)((double)xa[r] - mua);
      const TC b = (TC)((double)xb[r] - mub);
      v[r] = C{a * w[r], b * w[r]};
    }
    stockham<NF, 1>(v, buf, j, tw);
#pragma unroll
    for (int r = 0; r < 8; ++r) buf[j + r * P] = v[r];
    __syncthreads();

    // separate the two real spectra and write qhat[k][l][m0 .. m0+T)
    C* out = qhat + (int64_t)l * M;
    for (int idx = tid; idx < K * T; idx += NTH) {
      const int d = idx % T;
      const int k = idx / T;
      const C* row = lds + (d >> 1) * LD;
      const C A = row[k];
      const C Bc = row[(NF - k) & (NF - 1)];
      const C B = C{Bc.x, -Bc.y};
      C X;
      if ((d & 1) == 0) {
        X = cadd(A, B);
      } else {
        X = cmul_mi(csub(A, B));
      }
      const TC s = (TC)0.5 * kappa;
      const int64_t m = m0 + d;
      if (m < M) out[(int64_t)k * L * M + m] = C{X.x * s, X.y * s};
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
template <int NF, typename TC, typename TIN>
static spod_status launch_fft_nf(const Plan& p, const TIN* q, const double* mean, void* qhat,
                                 hipStream_t st) {
  using C = cpx_t<TC>;
  constexpr int P = NF / 8;
  constexpr int BASE = sizeof(TC) == 4 ? 16 : 8;          // pairs per tile
  constexpr int NPAIR0 = (BASE * P < 64) ? (64 / P) : BASE;
  constexpr int NPAIR = (NPAIR0 * P > 1024) ? (1024 / P) : NPAIR0;
  constexpr int T = 2 * NPAIR;
  const int64_t ntiles = (p.M + T - 1) / T;
  const int L = (int)p.nblocks;
  // split the blocks over workgroups only when the tiles alone cannot fill the GPU
  int64_t chunks = 1;
  if (ntiles < 4096) chunks = (4096 + ntiles - 1) / ntiles;
  if (chunks > L) chunks = L;
  const int bpw = (int)((L + chunks - 1) / chunks);
  chunks = (L + bpw - 1) / bpw;
  if (ntiles > 0x7fffffff) return fail(SPOD_ERR_UNSUPPORTED, "too many tiles");
  dim3 grid((unsigned)ntiles, (unsigned)chunks);
  const C* tw = reinterpret_cast<const C*>(sizeof(TC) == 4 ? (const void*)p.d_tw32 : (const void*)p.d_tw64);
  if (p.step * 2 == NF)
    hipLaunchKernelGGL((blocks_fft_kernel<NF, TC, TIN, NPAIR, 4>), grid, dim3(NPAIR * P), 0, st, q,
                       mean, p.d_window, tw, reinterpret_cast<C*>(qhat), (int64_t)p.M,
                       (int64_t)p.nt, (int)p.step, L, bpw, (TC)p.kappa);
  else
    hipLaunchKernelGGL((blocks_fft_kernel<NF, TC, TIN, NPAIR, 8>), grid, dim3(NPAIR * P), 0, st, q,
                       mean, p.d_window, tw, reinterpret_cast<C*>(qhat), (int64_t)p.M,
                       (int64_t)p.nt, (int)p.step, L, bpw, (TC)p.kappa);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPOD_OK : hip_fail(e, "blocks_fft_kernel");
}

template <typename TC, typename TIN>
static spod_status launch_fft_t(const Plan& p, const TIN* q, const double* mean, void* qhat,
                                hipStream_t st) {
  switch (p.nfft) {
    case 8: return launch_fft_nf<8, TC, TIN>(p, q, mean, qhat, st);
    case 16: return launch_fft_nf<16, TC, TIN>(p, q, mean, qhat, st);
    case 32: return launch_fft_nf<32, TC, TIN>(p, q, mean, qhat, st);
    case 64: return launch_fft_nf<64, TC, TIN>(p, q, mean, qhat, st);
    case 128: return launch_fft_nf<128, TC, TIN>(p, q, mean, qhat, st);
    case 256: return launch_fft_nf<256, TC, TIN>(p, q, mean, qhat, st);
    case 512: return launch_fft_nf<512, TC, TIN>(p, q, mean, qhat, st);
    case 1024: return launch_fft_nf<1024, TC, TIN>(p, q, mean, qhat, st);
  }
  return fail(SPOD_ERR_UNSUPPORTED, "nfft");
}

size_t fft_workspace(const Plan& p) { return sizeof(double) * (size_t)p.M; }

spod_status launch_blocks_fft(const Plan& p, const void* q, spod_dtype dtype, void* qhat,
                              double* mean, void* ws, hipStream_t st) {
  // the mean goes to the caller's buffer, or to the start of the workspace
  double* mu = mean ? mean : static_cast<double*>(ws);
  const int64_t mgrid = (p.M + 3) / 4;
  if (dtype == SPOD_F32)
    hipLaunchKernelGGL(mean_kernel<float>, dim3((unsigned)mgrid), dim3(256), 0, st,
                       (const float*)q, mu, (int64_t)p.M, (int64_t)p.nt);
  else
    hipLaunchKernelGGL(mean_kernel<double>, dim3((unsigned)mgrid), dim3(256), 0, st,
                       (const double*)q, mu, (int64_t)p.M, (int64_t)p.nt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "mean_kernel");
  spod_status s;
  const bool c128 = is_complex128(p);
  if (dtype == SPOD_F32)
    s = c128 ? launch_fft_t<double, float>(p, (const float*)q, mu, qhat, st)
             : launch_fft_t<float, float>(p, (const float*)q, mu, qhat, st);
  else
    s = c128 ? launch_fft_t<double, double>(p, (const double*)q, mu, qhat, st)
             : launch_fft_t<float, double>(p, (const double*)q, mu, qhat, st);
  return s;
}

}  // namespace spod
