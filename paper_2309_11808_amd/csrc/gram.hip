// Steps 3-4 of SPOD (eq. (spod-discrete-snapshots); Sec. 3.1 steps 3-4): the
// weighted inner product M_k = Qhat_k^* W Qhat_k for every frequency.
//
// Realified form.  With Y = sqrt(W) [Re Qhat_k^T ; Im Qhat_k^T] (2L rows, M
// columns), P = Y Y^T is a real symmetric (2L x 2L) matrix and
//   M_k[i][j] = (P[i][j] + P[L+i][L+j]) + i (P[i][L+j] - P[L+i][j]).
// P is a single SYRK with a long contraction over the degrees of freedom, run
// on MFMA in 16x16 output tiles (upper triangle of tiles only).  The paper
// reduces this sum over space across MPI ranks; here the M axis is split into
// S slices, one workgroup per (slice, frequency), and the S partial P's are
// combined in FP64 by a second kernel.
//
// Arithmetic per precision:
//   FP64    v_mfma_f64_16x16x4f64, FP64 accumulation.
//   FP32    v_mfma_f32_16x16x4f32 started from zero at every 4-wide step and
//           added into FP64 registers at once.
//   BF16X4  y = hi + lo with hi = bf16(y), lo = bf16(y - hi) (round to nearest
//           even) and all four products hi hi^T + hi lo^T + lo hi^T + lo lo^T
//           on v_mfma_f32_16x16x32_bf16: the exact product of the 16-bit
//           representation.  Dropping lo lo^T (the common three-product
//           scheme) is not used: on a Gram matrix it is a one-signed bias of
//           the diagonal (sum of lo^2) that shifts every small eigenvalue.
//           The dominant hi hi^T product starts from zero at every 32-wide
//           step and is added into FP64 at once, so each FP32 rounding only
//           sees 32 products; the three small correction products share one
//           FP32 accumulator flushed every 16 steps.
//   FP16X4  the same with FP16 operands, y scaled per frequency by a power of
//           two so that max |y| lies in [2^14, 2^15) (gram_scale_kernel).
#include <hip/hip_runtime.h>

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
  using TL = double;            // LDS element
  using C = double2;            // qhat element
  static constexpr int KS = 4;  // contraction per MFMA
  static constexpr int MC = 64; // degrees of freedom per LDS chunk
  using ACC = v4d;
};
template <> struct GramCfg<G_F32> {
  using TL = float;
  using C = float2;
  static constexpr int KS = 4;
  static constexpr int MC = 128;
  using ACC = v4f;
};
template <> struct GramCfg<G_BF16X4> {
  using TL = float;
  using C = float2;
  static constexpr int KS = 32;
  static constexpr int MC = 128;
  using ACC = v4f;
};
template <> struct GramCfg<G_FP16X4> {
  using TL = float;
  using C = float2;
  static constexpr int KS = 32;
  static constexpr int MC = 128;
  using ACC = v4f;
};

__device__ __forceinline__ void split_bf16(const float* y, v8bf& hi, v8bf& lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    __bf16 h = (__bf16)y[e];
    hi[e] = h;
    lo[e] = (__bf16)(y[e] - (float)h);
  }
}

__device__ __forceinline__ void split_f16(const float* y, float s, v8h& hi, v8h& lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float v = y[e] * s;
    _Float16 h = (_Float16)v;
    hi[e] = h;
    lo[e] = (_Float16)(v - (float)h);
  }
}

// NTI = tiles of 16 per side (2L <= 16*NTI); NP = NTI(NTI+1)/2 upper tile
// pairs, processed in groups of at most PG = 10 (grid z), so each lane holds
// at most 10 accumulator tiles.  The four waves of a workgroup split the
// contraction and are summed through LDS at the end.
constexpr int PG = 10;

template <int MODE, int NTI, int G>
__device__ __forceinline__ void gram_body(const typename GramCfg<MODE>::C* __restrict__ qhat,
                                          const typename GramCfg<MODE>::TL* __restrict__ sqrtw,
                                          float scale, double* __restrict__ part, int64_t M,
                                          int L, int S, typename GramCfg<MODE>::TL* Y) {
  using Cfg = GramCfg<MODE>;
  using TL = typename Cfg::TL;
  using C = typename Cfg::C;
  using ACC = typename Cfg::ACC;
  constexpr int KS = Cfg::KS, MC = Cfg::MC;
  constexpr int D = 16 * NTI;
  constexpr int NP = NTI * (NTI + 1) / 2;
  constexpr int P0 = G * PG;
  constexpr int NPG = (NP - P0) < PG ? (NP - P0) : PG;   // pairs in this group
  constexpr int LDY = MC + (sizeof(TL) == 8 ? 4 : 8);
  constexpr bool FLUSH = MODE == G_BF16X4 || MODE == G_FP16X4;  // correction accumulator
  constexpr int NSTEP = MC / KS;
  static_assert(NSTEP % 4 == 0, "chunk must split over four waves");
  constexpr int SPW = NSTEP / 4;                             // steps per wave per chunk

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int s = blockIdx.x;
  const int k = blockIdx.y;

  const int64_t nchunks = (M + MC - 1) / MC;
  const int64_t c0 = nchunks * s / S, c1 = nchunks * (s + 1) / S;

  for (int idx = tid; idx < (D - 2 * L) * LDY; idx += 256) Y[2 * L * LDY + idx] = (TL)0;

  ACC acc[NPG];
  double acc64[NPG][4];
#pragma unroll
  for (int i = 0; i < NPG; ++i) {
    acc[i] = ACC{0, 0, 0, 0};
#pragma unroll
    for (int v = 0; v < 4; ++v) acc64[i][v] = 0.0;
  }

  const C* base = qhat + (int64_t)k * L * M;
  int since_flush = 0;
  for (int64_t c = c0; c < c1; ++c) {
    const int64_t m0 = c * MC;
    __syncthreads();
    for (int idx = tid; idx < L * MC; idx += 256) {
      const int l = idx / MC, mm = idx % MC;
      const int64_t m = m0 + mm;
      TL re = 0, im = 0;
      if (m < M) {
        const C z = base[(int64_t)l * M + m];
        const TL w = sqrtw[m];
        re = z.x * w;
        im = z.y * w;
      }
      Y[l * LDY + mm] = re;
      Y[(L + l) * LDY + mm] = im;
    }
    __syncthreads();

#pragma unroll 1
    for (int st = 0; st < SPW; ++st) {
      const int kk0 = (wave * SPW + st) * KS;
      if constexpr (MODE == G_F64 || MODE == G_F32) {
        TL fr[NTI];
#pragma unroll
        for (int a = 0; a < NTI; ++a) fr[a] = Y[(16 * a + (lane & 15)) * LDY + kk0 + (lane >> 4)];
        int pi = 0;
#pragma unroll
        for (int a = 0; a < NTI; ++a) {
#pragma unroll
          for (int b = a; b < NTI; ++b, ++pi) {
            if (pi >= P0 && pi < P0 + NPG) {
              if constexpr (MODE == G_F64) {
                acc[pi - P0] = __builtin_amdgcn_mfma_f64_16x16x4f64(fr[a], fr[b], acc[pi - P0], 0, 0, 0);
              } else {
                const ACC t = __builtin_amdgcn_mfma_f32_16x16x4f32(fr[a], fr[b], ACC{0, 0, 0, 0}, 0, 0, 0);
#pragma unroll
                for (int v = 0; v < 4; ++v) acc64[pi - P0][v] += (double)t[v];
              }
            }
          }
        }
      } else {
        using FR = typename std::conditional<MODE == G_BF16X4, v8bf, v8h>::type;
        FR hi[NTI], lo[NTI];
#pragma unroll
        for (int a = 0; a < NTI; ++a) {
          const TL* src = &Y[(16 * a + (lane & 15)) * LDY + kk0 + 8 * (lane >> 4)];
          float y[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) y[e] = src[e];
          if constexpr (MODE == G_BF16X4) split_bf16(y, hi[a], lo[a]);
          else split_f16(y, scale, hi[a], lo[a]);
        }
        int pi = 0;
#pragma unroll
        for (int a = 0; a < NTI; ++a) {
#pragma unroll
          for (int b = a; b < NTI; ++b, ++pi) {
            if (pi >= P0 && pi < P0 + NPG) {
              ACC& x = acc[pi - P0];
              ACC t;
              if constexpr (MODE == G_BF16X4) {
                t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hi[a], hi[b], ACC{0, 0, 0, 0}, 0, 0, 0);
                x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hi[a], lo[b], x, 0, 0, 0);
                x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lo[a], hi[b], x, 0, 0, 0);
                x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lo[a], lo[b], x, 0, 0, 0);
              } else {
                t = __builtin_amdgcn_mfma_f32_16x16x32_f16(hi[a], hi[b], ACC{0, 0, 0, 0}, 0, 0, 0);
                x = __builtin_amdgcn_mfma_f32_16x16x32_f16(hi[a], lo[b], x, 0, 0, 0);
                x = __builtin_amdgcn_mfma_f32_16x16x32_f16(lo[a], hi[b], x, 0, 0, 0);
                x = __builtin_amdgcn_mfma_f32_16x16x32_f16(lo[a], lo[b], x, 0, 0, 0);
              }
#pragma unroll
              for (int v = 0; v < 4; ++v) acc64[pi - P0][v] += (double)t[v];
            }
          }
        }
      }
    }
    if constexpr (FLUSH) {
      if (++since_flush == 16) {
        since_flush = 0;
#pragma unroll
        for (int i = 0; i < NPG; ++i) {
#pragma unroll
          for (int v = 0; v < 4; ++v) acc64[i][v] += (double)acc[i][v];
          acc[i] = ACC{0, 0, 0, 0};
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NPG; ++i) {
#pragma unroll
    for (int v = 0; v < 4; ++v) acc64[i][v] += (double)acc[i][v];
  }
  if constexpr (MODE == G_FP16X4) {
    const double inv = 1.0 / ((double)scale * (double)scale);
#pragma unroll
    for (int i = 0; i < NPG; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc64[i][v] *= inv;
  }

  // sum the four waves in LDS (the tile buffer is free now), one wave at a time
  double* red = reinterpret_cast<double*>(Y);
  static_assert(sizeof(TL) * D * LDY >= sizeof(double) * NPG * 4 * 64, "reduction buffer");
  __syncthreads();
#pragma unroll 1
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int i = 0; i < NPG; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double* r = &red[(i * 4 + v) * 64 + lane];
          *r = (w == 0) ? acc64[i][v] : *r + acc64[i][v];
        }
    }
    __syncthreads();
  }
  // element (lane, v) of a 16x16 result tile sits in column lane%16 and row
  // 4*(lane/16)+v for the FP32-accumulating instructions, but row lane/16+4*v
  // for v_mfma_f64_16x16x4f64
  double* out = part + ((int64_t)k * S + s) * D * D;
  for (int idx = tid; idx < NPG * 4 * 64; idx += 256) {
    const int ln = idx & 63;
    const int v = (idx >> 6) & 3;
    const int pi = P0 + (idx >> 8);
    int a = 0, rem = pi;
    while (rem >= NTI - a) {
      rem -= NTI - a;
      ++a;
    }
    const int b = a + rem;
    const int r = (MODE == G_F64) ? (ln >> 4) + 4 * v : 4 * (ln >> 4) + v;
    out[(16 * a + r) * D + 16 * b + (ln & 15)] = red[idx];
  }
}

template <int MODE, int NTI>
__global__ __launch_bounds__(256) void gram_kernel(const typename GramCfg<MODE>::C* __restrict__ qhat,
                                                   const void* __restrict__ sqrtw_v,
                                                   const float* __restrict__ fscale,
                                                   double* __restrict__ part, int64_t M, int L,
                                                   int S) {
  using Cfg = GramCfg<MODE>;
  using TL = typename Cfg::TL;
  constexpr int D = 16 * NTI;
  constexpr int LDY = Cfg::MC + (sizeof(TL) == 8 ? 4 : 8);
  constexpr int NP = NTI * (NTI + 1) / 2;
  constexpr int NG = (NP + PG - 1) / PG;
  __shared__ TL Y[D * LDY];
  const TL* sqrtw = static_cast<const TL*>(sqrtw_v);
  const float scale = (MODE == G_FP16X4) ? fscale[blockIdx.y] : 1.0f;
  switch (blockIdx.z) {
    case 0: gram_body<MODE, NTI, 0>(qhat, sqrtw, scale, part, M, L, S, Y); break;
    case 1: if constexpr (NG > 1) gram_body<MODE, NTI, 1>(qhat, sqrtw, scale, part, M, L, S, Y); break;
    case 2: if constexpr (NG > 2) gram_body<MODE, NTI, 2>(qhat, sqrtw, scale, part, M, L, S, Y); break;
    case 3: if constexpr (NG > 3) gram_body<MODE, NTI, 3>(qhat, sqrtw, scale, part, M, L, S, Y); break;
    default: break;
  }
}

// Sum the S slices of P in FP64 and assemble the complex Hermitian M_k.
__global__ __launch_bounds__(256) void gram_combine_kernel(const double* __restrict__ part,
                                                           double2* __restrict__ gram, int L, int D,
                                                           int S) {
  const int k = blockIdx.x;
  const double* pk = part + (int64_t)k * S * D * D;
  for (int idx = threadIdx.x; idx < L * L; idx += blockDim.x) {
    const int i = idx / L, j = idx % L;
    // P is stored on upper tiles (tile(row) <= tile(col)); mirror otherwise
    auto at = [&](const double* P, int r, int c) {
      return ((r >> 4) <= (c >> 4)) ? P[r * D + c] : P[c * D + r];
    };
    double re = 0.0, im = 0.0;
    for (int s = 0; s < S; ++s) {
      const double* P = pk + (int64_t)s * D * D;
      re += at(P, i, j) + at(P, L + i, L + j);
      im += at(P, i, L + j) - at(P, L + i, j);
    }
    gram[((int64_t)k * L + i) * L + j] = make_double2(re, im);
  }
}

// Per-frequency power-of-two scale for the FP16 operands: 2^(15 - e) with e
// the exponent of max_m,l |sqrt(W_m) qhat[k][l][m]| (real or imaginary part),
// so the largest scaled value lies in [2^14, 2^15) < 65504.
__global__ __launch_bounds__(256) void gram_scale_kernel(const float2* __restrict__ qhat,
                                                         const float* __restrict__ sqrtw,
                                                         float* __restrict__ scale, int64_t M, int L) {
  const int k = blockIdx.x;
  const float2* base = qhat + (int64_t)k * L * M;
  float mx = 0.0f;
  for (int64_t idx = threadIdx.x; idx < (int64_t)L * M; idx += 256) {
    const float2 z = base[idx];
    const float w = sqrtw[idx % M];
    mx = fmaxf(mx, fmaxf(fabsf(z.x * w), fabsf(z.y * w)));
  }
  __shared__ float red[256];
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float m = red[0];
    int e = 0;
    if (m > 0.0f) (void)frexpf(m, &e);
    scale[k] = ldexpf(1.0f, 15 - e);
  }
}

// ---------------------------------------------------------------------------
size_t csd_workspace(const Plan& p) {
  const size_t D = (size_t)p.gram_dim;
  size_t b = sizeof(double) * (size_t)p.nfreq * (size_t)p.gram_split * D * D;
  if (p.prec == SPOD_PREC_FP16X4) b += sizeof(float) * (size_t)p.nfreq + 256;
  return b;
}

template <int MODE, int NTI>
static void launch_gram_nti(const Plan& p, const void* qhat, const void* sqrtw, const float* fs,
                            double* part, hipStream_t st) {
  using C = typename GramCfg<MODE>::C;
  constexpr int NP = NTI * (NTI + 1) / 2;
  dim3 grid((unsigned)p.gram_split, (unsigned)p.nfreq, (unsigned)((NP + PG - 1) / PG));
  hipLaunchKernelGGL((gram_kernel<MODE, NTI>), grid, dim3(256), 0, st,
                     static_cast<const C*>(qhat), sqrtw, fs, part, (int64_t)p.M, (int)p.nblocks,
                     p.gram_split);
}

template <int MODE>
static spod_status launch_gram_mode(const Plan& p, const void* qhat, const void* sqrtw,
                                    const float* fs, double* part, hipStream_t st) {
  switch (p.gram_dim / 16) {
    case 1: launch_gram_nti<MODE, 1>(p, qhat, sqrtw, fs, part, st); break;
    case 2: launch_gram_nti<MODE, 2>(p, qhat, sqrtw, fs, part, st); break;
    case 3: launch_gram_nti<MODE, 3>(p, qhat, sqrtw, fs, part, st); break;
    case 4: launch_gram_nti<MODE, 4>(p, qhat, sqrtw, fs, part, st); break;
    case 5: launch_gram_nti<MODE, 5>(p, qhat, sqrtw, fs, part, st); break;
    case 6: launch_gram_nti<MODE, 6>(p, qhat, sqrtw, fs, part, st); break;
    case 7: launch_gram_nti<MODE, 7>(p, qhat, sqrtw, fs, part, st); break;
    case 8: launch_gram_nti<MODE, 8>(p, qhat, sqrtw, fs, part, st); break;
    default: return fail(SPOD_ERR_UNSUPPORTED, "nblocks > 64");
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPOD_OK : hip_fail(e, "gram_kernel");
}

spod_status launch_csd(const Plan& p, const void* qhat, void* gram, void* ws, hipStream_t st) {
  if (p.nblocks > 64) return fail(SPOD_ERR_UNSUPPORTED, "nblocks > 64");
  double* part = static_cast<double*>(ws);
  const size_t D = (size_t)p.gram_dim;
  float* fs = reinterpret_cast<float*>(
      static_cast<char*>(ws) + sizeof(double) * (size_t)p.nfreq * (size_t)p.gram_split * D * D);
  spod_status s;
  switch (p.prec) {
    case SPOD_PREC_FP64: s = launch_gram_mode<G_F64>(p, qhat, p.d_sqrtw, nullptr, part, st); break;
    case SPOD_PREC_FP32: s = launch_gram_mode<G_F32>(p, qhat, p.d_sqrtw32, nullptr, part, st); break;
    case SPOD_PREC_BF16X4: s = launch_gram_mode<G_BF16X4>(p, qhat, p.d_sqrtw32, nullptr, part, st); break;
    case SPOD_PREC_FP16X4:
      hipLaunchKernelGGL(gram_scale_kernel, dim3((unsigned)p.nfreq), dim3(256), 0, st,
                         static_cast<const float2*>(qhat), p.d_sqrtw32, fs, (int64_t)p.M,
                         (int)p.nblocks);
      s = launch_gram_mode<G_FP16X4>(p, qhat, p.d_sqrtw32, fs, part, st);
      break;
    default: return fail(SPOD_ERR_INVALID_ARG, "precision");
  }
  if (s != SPOD_OK) return s;
  hipLaunchKernelGGL(gram_combine_kernel, dim3((unsigned)p.nfreq), dim3(256), 0, st, part,
                     static_cast<double2*>(gram), (int)p.nblocks, (int)D, p.gram_split);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPOD_OK : hip_fail(e, "gram_combine_kernel");
}

}  // namespace spod
