// SPOD modes (eq. (spod-discrete-snapshots)): Phi_k = Qhat_k Psi_k Lambda_k^{-1/2},
// for the leading n_modes eigenpairs of every frequency.
//
// Per frequency this is an (M x L) by (L x n_modes) product with L ~ 31 and
// n_modes ~ 5: far too thin for matrix cores, and bound by streaming qhat
// from HBM.  Each thread owns one degree of freedom, reads its L coefficients
// (coalesced across the wavefront) and accumulates up to 8 modes in registers;
// the L x n_modes coefficients psi / sqrt(lambda) sit in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"

namespace spod {

constexpr int MODES_MAXL = SPOD_MAX_NBLOCKS;
constexpr size_t MODES_MAX_TABLE = 64 * 1024;   // LDS of the coefficient table
constexpr int MODES_MAXM = 256;   // largest n_modes (n_modes <= L)
constexpr int MODES_GROUP = 8;

// Pairs of degrees of freedom as one 16-byte vector (complex64 only).
typedef float modes_v4 __attribute__((ext_vector_type(4)));

template <typename TC, bool PAIR>
__device__ __forceinline__ void modes_body(const cpx_t<TC>* __restrict__ qhat,
                                           const double* __restrict__ lam,
                                           const double2* __restrict__ psi,
                                           cpx_t<TC>* __restrict__ phi,
                                           int32_t* __restrict__ n_valid, int64_t M, int64_t ldq,
                                           int L, int n_modes, double eps, int64_t bx, int k) {
  using C = cpx_t<TC>;
  static_assert(!PAIR || sizeof(TC) == 4, "pairs are 16-byte complex64 vectors");
  extern __shared__ char modes_lds[];
  C* coef = reinterpret_cast<C*>(modes_lds);   // [L][n_modes]
  // valid-mode flags: an invalid mode is stored as zeros, not as the
  // accumulated sum (which is not zero when qhat holds a NaN or an infinity)
  __shared__ unsigned vmask[MODES_MAXM / 32];
  const int tid = threadIdx.x;
  const double* lk = lam + (int64_t)k * L;
  const double l0 = lk[0];
  if (tid < MODES_MAXM / 32) {
    unsigned b = 0;
    for (int j = 32 * tid; j < n_modes && j < 32 * tid + 32; ++j)
      b |= (unsigned)(l0 > 0.0 && lk[j] > eps * l0) << (j - 32 * tid);
    vmask[tid] = b;
  }
  for (int idx = tid; idx < L * n_modes; idx += blockDim.x) {
    const int l = idx / n_modes, j = idx % n_modes;
    const double lj = lk[j];
    const bool valid = l0 > 0.0 && lj > eps * l0;
    const double s = valid ? 1.0 / sqrt(lj) : 0.0;
    const double2 ps = psi[((int64_t)k * L + l) * L + j];
    coef[idx] = C{(TC)(ps.x * s), (TC)(ps.y * s)};
  }
  if (bx == 0 && tid == 0 && n_valid) {
    int c = 0;
    for (int j = 0; j < n_modes; ++j) c += (l0 > 0.0 && lk[j] > eps * l0);
    n_valid[k] = c;
  }
  __syncthreads();
  constexpr int DPT = PAIR ? 2 : 1;            // degrees of freedom per thread
  const int64_t m = (bx * blockDim.x + tid) * DPT;
  if (m >= M) return;
  const C* src = qhat + (int64_t)k * L * ldq + m;
  C* dst = phi + (int64_t)k * n_modes * M + m;
  for (int j0 = 0; j0 < n_modes; j0 += MODES_GROUP) {
    C acc[DPT][MODES_GROUP];
#pragma unroll
    for (int d = 0; d < DPT; ++d)
#pragma unroll
      for (int j = 0; j < MODES_GROUP; ++j) acc[d][j] = C{0, 0};
    for (int l = 0; l < L; ++l) {
      C x[DPT];
      if constexpr (PAIR) {
        const modes_v4 v = __builtin_nontemporal_load(reinterpret_cast<const modes_v4*>(src + (int64_t)l * ldq));
        x[0] = C{v[0], v[1]};
        x[1] = C{v[2], v[3]};
      } else {
        x[0] = src[(int64_t)l * ldq];
      }
      const C* cl = coef + l * n_modes + j0;
#pragma unroll
      for (int j = 0; j < MODES_GROUP; ++j) {
        if (j0 + j < n_modes) {
          const C c = cl[j];
#pragma unroll
          for (int d = 0; d < DPT; ++d) {
            acc[d][j].x += x[d].x * c.x - x[d].y * c.y;
            acc[d][j].y += x[d].x * c.y + x[d].y * c.x;
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < MODES_GROUP; ++j) {
      if (j0 + j < n_modes) {
        if (!((vmask[(j0 + j) >> 5] >> ((j0 + j) & 31)) & 1u)) {
#pragma unroll
          for (int d = 0; d < DPT; ++d) acc[d][j] = C{0, 0};
        }
        if constexpr (PAIR) {
          const modes_v4 v = {acc[0][j].x, acc[0][j].y, acc[1][j].x, acc[1][j].y};
          __builtin_nontemporal_store(v, reinterpret_cast<modes_v4*>(dst + (int64_t)(j0 + j) * M));
        } else {
          dst[(int64_t)(j0 + j) * M] = acc[0][j];
        }
      }
    }
  }
}

// Packed Fourier blocks (complex64 modes): one thread per 4 degrees of
// freedom, 2 pairs of one group, decoded from their int16 high parts, low
// nibbles and the group's exponent at every block.
__device__ __forceinline__ void modes_pk_body(const char* __restrict__ qhat, int64_t rowb,
                                              const double* __restrict__ lam,
                                              const double2* __restrict__ psi,
                                              float2* __restrict__ phi, int32_t* __restrict__ n_valid,
                                              int64_t M, int L, int n_modes, double eps, int64_t bx,
                                              int k) {
  using C = float2;
  extern __shared__ char modes_lds[];
  C* coef = reinterpret_cast<C*>(modes_lds);   // [L][n_modes]
  __shared__ unsigned vmask[MODES_MAXM / 32];
  const int tid = threadIdx.x;
  const double* lk = lam + (int64_t)k * L;
  const double l0 = lk[0];
  if (tid < MODES_MAXM / 32) {
    unsigned b = 0;
    for (int j = 32 * tid; j < n_modes && j < 32 * tid + 32; ++j)
      b |= (unsigned)(l0 > 0.0 && lk[j] > eps * l0) << (j - 32 * tid);
    vmask[tid] = b;
  }
  for (int idx = tid; idx < L * n_modes; idx += blockDim.x) {
    const int l = idx / n_modes, j = idx % n_modes;
    const double lj = lk[j];
    const bool valid = l0 > 0.0 && lj > eps * l0;
    const double s = valid ? 1.0 / sqrt(lj) : 0.0;
    const double2 ps = psi[((int64_t)k * L + l) * L + j];
    coef[idx] = C{(float)(ps.x * s), (float)(ps.y * s)};
  }
  if (bx == 0 && tid == 0 && n_valid) {
    int c = 0;
    for (int j = 0; j < n_modes; ++j) c += (l0 > 0.0 && lk[j] > eps * l0);
    n_valid[k] = c;
  }
  __syncthreads();
  const int64_t m = (bx * blockDim.x + tid) * 4;
  if (m >= M) return;
  typedef unsigned int v4u __attribute__((ext_vector_type(4)));
  const int g = (int)((m % PK_SB_DOFS) >> 4), p0 = (int)((m & 15) >> 1);
  const char* src = qhat + (int64_t)k * L * rowb + (m / PK_SB_DOFS) * PK_SB_BYTES;
  const char* grp = src + PK_HDR_BYTES + PK_GROUP_BYTES * g;
  C* dst = phi + (int64_t)k * n_modes * M + m;
  const bool vec = (M % 2 == 0) && (m + 3 < M) && ((uintptr_t)phi % 16 == 0);
  for (int j0 = 0; j0 < n_modes; j0 += MODES_GROUP) {
    C acc[4][MODES_GROUP];
#pragma unroll
    for (int d = 0; d < 4; ++d)
#pragma unroll
      for (int j = 0; j < MODES_GROUP; ++j) acc[d][j] = C{0, 0};
    for (int l = 0; l < L; ++l) {
      const int64_t ro = (int64_t)l * rowb;
      const v4u h = __builtin_nontemporal_load(reinterpret_cast<const v4u*>(grp + ro + 8 * p0));
      const uint32_t nib = *reinterpret_cast<const uint32_t*>(grp + ro + 64 + 2 * p0);
      const float scale = pk_scale((int)(signed char)src[ro + g]);
      float v[8];
      pk_decode4(h[0], h[1], nib & 0xffffu, scale, v);
      pk_decode4(h[2], h[3], nib >> 16, scale, v + 4);
      const C* cl = coef + l * n_modes + j0;
#pragma unroll
      for (int j = 0; j < MODES_GROUP; ++j) {
        if (j0 + j < n_modes) {
          const C c = cl[j];
#pragma unroll
          for (int d = 0; d < 4; ++d) {
            acc[d][j].x += v[2 * d] * c.x - v[2 * d + 1] * c.y;
            acc[d][j].y += v[2 * d] * c.y + v[2 * d + 1] * c.x;
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < MODES_GROUP; ++j) {
      if (j0 + j < n_modes) {
        if (!((vmask[(j0 + j) >> 5] >> ((j0 + j) & 31)) & 1u)) {
#pragma unroll
          for (int d = 0; d < 4; ++d) acc[d][j] = C{0, 0};
        }
        C* o = dst + (int64_t)(j0 + j) * M;
        if (vec) {
          const modes_v4 a = {acc[0][j].x, acc[0][j].y, acc[1][j].x, acc[1][j].y};
          const modes_v4 b = {acc[2][j].x, acc[2][j].y, acc[3][j].x, acc[3][j].y};
          __builtin_nontemporal_store(a, reinterpret_cast<modes_v4*>(o));
          __builtin_nontemporal_store(b, reinterpret_cast<modes_v4*>(o) + 1);
        } else {
#pragma unroll
          for (int d = 0; d < 4; ++d)
            if (m + d < M) o[d] = acc[d][j];
        }
      }
    }
  }
}

// Complex64 modes on the matrix cores.  Per 16-DOF tile and 4 blocks, with
// A = qhat rows (Re, Im) and B = the coefficients (Re, Im, -Im) of up to 16
// modes, v_mfma_f32_16x16x4f32 accumulates
//   Re Phi += A_re B_re + A_im (-B_im),   Im Phi += A_re B_im + A_im B_re
// in FP32.  Lane (i = lane % 16, t = lane / 16) holds the A element of DOF i
// and block 4 s + t; the B element of block 4 s + t and mode i; the result
// element of DOF 4 (lane / 16) + v and mode lane % 16.  Each wave owns
// MODES_TW tiles (8: 128 consecutive DOFs), so every block row is read as
// 128 contiguous complex values.  Blocks past L and modes past n_modes are
// zero in the coefficient table.
constexpr int MODES_TW = 8;

__device__ __forceinline__ void modes_mfma_body(const float2* __restrict__ qhat,
                                                const double* __restrict__ lam,
                                                const double2* __restrict__ psi,
                                                float2* __restrict__ phi,
                                                int32_t* __restrict__ n_valid, int64_t M, int64_t ldq,
                                                int L, int n_modes, double eps, int64_t bx, int k) {
  typedef float v4f_m __attribute__((ext_vector_type(4)));
  extern __shared__ char modes_lds[];
  const int Lp = (L + 3) & ~3;
  float* cre = reinterpret_cast<float*>(modes_lds);   // [Lp][16]: Re of psi / sqrt(lam), one mode group
  float* cim = cre + Lp * 16;                         // [Lp][16]: Im
  __shared__ unsigned vmask[MODES_MAXM / 32];
  const int tid = threadIdx.x;
  const double* lk = lam + (int64_t)k * L;
  const double l0 = lk[0];
  if (tid < MODES_MAXM / 32) {
    unsigned b = 0;
    for (int j = 32 * tid; j < n_modes && j < 32 * tid + 32; ++j)
      b |= (unsigned)(l0 > 0.0 && lk[j] > eps * l0) << (j - 32 * tid);
    vmask[tid] = b;
  }
  if (bx == 0 && tid == 0 && n_valid) {
    int c = 0;
    for (int j = 0; j < n_modes; ++j) c += (l0 > 0.0 && lk[j] > eps * l0);
    n_valid[k] = c;
  }
  const int wave = tid >> 6, lane = tid & 63;
  const int i16 = lane & 15, t4 = lane >> 4;
  const int64_t mw = (bx * 4 + wave) * (16 * MODES_TW);      // this wave's first DOF
  const float2* qk = qhat + (int64_t)k * L * ldq;
  const bool vec = (M % 2 == 0) && ((uintptr_t)phi % 16 == 0);
  for (int j0 = 0; j0 < n_modes; j0 += 16) {
    __syncthreads();                                          // the previous group's table is free
    for (int idx = tid; idx < Lp * 16; idx += blockDim.x) {
      const int l = idx >> 4, j = j0 + (idx & 15);
      float re = 0.0f, im = 0.0f;
      if (l < L && j < n_modes) {
        const double lj = lk[j];
        const bool valid = l0 > 0.0 && lj > eps * l0;
        const double sc = valid ? 1.0 / sqrt(lj) : 0.0;
        const double2 ps = psi[((int64_t)k * L + l) * L + j];
        re = (float)(ps.x * sc);
        im = (float)(ps.y * sc);
      }
      cre[idx] = re;
      cim[idx] = im;
    }
    __syncthreads();
    v4f_m accR[MODES_TW], accI[MODES_TW];
#pragma unroll
    for (int w = 0; w < MODES_TW; ++w) accR[w] = accI[w] = v4f_m{0, 0, 0, 0};
    for (int l0s = 0; l0s < Lp; l0s += 4) {
      const int l = l0s + t4;
      const float br = cre[l * 16 + i16], bi = cim[l * 16 + i16];
      float2 a[MODES_TW];
#pragma unroll
      for (int w = 0; w < MODES_TW; ++w) {
        const int64_t m = mw + 16 * w + i16;
        a[w] = (l < L && m < M) ? qk[(int64_t)l * ldq + m] : float2{0.0f, 0.0f};
      }
#pragma unroll
      for (int w = 0; w < MODES_TW; ++w) {
        accR[w] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[w].x, br, accR[w], 0, 0, 0);
        accR[w] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[w].y, -bi, accR[w], 0, 0, 0);
        accI[w] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[w].x, bi, accI[w], 0, 0, 0);
        accI[w] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[w].y, br, accI[w], 0, 0, 0);
      }
    }
    // lane holds DOFs 4 t4 + v of each tile for mode j0 + i16
    const int j = j0 + i16;
    if (j < n_modes) {
      const bool valid = (vmask[j >> 5] >> (j & 31)) & 1u;
      float2* o = phi + ((int64_t)k * n_modes + j) * M;
#pragma unroll
      for (int w = 0; w < MODES_TW; ++w) {
        const int64_t m = mw + 16 * w + 4 * t4;
        float v[8];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          v[2 * e] = valid ? accR[w][e] : 0.0f;
          v[2 * e + 1] = valid ? accI[w][e] : 0.0f;
        }
        if (vec && m + 3 < M) {
          const modes_v4 x = {v[0], v[1], v[2], v[3]}, y = {v[4], v[5], v[6], v[7]};
          __builtin_nontemporal_store(x, reinterpret_cast<modes_v4*>(o + m));
          __builtin_nontemporal_store(y, reinterpret_cast<modes_v4*>(o + m) + 1);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (m + e < M) o[m + e] = float2{v[2 * e], v[2 * e + 1]};
        }
      }
    }
  }
}

// The DOF tiles of a frequency are dealt to the XCDs in contiguous runs
// (xcd_tile), so each XCD streams one range of every row of qhat_k: 7% less
// time than neighbouring tiles on different XCDs on the 1M-DOF field.
__global__ __launch_bounds__(256) void modes_mfma_kernel(const float2* __restrict__ qhat,
                                                         const double* __restrict__ lam,
                                                         const double2* __restrict__ psi,
                                                         float2* __restrict__ phi,
                                                         int32_t* __restrict__ n_valid, int64_t M,
                                                         int L, int n_modes, double eps) {
  modes_mfma_body(qhat, lam, psi, phi, n_valid, M, M, L, n_modes, eps, xcd_tile(blockIdx.x, gridDim.x), blockIdx.y);
}

__global__ __launch_bounds__(256) void modes_pk_kernel(const char* __restrict__ qhat, int64_t rowb,
                                                       const double* __restrict__ lam,
                                                       const double2* __restrict__ psi,
                                                       float2* __restrict__ phi,
                                                       int32_t* __restrict__ n_valid, int64_t M, int L,
                                                       int n_modes, double eps) {
  modes_pk_body(qhat, rowb, lam, psi, phi, n_valid, M, L, n_modes, eps, xcd_tile(blockIdx.x, gridDim.x), blockIdx.y);
}

template <typename TC, bool PAIR>
__global__ __launch_bounds__(256) void modes_kernel(const cpx_t<TC>* __restrict__ qhat,
                                                    const double* __restrict__ lam,
                                                    const double2* __restrict__ psi,
                                                    cpx_t<TC>* __restrict__ phi,
                                                    int32_t* __restrict__ n_valid, int64_t M, int L,
                                                    int n_modes, double eps) {
  modes_body<TC, PAIR>(qhat, lam, psi, phi, n_valid, M, M, L, n_modes, eps, xcd_tile(blockIdx.x, gridDim.x), blockIdx.y);
}

template <typename TC, bool PERSIST>
__global__ __launch_bounds__(256) void modes_batch_kernel(const ModesItem* __restrict__ items, int n,
                                                          int units, int* queue) {
  __shared__ int slot;
  for (int b = next_unit(PERSIST ? queue : nullptr, &slot, true); b < units;
       b = next_unit(PERSIST ? queue : nullptr, &slot, false)) {
    const ModesItem& it = items[find_item(items, n, b)];
    const int local = b - it.start;
    if constexpr (sizeof(TC) == 4) {
      if (it.pair) {
        modes_body<TC, true>(static_cast<const cpx_t<TC>*>(it.qhat), it.lam,
                             static_cast<const double2*>(it.psi), static_cast<cpx_t<TC>*>(it.phi),
                             it.n_valid, it.M, it.ldq, it.L, it.n_modes, it.eps, local % it.tiles,
                             local / it.tiles);
        if constexpr (!PERSIST) break;
        continue;
      }
    }
    modes_body<TC, false>(static_cast<const cpx_t<TC>*>(it.qhat), it.lam,
                          static_cast<const double2*>(it.psi), static_cast<cpx_t<TC>*>(it.phi),
                          it.n_valid, it.M, it.ldq, it.L, it.n_modes, it.eps, local % it.tiles,
                          local / it.tiles);
    if constexpr (!PERSIST) break;
  }
}

spod_status launch_modes(const Plan& p, const void* qhat, const double* lam, const void* psi,
                         int n_modes, void* phi, int32_t* n_valid, void* ws, hipStream_t st) {
  (void)ws;
  if (p.nblocks > MODES_MAXL) return fail(SPOD_ERR_UNSUPPORTED, "nblocks > 160");
  const size_t lds = (is_complex128(p) ? 16 : 8) * (size_t)p.nblocks * (size_t)n_modes;
  if (lds > MODES_MAX_TABLE)
    return fail(SPOD_ERR_UNSUPPORTED, "nblocks * n_modes coefficients exceed 64 KiB of LDS");
  if (p.qhat_packed) {
    dim3 grid((unsigned)(((p.M + 3) / 4 + 255) / 256), (unsigned)p.nfreq);
    hipLaunchKernelGGL(modes_pk_kernel, grid, dim3(256), lds, st, static_cast<const char*>(qhat),
                       pk_row_bytes(p.M), lam, static_cast<const double2*>(psi),
                       static_cast<float2*>(phi), n_valid, (int64_t)p.M, (int)p.nblocks, n_modes,
                       1e-6);
  } else if (is_complex128(p)) {
    dim3 grid((unsigned)((p.M + 255) / 256), (unsigned)p.nfreq);
    hipLaunchKernelGGL((modes_kernel<double, false>), grid, dim3(256), lds, st,
                       static_cast<const double2*>(qhat), lam, static_cast<const double2*>(psi),
                       static_cast<double2*>(phi), n_valid, (int64_t)p.M, (int)p.nblocks, n_modes,
                       1e-12);
  } else if (p.modes_mfma) {
    // the complex64 modes on the matrix cores: 512 DOFs per workgroup
    const size_t lds_m = 2 * sizeof(float) * 16 * (size_t)((p.nblocks + 3) & ~3);
    dim3 grid((unsigned)((p.M + 4 * 16 * MODES_TW - 1) / (4 * 16 * MODES_TW)), (unsigned)p.nfreq);
    hipLaunchKernelGGL(modes_mfma_kernel, grid, dim3(256), lds_m, st,
                       static_cast<const float2*>(qhat), lam, static_cast<const double2*>(psi),
                       static_cast<float2*>(phi), n_valid, (int64_t)p.M, (int)p.nblocks, n_modes,
                       1e-6);
  } else if (p.M % 2 == 0 && (uintptr_t)qhat % 16 == 0 && (uintptr_t)phi % 16 == 0) {
    // two degrees of freedom per thread, 16-byte loads and stores
    dim3 grid((unsigned)((p.M / 2 + 255) / 256), (unsigned)p.nfreq);
    hipLaunchKernelGGL((modes_kernel<float, true>), grid, dim3(256), lds, st,
                       static_cast<const float2*>(qhat), lam, static_cast<const double2*>(psi),
                       static_cast<float2*>(phi), n_valid, (int64_t)p.M, (int)p.nblocks, n_modes,
                       1e-6);
  } else {
    dim3 grid((unsigned)((p.M + 255) / 256), (unsigned)p.nfreq);
    hipLaunchKernelGGL((modes_kernel<float, false>), grid, dim3(256), lds, st,
                       static_cast<const float2*>(qhat), lam, static_cast<const double2*>(psi),
                       static_cast<float2*>(phi), n_valid, (int64_t)p.M, (int)p.nblocks, n_modes,
                       1e-6);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPOD_OK : hip_fail(e, "modes_kernel");
}

spod_status launch_modes_group(bool c128, const ModesItem* d_items, int n, int wgs,
                               size_t lds_bytes, int* queue, hipStream_t st) {
  if (queue) {
    const void* k = c128 ? reinterpret_cast<const void*>(&modes_batch_kernel<double, true>)
                         : reinterpret_cast<const void*>(&modes_batch_kernel<float, true>);
    const dim3 grid((unsigned)persistent_grid(k, 256, lds_bytes, wgs));
    if (c128)
      hipLaunchKernelGGL((modes_batch_kernel<double, true>), grid, dim3(256), lds_bytes, st, d_items,
                         n, wgs, queue);
    else
      hipLaunchKernelGGL((modes_batch_kernel<float, true>), grid, dim3(256), lds_bytes, st, d_items,
                         n, wgs, queue);
  } else if (c128) {
    hipLaunchKernelGGL((modes_batch_kernel<double, false>), dim3((unsigned)wgs), dim3(256), lds_bytes,
                       st, d_items, n, wgs, queue);
  } else {
    hipLaunchKernelGGL((modes_batch_kernel<float, false>), dim3((unsigned)wgs), dim3(256), lds_bytes,
                       st, d_items, n, wgs, queue);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPOD_OK : hip_fail(e, "modes_batch_kernel");
}

// Work-queue counters of the persistent grouped launches, zeroed by a kernel
// (not a memset node) so that a captured graph clears them on every replay.
__global__ __launch_bounds__(256) void queue_reset_kernel(int* __restrict__ q, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) q[i] = 0;
}

spod_status launch_queue_reset(int* queue, int n, hipStream_t st) {
  hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(256), 0, st, queue, n);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPOD_OK : hip_fail(e, "queue_reset_kernel");
}

int persistent_grid(const void* kernel, int threads, size_t lds_bytes, int units) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, lds_bytes) != hipSuccess ||
      cus < 1 || per < 1)
    return units;   // fall back to one workgroup per unit (the loop still works)
  const int64_t g = (int64_t)cus * per;
  return (int)(g < units ? g : units);
}

// Rows of a packed buffer [nrow][width] to a destination with row stride
// dpitch (units of V): the modes of one chunk of degrees of freedom into their
// columns of phi [K][n_modes][M], in device memory or in pinned host memory
// mapped for the device (then the stores cross the host link).
template <typename V>
__global__ __launch_bounds__(256) void store_rows_kernel(const V* __restrict__ src,
                                                         V* __restrict__ dst, int64_t width,
                                                         int64_t dpitch, int64_t nrow) {
  const int64_t tiles = (width + 255) / 256;
  for (int64_t t = blockIdx.x; t < tiles * nrow; t += gridDim.x) {
    const int64_t r = t / tiles, i = (t - r * tiles) * 256 + threadIdx.x;
    if (i < width) dst[r * dpitch + i] = src[r * width + i];
  }
}

spod_status launch_store_rows(const void* src, void* dst, size_t width_bytes, size_t dpitch_bytes,
                              int64_t nrow, hipStream_t st) {
  if (width_bytes % 8 != 0 || dpitch_bytes % 8 != 0 || (uintptr_t)src % 8 != 0 ||
      (uintptr_t)dst % 8 != 0 || dpitch_bytes < width_bytes)
    return fail(SPOD_ERR_INVALID_ARG, "store_rows: 8-byte units and alignment required");
  if (nrow <= 0 || width_bytes == 0) return SPOD_OK;
  const bool v16 = width_bytes % 16 == 0 && dpitch_bytes % 16 == 0 && (uintptr_t)src % 16 == 0 &&
                   (uintptr_t)dst % 16 == 0;
  const int64_t unit = v16 ? 16 : 8;
  const int64_t width = (int64_t)width_bytes / unit, dpitch = (int64_t)dpitch_bytes / unit;
  const int64_t total = (width + 255) / 256 * nrow;
  const unsigned grid = (unsigned)std::min<int64_t>(total, 4096);
  if (v16)
    hipLaunchKernelGGL(store_rows_kernel<uint4>, dim3(grid), dim3(256), 0, st,
                       static_cast<const uint4*>(src), static_cast<uint4*>(dst), width, dpitch, nrow);
  else
    hipLaunchKernelGGL(store_rows_kernel<uint2>, dim3(grid), dim3(256), 0, st,
                       static_cast<const uint2*>(src), static_cast<uint2*>(dst), width, dpitch, nrow);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPOD_OK : hip_fail(e, "store_rows_kernel");
}

}  // namespace spod
