// SPOD modes (eq. (spod-discrete-snapshots)): Phi_k = Qhat_k Psi_k Lambda_k^{-1/2},
// for the leading n_modes eigenpairs of every frequency.
//
// Per frequency this is an (M x L) by (L x n_modes) product with L ~ 31 and
// n_modes ~ 5: far too thin for matrix cores, and bound by streaming qhat
// from HBM.  Each thread owns one degree of freedom, reads its L coefficients
// (coalesced across the wavefront) and accumulates up to 8 modes in registers;
// the L x n_modes coefficients psi / sqrt(lambda) sit in LDS.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace spod {

constexpr int MODES_MAXL = 64;
constexpr int MODES_GROUP = 8;

template <typename TC>
__device__ __forceinline__ void modes_body(const cpx_t<TC>* __restrict__ qhat,
                                           const double* __restrict__ lam,
                                           const double2* __restrict__ psi,
                                           cpx_t<TC>* __restrict__ phi,
                                           int32_t* __restrict__ n_valid, int64_t M, int L,
                                           int n_modes, double eps, int64_t bx, int k) {
  using C = cpx_t<TC>;
  extern __shared__ char modes_lds[];
  C* coef = reinterpret_cast<C*>(modes_lds);   // [L][n_modes]
  const int tid = threadIdx.x;
  const double* lk = lam + (int64_t)k * L;
  const double l0 = lk[0];
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
  const int64_t m = bx * blockDim.x + tid;
  if (m >= M) return;
  const C* src = qhat + (int64_t)k * L * M + m;
  C* dst = phi + (int64_t)k * n_modes * M + m;
  for (int j0 = 0; j0 < n_modes; j0 += MODES_GROUP) {
    C acc[MODES_GROUP];
#pragma unroll
    for (int j = 0; j < MODES_GROUP; ++j) acc[j] = C{0, 0};
    for (int l = 0; l < L; ++l) {
      const C x = src[(int64_t)l * M];
      const C* cl = coef + l * n_modes + j0;
#pragma unroll
      for (int j = 0; j < MODES_GROUP; ++j) {
        if (j0 + j < n_modes) {
          const C c = cl[j];
          acc[j].x += x.x * c.x - x.y * c.y;
          acc[j].y += x.x * c.y + x.y * c.x;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < MODES_GROUP; ++j)
      if (j0 + j < n_modes) dst[(int64_t)(j0 + j) * M] = acc[j];
  }
}

template <typename TC>
__global__ __launch_bounds__(256) void modes_kernel(const cpx_t<TC>* __restrict__ qhat,
                                                    const double* __restrict__ lam,
                                                    const double2* __restrict__ psi,
                                                    cpx_t<TC>* __restrict__ phi,
                                                    int32_t* __restrict__ n_valid, int64_t M, int L,
                                                    int n_modes, double eps) {
  modes_body<TC>(qhat, lam, psi, phi, n_valid, M, L, n_modes, eps, blockIdx.x, blockIdx.y);
}

template <typename TC>
__global__ __launch_bounds__(256) void modes_batch_kernel(const ModesItem* __restrict__ items, int n) {
  const ModesItem& it = items[find_item(items, n, (int)blockIdx.x)];
  const int local = (int)blockIdx.x - it.start;
  modes_body<TC>(static_cast<const cpx_t<TC>*>(it.qhat), it.lam, static_cast<const double2*>(it.psi),
                 static_cast<cpx_t<TC>*>(it.phi), it.n_valid, it.M, it.L, it.n_modes, it.eps,
                 local % it.tiles, local / it.tiles);
}

spod_status launch_modes(const Plan& p, const void* qhat, const double* lam, const void* psi,
                         int n_modes, void* phi, int32_t* n_valid, void* ws, hipStream_t st) {
  (void)ws;
  if (p.nblocks > MODES_MAXL) return fail(SPOD_ERR_UNSUPPORTED, "nblocks > 64");
  dim3 grid((unsigned)((p.M + 255) / 256), (unsigned)p.nfreq);
  const size_t lds = (is_complex128(p) ? 16 : 8) * (size_t)p.nblocks * (size_t)n_modes;
  if (is_complex128(p))
    hipLaunchKernelGGL(modes_kernel<double>, grid, dim3(256), lds, st,
                       static_cast<const double2*>(qhat), lam, static_cast<const double2*>(psi),
                       static_cast<double2*>(phi), n_valid, (int64_t)p.M, (int)p.nblocks, n_modes,
                       1e-12);
  else
    hipLaunchKernelGGL(modes_kernel<float>, grid, dim3(256), lds, st,
                       static_cast<const float2*>(qhat), lam, static_cast<const double2*>(psi),
                       static_cast<float2*>(phi), n_valid, (int64_t)p.M, (int)p.nblocks, n_modes,
                       1e-6);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPOD_OK : hip_fail(e, "modes_kernel");
}

spod_status launch_modes_group(bool c128, const ModesItem* d_items, int n, int wgs,
                               size_t lds_bytes, hipStream_t st) {
  if (c128)
    hipLaunchKernelGGL(modes_batch_kernel<double>, dim3((unsigned)wgs), dim3(256), lds_bytes, st,
                       d_items, n);
  else
    hipLaunchKernelGGL(modes_batch_kernel<float>, dim3((unsigned)wgs), dim3(256), lds_bytes, st,
                       d_items, n);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPOD_OK : hip_fail(e, "modes_batch_kernel");
}

}  // namespace spod
