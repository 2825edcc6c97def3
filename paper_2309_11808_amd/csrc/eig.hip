// Step 5 of SPOD (eq. (spod-discrete-snapshots); Sec. 3.1 step 5): the
// eigendecomposition of every Hermitian L x L matrix M_k, in FP64.  The paper
// solves these serially and redundantly on every rank; here one workgroup per
// frequency runs a parallel two-sided complex Jacobi method entirely in LDS.
//
// Ordering: round-robin ("circle") pairing of n = L (rounded up to even)
// indices, so each of the n-1 rounds of a sweep rotates n/2 disjoint planes at
// once.  Plane (p, q) with a = A_pp, b = A_qq, c = A_pq = |c| e^{i phi} is
// reduced by
//     J = [[cs, sn e^{i phi}], [-sn e^{-i phi}, cs]],
// where t = sn/cs is the smaller root of t^2 + 2 tau t - 1 = 0,
// tau = (b - a) / (2|c|) (the symmetric Schur decomposition of the real
// 2 x 2 matrix [[a, |c|], [|c|, b]]); afterwards A_pp = a - t|c|,
// A_qq = b + t|c|, A_pq = 0.  A plane is skipped when
// |c| <= tol sqrt(|a b|) (tol = 1e-15) or c == 0; the iteration stops after a
// sweep without rotations.
//
// Output: eigenvalues in descending order (stable on ties), eigenvector j in
// column j with its entry of largest modulus (lowest index on ties) made real
// and positive.  A matrix with a non-finite entry (NaN or Inf data) is not
// iterated: every eigenvalue and eigenvector entry is written as NaN and info
// is SPOD_INFO_NONFINITE.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "internal.h"

namespace spod {

constexpr int EIG_MAXN = 64;      // A and V in LDS up to here
constexpr int EIG_BIGN = 160;     // above: A and V in the workspace (L2 and HBM)

// LDS of one eigenproblem: A and V with rows of n + 1 entries (n = L rounded
// up to even), sized at launch so that small problems share a CU.  The same
// layout, per frequency, in the workspace for L > 64.
__host__ __device__ constexpr size_t eig_lds_bytes(int L) {
  return 2 * sizeof(double2) * (size_t)((L + 1) & ~1) * (size_t)(((L + 1) & ~1) + 1);
}

struct Rot {
  double cs, sn, er, ei, tr, a, b;
  int p, q, on;
};

// MAXN: the largest n of the instantiation; GMEM: A and V live in `work`
// (this frequency's slice of the workspace) instead of LDS.  Within the
// workgroup the barriers order the global accesses as they order the LDS ones.
template <int MAXN, bool GMEM>
__device__ __forceinline__ void jacobi_body(const double2* __restrict__ gram,
                                            double* __restrict__ lam, double2* __restrict__ psi,
                                            int32_t* __restrict__ info, int L, int max_sweeps,
                                            int k, double2* __restrict__ work) {
  extern __shared__ double2 eig_dyn[];
  __shared__ Rot rot[MAXN / 2];
  __shared__ int any_rot;
  __shared__ int nonfinite;
  __shared__ double lsh[MAXN];
  __shared__ int rank_of[MAXN];
  __shared__ double2 phase[MAXN];
  __shared__ int pivot[MAXN];

  const int tid = threadIdx.x;
  const int n = (L + 1) & ~1;             // even, includes a dummy index when L is odd
  const int half = n / 2;
  const int EIG_LD = n + 1;
  double2* A = GMEM ? work + (int64_t)k * 2 * n * EIG_LD : eig_dyn;   // [n][n + 1]
  double2* V = A + n * EIG_LD;                                          // [n][n + 1]
  const double2* G = gram + (int64_t)k * L * L;

  if (tid == 0) nonfinite = 0;
  __syncthreads();
  for (int idx = tid; idx < n * n; idx += blockDim.x) {
    const int i = idx / n, j = idx % n;
    double2 g = make_double2(0.0, 0.0);
    if (i < L && j < L) g = G[i * L + j];
    if (i == j) g.y = 0.0;
    if (!isfinite(g.x) || !isfinite(g.y)) nonfinite = 1;
    A[i * EIG_LD + j] = g;
    V[i * EIG_LD + j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  if (nonfinite) {
    // no rotation is meaningful: report every output as NaN
    const double qnan = __builtin_nan("");
    for (int i = tid; i < L; i += blockDim.x) lam[(int64_t)k * L + i] = qnan;
    for (int idx = tid; idx < L * L; idx += blockDim.x)
      psi[(int64_t)k * L * L + idx] = make_double2(qnan, qnan);
    if (tid == 0 && info) info[k] = SPOD_INFO_NONFINITE;
    return;
  }

  const double tol = 1e-15;
  int sweep = 0;
  bool converged = false;
  for (sweep = 1; sweep <= max_sweeps; ++sweep) {
    if (tid == 0) any_rot = 0;
    __syncthreads();
    for (int round = 0; round < n - 1; ++round) {
      if (tid < half) {
        // circle method: slot 0 fixed, slots 1..n-1 rotate by `round`
        const int s0 = tid, s1 = n - 1 - tid;
        const int x0 = s0 == 0 ? 0 : 1 + (s0 - 1 + round) % (n - 1);
        const int x1 = s1 == 0 ? 0 : 1 + (s1 - 1 + round) % (n - 1);
        const int p = x0 < x1 ? x0 : x1, q = x0 < x1 ? x1 : x0;
        Rot r;
        r.p = p;
        r.q = q;
        r.on = 0;
        if (q < L) {
          const double a = A[p * EIG_LD + p].x, b = A[q * EIG_LD + q].x;
          const double2 c = A[p * EIG_LD + q];
          const double ac = hypot(c.x, c.y);
          if (ac > 0.0 && ac > tol * sqrt(fabs(a * b))) {
            const double tau = (b - a) / (2.0 * ac);
            double t;
            if (fabs(tau) > 1e150) t = 0.5 / tau;
            else t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            const double cs = 1.0 / sqrt(1.0 + t * t);
            r.cs = cs;
            r.sn = t * cs;
            r.er = c.x / ac;
            r.ei = c.y / ac;
            r.tr = t * ac;
            r.a = a;
            r.b = b;
            r.on = 1;
            any_rot = 1;
          }
        }
        rot[tid] = r;
      }
      __syncthreads();
      // A <- J^H A J and V <- V J.  The planes of a round are disjoint, so the
      // 2 x 2 block of A in the rows of plane P and the columns of plane Q
      // depends on itself only: one thread updates it (rows, then columns:
      //   row p' = cs A_p - sn e A_q,        row q' = sn conj(e) A_p + cs A_q,
      //   col p' = cs A_p - sn conj(e) A_q,  col q' = sn e A_p + cs A_q),
      // and a diagonal block (P = Q) is set to its exact result.
      for (int idx = tid; idx < half * half + n * half; idx += blockDim.x) {
        if (idx < half * half) {
          const int P = idx / half, Q = idx % half;
          const Rot& r1 = rot[P];
          const Rot& r2 = rot[Q];
          if (!r1.on && !r2.on) continue;
          double2* x00 = &A[r1.p * EIG_LD + r2.p];
          double2* x01 = &A[r1.p * EIG_LD + r2.q];
          double2* x10 = &A[r1.q * EIG_LD + r2.p];
          double2* x11 = &A[r1.q * EIG_LD + r2.q];
          double2 y00 = *x00, y01 = *x01, y10 = *x10, y11 = *x11;
          if (r1.on) {
            const double2 e = make_double2(r1.er, r1.ei);
            const double2 eq0 = cmul(e, y10), eq1 = cmul(e, y11);      // e * A_q
            const double2 ep0 = cmulc(y00, e), ep1 = cmulc(y01, e);    // conj(e) * A_p
            y00 = make_double2(r1.cs * y00.x - r1.sn * eq0.x, r1.cs * y00.y - r1.sn * eq0.y);
            y01 = make_double2(r1.cs * y01.x - r1.sn * eq1.x, r1.cs * y01.y - r1.sn * eq1.y);
            y10 = make_double2(r1.sn * ep0.x + r1.cs * y10.x, r1.sn * ep0.y + r1.cs * y10.y);
            y11 = make_double2(r1.sn * ep1.x + r1.cs * y11.x, r1.sn * ep1.y + r1.cs * y11.y);
          }
          if (r2.on) {
            const double2 e = make_double2(r2.er, r2.ei);
            const double2 cq0 = cmulc(y01, e), cq1 = cmulc(y11, e);    // conj(e) * A_q
            const double2 ep0 = cmul(e, y00), ep1 = cmul(e, y10);      // e * A_p
            const double2 z00 = make_double2(r2.cs * y00.x - r2.sn * cq0.x, r2.cs * y00.y - r2.sn * cq0.y);
            const double2 z10 = make_double2(r2.cs * y10.x - r2.sn * cq1.x, r2.cs * y10.y - r2.sn * cq1.y);
            y01 = make_double2(r2.sn * ep0.x + r2.cs * y01.x, r2.sn * ep0.y + r2.cs * y01.y);
            y11 = make_double2(r2.sn * ep1.x + r2.cs * y11.x, r2.sn * ep1.y + r2.cs * y11.y);
            y00 = z00;
            y10 = z10;
          }
          if (P == Q) {
            y00 = make_double2(r1.a - r1.tr, 0.0);
            y11 = make_double2(r1.b + r1.tr, 0.0);
            y01 = y10 = make_double2(0.0, 0.0);
          }
          *x00 = y00;
          *x01 = y01;
          *x10 = y10;
          *x11 = y11;
        } else {
          const int rem = idx - half * half;
          const int row = rem / half;
          const Rot& r = rot[rem % half];
          if (!r.on) continue;
          const double2 xp = V[row * EIG_LD + r.p], xq = V[row * EIG_LD + r.q];
          const double2 e = make_double2(r.er, r.ei);
          const double2 ecxq = cmulc(xq, e);        // conj(e) * V_q
          const double2 exp_ = cmul(e, xp);         // e * V_p
          V[row * EIG_LD + r.p] = make_double2(r.cs * xp.x - r.sn * ecxq.x, r.cs * xp.y - r.sn * ecxq.y);
          V[row * EIG_LD + r.q] = make_double2(r.sn * exp_.x + r.cs * xq.x, r.sn * exp_.y + r.cs * xq.y);
        }
      }
      __syncthreads();
    }
    if (!any_rot) {
      converged = true;
      break;
    }
    __syncthreads();
  }

  // eigenvalues, ranks (descending, stable), phases.  The order is total:
  // j goes before i when lj > li, or when they are equal (or both NaN) and
  // j < i, or when only li is NaN; so the ranks are a permutation even if an
  // overflow produced a NaN.
  for (int i = tid; i < L; i += blockDim.x) lsh[i] = A[i * EIG_LD + i].x;
  __syncthreads();
  for (int i = tid; i < L; i += blockDim.x) {
    const double li = lsh[i];
    const bool ni = isnan(li);
    int r = 0;
    for (int j = 0; j < L; ++j) {
      const double lj = lsh[j];
      const bool nj = isnan(lj);
      const bool before = (ni || nj) ? ((ni && !nj) || (ni && nj && j < i))
                                     : ((lj > li) || (lj == li && j < i));
      r += before;
    }
    rank_of[i] = r;
    int piv = 0;
    double best = -1.0;
    for (int row = 0; row < L; ++row) {
      const double2 v = V[row * EIG_LD + i];
      const double m2 = v.x * v.x + v.y * v.y;
      if (m2 > best) {
        best = m2;
        piv = row;
      }
    }
    const double2 v = V[piv * EIG_LD + i];
    const double mag = hypot(v.x, v.y);
    phase[i] = mag > 0.0 ? make_double2(v.x / mag, -v.y / mag) : make_double2(1.0, 0.0);
    pivot[i] = piv;
  }
  __syncthreads();
  for (int i = tid; i < L; i += blockDim.x) lam[(int64_t)k * L + rank_of[i]] = lsh[i];
  for (int idx = tid; idx < L * L; idx += blockDim.x) {
    const int row = idx / L, i = idx % L;
    const double2 v = V[row * EIG_LD + i];
    // the pivot entry is written as exactly |v| (real, positive)
    psi[((int64_t)k * L + row) * L + rank_of[i]] =
        row == pivot[i] ? make_double2(hypot(v.x, v.y), 0.0) : cmul(v, phase[i]);
  }
  if (tid == 0 && info) info[k] = converged ? sweep : -(sweep - 1);
}

// NT threads per eigenproblem.  A round updates n/2 x n/2 blocks of A and
// n x n/2 pairs of V between two barriers (3072 items at n = 64), so the large
// problems take 1024 threads: the round's latency is spread over 16
// wavefronts instead of 4 (one problem fills a CU's LDS either way).  Every
// item is computed by one thread with the same arithmetic whatever NT is.
template <int NT>
__global__ __launch_bounds__(NT) void jacobi_kernel(const double2* __restrict__ gram,
                                                    double* __restrict__ lam,
                                                    double2* __restrict__ psi,
                                                    int32_t* __restrict__ info, int L,
                                                    int max_sweeps) {
  jacobi_body<EIG_MAXN, false>(gram, lam, psi, info, L, max_sweeps, blockIdx.x, nullptr);
}

// L > 64: A and V of frequency k in work [K][2][n][n + 1] complex.
__global__ __launch_bounds__(1024) void jacobi_big_kernel(const double2* __restrict__ gram,
                                                          double* __restrict__ lam,
                                                          double2* __restrict__ psi,
                                                          int32_t* __restrict__ info, int L,
                                                          int max_sweeps, double2* __restrict__ work) {
  jacobi_body<EIG_BIGN, true>(gram, lam, psi, info, L, max_sweeps, blockIdx.x, work);
}

template <int NT, bool PERSIST>
__global__ __launch_bounds__(NT) void jacobi_batch_kernel(const EigItem* __restrict__ items, int n,
                                                          int max_sweeps, int units, int* queue) {
  __shared__ int slot;
  for (int b = next_unit(PERSIST ? queue : nullptr, &slot, true); b < units;
       b = next_unit(PERSIST ? queue : nullptr, &slot, false)) {
    const EigItem& it = items[find_item(items, n, b)];
    jacobi_body<EIG_MAXN, false>(static_cast<const double2*>(it.gram), it.lam,
                                 static_cast<double2*>(it.psi), it.info, it.L, max_sweeps,
                                 b - it.start, nullptr);
    if constexpr (!PERSIST) break;
  }
}

constexpr int EIG_SMALL_NT = 256, EIG_LARGE_NT = 1024;
// 1024 threads only above L = 32: at L = 31 they were measured slower (0.86
// against 0.70 ms for 257 problems), the round's 768 items being too few.
constexpr int eig_threads(int L) { return L > 32 ? EIG_LARGE_NT : EIG_SMALL_NT; }

// The attribute is set once per process (std::call_once: plans may be used
// from several host threads).
static hipError_t eig_attr() {
  static std::once_flag once;
  static hipError_t result = hipSuccess;
  std::call_once(once, [] {
  const void* fns[] = {reinterpret_cast<const void*>(&jacobi_kernel<EIG_SMALL_NT>),
                       reinterpret_cast<const void*>(&jacobi_kernel<EIG_LARGE_NT>),
                       reinterpret_cast<const void*>(&jacobi_batch_kernel<EIG_SMALL_NT, false>),
                       reinterpret_cast<const void*>(&jacobi_batch_kernel<EIG_LARGE_NT, false>),
                       reinterpret_cast<const void*>(&jacobi_batch_kernel<EIG_SMALL_NT, true>),
                       reinterpret_cast<const void*>(&jacobi_batch_kernel<EIG_LARGE_NT, true>)};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)eig_lds_bytes(EIG_MAXN));
    if (e != hipSuccess) {
      result = e;
      return;
    }
  }
  });
  return result;
}

size_t eig_workspace(const Plan& p) {
  return p.nblocks > EIG_MAXN ? (size_t)p.nfreq * eig_lds_bytes((int)p.nblocks) : 0;
}

spod_status launch_eig(const Plan& p, const void* gram, double* lam, void* psi, int32_t* info,
                       void* ws, hipStream_t st) {
  if (p.nblocks > EIG_BIGN) return fail(SPOD_ERR_UNSUPPORTED, "nblocks > 160");
  const int L = (int)p.nblocks;
  if (L > EIG_MAXN) {
    hipLaunchKernelGGL(jacobi_big_kernel, dim3((unsigned)p.nfreq), dim3(1024), 0, st,
                       static_cast<const double2*>(gram), lam, static_cast<double2*>(psi), info, L,
                       p.max_sweeps, static_cast<double2*>(ws));
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPOD_OK : hip_fail(e, "jacobi_big_kernel");
  }
  hipError_t ea = eig_attr();
  if (ea != hipSuccess) return hip_fail(ea, "hipFuncSetAttribute");
  if (eig_threads(L) == EIG_LARGE_NT)
    hipLaunchKernelGGL(jacobi_kernel<EIG_LARGE_NT>, dim3((unsigned)p.nfreq), dim3(EIG_LARGE_NT),
                       eig_lds_bytes(L), st, static_cast<const double2*>(gram), lam,
                       static_cast<double2*>(psi), info, L, p.max_sweeps);
  else
    hipLaunchKernelGGL(jacobi_kernel<EIG_SMALL_NT>, dim3((unsigned)p.nfreq), dim3(EIG_SMALL_NT),
                       eig_lds_bytes(L), st, static_cast<const double2*>(gram), lam,
                       static_cast<double2*>(psi), info, L, p.max_sweeps);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPOD_OK : hip_fail(e, "jacobi_kernel");
}

spod_status launch_eig_group(const EigItem* d_items, int n, int wgs, int max_sweeps, int lmax,
                             int threads, int* queue, hipStream_t st) {
  hipError_t ea = eig_attr();
  if (ea != hipSuccess) return hip_fail(ea, "hipFuncSetAttribute");
  const size_t lds_bytes = eig_lds_bytes(lmax);
  const int nt = threads ? threads : eig_threads(lmax);
  if (nt != EIG_LARGE_NT && nt != EIG_SMALL_NT) return fail(SPOD_ERR_INVALID_ARG, "eigensolver threads");
#define SPOD_EIG_GROUP(NTH)                                                                      \
  if (queue) {                                                                                   \
    const void* k = reinterpret_cast<const void*>(&jacobi_batch_kernel<NTH, true>);              \
    hipLaunchKernelGGL((jacobi_batch_kernel<NTH, true>),                                         \
                       dim3((unsigned)persistent_grid(k, NTH, lds_bytes, wgs)), dim3(NTH),       \
                       lds_bytes, st, d_items, n, max_sweeps, wgs, queue);                       \
  } else {                                                                                       \
    hipLaunchKernelGGL((jacobi_batch_kernel<NTH, false>), dim3((unsigned)wgs), dim3(NTH),        \
                       lds_bytes, st, d_items, n, max_sweeps, wgs, queue);                       \
  }
  if (nt == EIG_LARGE_NT) {
    SPOD_EIG_GROUP(EIG_LARGE_NT)
  } else {
    SPOD_EIG_GROUP(EIG_SMALL_NT)
  }
#undef SPOD_EIG_GROUP
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPOD_OK : hip_fail(e, "jacobi_batch_kernel");
}

}  // namespace spod
