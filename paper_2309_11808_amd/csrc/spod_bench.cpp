// spod_bench: a plain C-ABI caller of libspod, with nothing else in the
// process (no Python, no framework), for hardware-counter runs.
//
//   spod_bench [nspace nvar nt nfft noverlap reps precision path qhat_format]
//   defaults:   524288  2   8192 512  256      3    2 (bf16x4)  0    0 (complex)
//
// Fills q [M][nt] float32 on the device with hashed values in [-1, 1).
// path 0: runs spod_blocks_fft `reps` times, then copies 1 GiB device to
//         device three times with its own copy kernel (a dispatch of known
//         traffic: 1 GiB read and 1 GiB written).
// path 1: runs the whole forward path (blocks_fft, csd, eig, modes with 5
//         modes) `reps` times with the plan of `precision`, then with the
//         FP64 plan.
// path 2: out-of-core: Q copied to pinned host memory, then spod_ooc_forward
//         with chunks of 32768 rows, `reps` times with no chunk resident and
//         `reps` times with every chunk resident (plan of `precision`, 5
//         modes to pinned host memory).
// path 3: HBM reference rates of streaming kernels with 16-byte accesses over
//         16 GiB in / 32 GiB out: write only, read only, copy 1:1, and
//         read 1 : write 2 (the transform's mix: q in, twice the bytes out)
//         as two output streams; a sweep over grids (2048-65536 workgroups),
//         accesses in flight per thread (1, 4, 8), plain or non-temporal
//         accesses, and grid-stride or one contiguous range per workgroup;
//         the best of three launches per configuration, then the best
//         configuration per mix.
// Prints the event timings.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "spod.h"

#define CHECK_HIP(x)                                                              \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) {                                                       \
      std::fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));         \
      return 1;                                                                   \
    }                                                                             \
  } while (0)

#define CHECK_SPOD(x)                                                             \
  do {                                                                            \
    spod_status s_ = (x);                                                         \
    if (s_ != SPOD_OK) {                                                          \
      std::fprintf(stderr, "%s failed: %s\n", #x, spod_last_error());             \
      return 1;                                                                   \
    }                                                                             \
  } while (0)

__global__ void fill_kernel(float* __restrict__ q, int64_t n, uint32_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t h = (uint32_t)i * 2654435761u ^ (uint32_t)(i >> 32) * 40503u ^ seed;
    h ^= h >> 16;
    h *= 0x7feb352du;
    h ^= h >> 15;
    h *= 0x846ca68bu;
    h ^= h >> 16;
    q[i] = (float)(h >> 8) * (1.0f / 8388608.0f) - 1.0f;
  }
}

__global__ void copy_kernel(const float4* __restrict__ src, float4* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// Streaming kernels for the HBM reference rates.  KIND 0: write 2n float4;
// 1: read n; 2: copy n; 3: read n, write 2n as two streams o[i] and o[n + i]
// (the transform's mix).  Each thread keeps U 16-byte accesses in flight per
// stream; NT: non-temporal loads and stores; BLOCKED: workgroup b streams one
// contiguous range (else a grid-stride loop over the whole array).
typedef float v4f __attribute__((ext_vector_type(4)));

template <int KIND, int U, bool NT, bool BLOCKED>
__global__ __launch_bounds__(256) void stream_kernel(const v4f* __restrict__ a,
                                                     v4f* __restrict__ o, int64_t n,
                                                     float* __restrict__ sink) {
  const int64_t N = KIND == 0 ? 2 * n : n;              // units of the index space
  const int64_t span = (int64_t)U * blockDim.x;
  int64_t b0, b1, step;
  if (BLOCKED) {
    const int64_t per = (N + gridDim.x - 1) / gridDim.x;
    const int64_t chunk = (per + span - 1) / span * span;
    b0 = (int64_t)blockIdx.x * chunk;
    b1 = b0 + chunk < N ? b0 + chunk : N;
    step = span;
  } else {
    b0 = (int64_t)blockIdx.x * span;
    b1 = N;
    step = (int64_t)gridDim.x * span;
  }
  float s = 0.f;
  for (int64_t base = b0 + threadIdx.x; base - threadIdx.x < b1; base += step) {
    v4f v[U];
    if (KIND != 0) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = base + (int64_t)u * blockDim.x;
        if (i < b1) v[u] = NT ? __builtin_nontemporal_load(a + i) : a[i];
        else v[u] = v4f{0.f, 0.f, 0.f, 0.f};
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = v4f{(float)(base + u), 1.f, 2.f, 3.f};
    }
    if (KIND == 1) {
#pragma unroll
      for (int u = 0; u < U; ++u) s += v[u].x + v[u].y + v[u].z + v[u].w;
      continue;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + (int64_t)u * blockDim.x;
      if (i >= b1) continue;
      if (NT) __builtin_nontemporal_store(v[u], o + i);
      else o[i] = v[u];
      if (KIND == 3) {
        const v4f w = v4f{v[u].y, v[u].x, v[u].w, v[u].z};
        if (NT) __builtin_nontemporal_store(w, o + n + i);
        else o[n + i] = w;
      }
    }
  }
  if (KIND == 1 && s == 123.456f) sink[0] = s;   // keeps the loads
}

template <int KIND, int U, bool NT, bool BLOCKED>
static void launch_stream(int grid, const float4* a, float4* o, int64_t n, float* sink) {
  hipLaunchKernelGGL((stream_kernel<KIND, U, NT, BLOCKED>), dim3(grid), dim3(256), 0, 0,
                     reinterpret_cast<const v4f*>(a), reinterpret_cast<v4f*>(o), n, sink);
}

template <int KIND>
static void launch_stream_cfg(int u, bool nt, bool blocked, int grid, const float4* a, float4* o,
                              int64_t n, float* sink) {
#define SPOD_STREAM(U_)                                                                    \
  if (u == U_) {                                                                           \
    if (nt && blocked) launch_stream<KIND, U_, true, true>(grid, a, o, n, sink);           \
    if (nt && !blocked) launch_stream<KIND, U_, true, false>(grid, a, o, n, sink);         \
    if (!nt && blocked) launch_stream<KIND, U_, false, true>(grid, a, o, n, sink);         \
    if (!nt && !blocked) launch_stream<KIND, U_, false, false>(grid, a, o, n, sink);       \
  }
  SPOD_STREAM(1)
  SPOD_STREAM(4)
  SPOD_STREAM(8)
#undef SPOD_STREAM
}

static int run_rates() {
  const int64_t n = (int64_t(16) << 30) / 16;   // 16 GiB of float4 in
  float4 *a = nullptr, *o = nullptr;
  float* sink = nullptr;
  CHECK_HIP(hipMalloc(&a, 16 * (size_t)n));
  CHECK_HIP(hipMalloc(&o, 32 * (size_t)n));
  CHECK_HIP(hipMalloc(&sink, 64));
  hipLaunchKernelGGL(fill_kernel, dim3(8192), dim3(256), 0, 0, reinterpret_cast<float*>(a), 4 * n,
                     7u);
  CHECK_HIP(hipGetLastError());
  hipEvent_t e0, e1;
  CHECK_HIP(hipEventCreate(&e0));
  CHECK_HIP(hipEventCreate(&e1));
  const char* names[] = {"write only", "read only", "copy 1:1", "read 1 : write 2"};
  const double bytes[] = {32.0 * n, 16.0 * n, 32.0 * n, 48.0 * n};
  double best[4] = {0, 0, 0, 0};
  char best_cfg[4][96] = {};
  for (int k = 0; k < 4; ++k) {
    for (int grid : {2048, 16384, 65536}) {
      for (int u : {1, 4, 8}) {
        for (int nt = 0; nt < 2; ++nt) {
          for (int blocked = 0; blocked < 2; ++blocked) {
            float ms = 0.0f, best_ms = 1e30f;
            for (int r = 0; r < 3; ++r) {
              CHECK_HIP(hipEventRecord(e0, 0));
              if (k == 0) launch_stream_cfg<0>(u, nt, blocked, grid, a, o, n, sink);
              if (k == 1) launch_stream_cfg<1>(u, nt, blocked, grid, a, o, n, sink);
              if (k == 2) launch_stream_cfg<2>(u, nt, blocked, grid, a, o, n, sink);
              if (k == 3) launch_stream_cfg<3>(u, nt, blocked, grid, a, o, n, sink);
              CHECK_HIP(hipGetLastError());
              CHECK_HIP(hipEventRecord(e1, 0));
              CHECK_HIP(hipEventSynchronize(e1));
              CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
              if (ms < best_ms) best_ms = ms;
            }
            const double tbs = bytes[k] / (best_ms * 1e-3) / 1e12;
            std::printf("%-18s grid %6d U %d %-9s %-11s %8.3f ms %6.2f TB/s\n", names[k], grid, u,
                        nt ? "nt" : "plain", blocked ? "blocked" : "gridstride", best_ms, tbs);
            std::fflush(stdout);
            if (tbs > best[k]) {
              best[k] = tbs;
              std::snprintf(best_cfg[k], sizeof(best_cfg[k]), "grid %d U %d %s %s", grid, u,
                            nt ? "nt" : "plain", blocked ? "blocked" : "gridstride");
            }
          }
        }
      }
    }
  }
  for (int k = 0; k < 4; ++k)
    std::printf("best %-18s %6.2f TB/s  (%s)\n", names[k], best[k], best_cfg[k]);
  void* bufs[] = {a, o, sink};
  for (void* b : bufs) CHECK_HIP(hipFree(b));
  return 0;
}

static int run_path(int64_t nspace, int64_t nvar, int64_t nt, int64_t nfft, int64_t nov,
                    int64_t reps, spod_precision prec, const float* q, int64_t fmt) {
  const int64_t M = nspace * nvar, n_modes = 5;
  spod_plan plan = nullptr;
  CHECK_SPOD(spod_plan_create(nspace, nvar, nt, nfft, nov, nullptr, nullptr, &plan));
  CHECK_SPOD(spod_plan_set_precision(plan, prec));
  CHECK_SPOD(spod_plan_set_option(plan, SPOD_OPT_QHAT_FORMAT, fmt));
  int64_t L = 0, K = 0;
  size_t wsb = 0, qhb = 0;
  CHECK_SPOD(spod_plan_query(plan, &L, &K, &wsb));
  CHECK_SPOD(spod_plan_qhat_bytes(plan, &qhb));
  const size_t csz = prec == SPOD_PREC_FP64 ? 16 : 8;
  void *qhat = nullptr, *gram = nullptr, *psi = nullptr, *phi = nullptr, *ws = nullptr;
  double *mean = nullptr, *lam = nullptr;
  int32_t *info = nullptr, *nval = nullptr;
  CHECK_HIP(hipMalloc(&qhat, qhb));
  CHECK_HIP(hipMalloc(&phi, csz * (size_t)(K * n_modes * M)));
  CHECK_HIP(hipMalloc(&gram, 16 * (size_t)(K * L * L)));
  CHECK_HIP(hipMalloc(&psi, 16 * (size_t)(K * L * L)));
  CHECK_HIP(hipMalloc(&lam, 8 * (size_t)(K * L)));
  CHECK_HIP(hipMalloc(&mean, 8 * (size_t)M));
  CHECK_HIP(hipMalloc(&info, 4 * (size_t)K));
  CHECK_HIP(hipMalloc(&nval, 4 * (size_t)K));
  CHECK_HIP(hipMalloc(&ws, wsb > 0 ? wsb : 256));
  hipEvent_t e[5];
  for (auto& x : e) CHECK_HIP(hipEventCreate(&x));
  for (int64_t r = 0; r < reps; ++r) {
    CHECK_HIP(hipEventRecord(e[0], 0));
    CHECK_SPOD(spod_blocks_fft(plan, q, SPOD_F32, qhat, mean, ws, wsb, nullptr));
    CHECK_HIP(hipEventRecord(e[1], 0));
    CHECK_SPOD(spod_csd(plan, qhat, gram, ws, wsb, nullptr));
    CHECK_HIP(hipEventRecord(e[2], 0));
    CHECK_SPOD(spod_eig(plan, gram, lam, psi, info, ws, wsb, nullptr));
    CHECK_HIP(hipEventRecord(e[3], 0));
    CHECK_SPOD(spod_modes(plan, qhat, lam, psi, n_modes, phi, nval, ws, wsb, nullptr));
    CHECK_HIP(hipEventRecord(e[4], 0));
    CHECK_HIP(hipEventSynchronize(e[4]));
    float ms[4];
    for (int i = 0; i < 4; ++i) CHECK_HIP(hipEventElapsedTime(&ms[i], e[i], e[i + 1]));
    static const char* names[] = {"fp64", "fp32", "bf16x4", "fp16x4"};
    std::printf("%s path %lld: blocks_fft %.3f ms, csd %.3f ms, eig %.3f ms, modes %.3f ms\n",
                names[prec & 3], (long long)r, ms[0], ms[1], ms[2], ms[3]);
    std::fflush(stdout);
  }
  for (auto& x : e) CHECK_HIP(hipEventDestroy(x));
  spod_plan_destroy(plan);
  void* bufs[] = {qhat, gram, psi, phi, ws, mean, lam, info, nval};
  for (void* b : bufs) CHECK_HIP(hipFree(b));
  return 0;
}

static int run_ooc(int64_t nspace, int64_t nvar, int64_t nt, int64_t nfft, int64_t nov,
                   int64_t reps, spod_precision prec) {
  const int64_t M = nspace * nvar, n_modes = 5, rows = 32768;
  const size_t qbytes = sizeof(float) * (size_t)M * (size_t)nt;
  float* qd = nullptr;
  float* qh = nullptr;
  CHECK_HIP(hipMalloc(&qd, qbytes));
  hipLaunchKernelGGL(fill_kernel, dim3(8192), dim3(256), 0, 0, qd, (int64_t)(qbytes / 4), 12345u);
  CHECK_HIP(hipGetLastError());
  CHECK_HIP(hipHostMalloc(reinterpret_cast<void**>(&qh), qbytes, hipHostMallocDefault));
  CHECK_HIP(hipMemcpy(qh, qd, qbytes, hipMemcpyDeviceToHost));
  CHECK_HIP(hipFree(qd));
  spod_plan plan = nullptr;
  CHECK_SPOD(spod_plan_create(nspace, nvar, nt, nfft, nov, nullptr, nullptr, &plan));
  CHECK_SPOD(spod_plan_set_precision(plan, prec));
  int64_t L = 0, K = 0;
  CHECK_SPOD(spod_plan_query(plan, &L, &K, nullptr));
  const size_t csz = prec == SPOD_PREC_FP64 ? 16 : 8;
  void *phi = nullptr, *psi = nullptr;
  double* lam = nullptr;
  int32_t *info = nullptr, *nval = nullptr;
  std::vector<double> mean((size_t)M);
  CHECK_HIP(hipHostMalloc(&phi, csz * (size_t)(K * n_modes * M), hipHostMallocDefault));
  CHECK_HIP(hipMalloc(&psi, 16 * (size_t)(K * L * L)));
  CHECK_HIP(hipMalloc(&lam, 8 * (size_t)(K * L)));
  CHECK_HIP(hipMalloc(&info, 4 * (size_t)K));
  CHECK_HIP(hipMalloc(&nval, 4 * (size_t)K));
  for (int64_t resident : {int64_t(0), int64_t(1) << 30}) {
    spod_ooc o = nullptr;
    CHECK_SPOD(spod_ooc_create(plan, SPOD_F32, rows, n_modes, resident, &o));
    int64_t nchunks = 0, nres = 0;
    CHECK_SPOD(spod_ooc_query(o, nullptr, &nchunks, &nres, nullptr, nullptr));
    for (int64_t r = 0; r < reps; ++r) {
      auto t0 = std::chrono::steady_clock::now();
      CHECK_SPOD(spod_ooc_forward(o, qh, nullptr, nullptr, mean.data(), lam, psi, info, phi, nval,
                                  nullptr));
      const double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      const double link = (double)qbytes * (double)(2 * nchunks - nres) / (double)nchunks;
      std::printf("out-of-core %lld/%lld chunks resident, %lld: %.1f ms, Q %.2f GB/s, link in %.2f GB/s\n",
                  (long long)nres, (long long)nchunks, (long long)r, s * 1e3, qbytes / s / 1e9,
                  link / s / 1e9);
      std::fflush(stdout);
    }
    spod_ooc_destroy(o);
  }
  spod_plan_destroy(plan);
  CHECK_HIP(hipHostFree(qh));
  CHECK_HIP(hipHostFree(phi));
  void* bufs[] = {psi, lam, info, nval};
  for (void* b : bufs) CHECK_HIP(hipFree(b));
  return 0;
}

int main(int argc, char** argv) {
  int64_t nspace = 524288, nvar = 2, nt = 8192, nfft = 512, nov = 256, reps = 3, prec = 2, path = 0,
          fmt = 0;
  int64_t* args[] = {&nspace, &nvar, &nt, &nfft, &nov, &reps, &prec, &path, &fmt};
  for (int i = 1; i < argc && i <= 9; ++i) *args[i - 1] = std::atoll(argv[i]);
  const int64_t M = nspace * nvar;
  if (path == 3) {
    if (run_rates()) return 1;
    std::printf("done\n");
    return 0;
  }
  if (path == 2) {
    if (run_ooc(nspace, nvar, nt, nfft, nov, reps, (spod_precision)prec)) return 1;
    std::printf("done\n");
    return 0;
  }
  if (path == 1) {
    float* q = nullptr;
    const size_t qbytes = sizeof(float) * (size_t)M * (size_t)nt;
    CHECK_HIP(hipMalloc(&q, qbytes));
    hipLaunchKernelGGL(fill_kernel, dim3(8192), dim3(256), 0, 0, q, (int64_t)(qbytes / 4), 12345u);
    CHECK_HIP(hipGetLastError());
    CHECK_HIP(hipDeviceSynchronize());
    if (run_path(nspace, nvar, nt, nfft, nov, reps, (spod_precision)prec, q, fmt)) return 1;
    if (run_path(nspace, nvar, nt, nfft, nov, reps, SPOD_PREC_FP64, q, 0)) return 1;
    CHECK_HIP(hipFree(q));
    std::printf("done\n");
    return 0;
  }

  spod_plan plan = nullptr;
  CHECK_SPOD(spod_plan_create(nspace, nvar, nt, nfft, nov, nullptr, nullptr, &plan));
  CHECK_SPOD(spod_plan_set_precision(plan, (spod_precision)prec));
  CHECK_SPOD(spod_plan_set_option(plan, SPOD_OPT_QHAT_FORMAT, fmt));
  int64_t L = 0, K = 0;
  size_t wsb = 0, hbytes = 0;
  CHECK_SPOD(spod_plan_query(plan, &L, &K, &wsb));
  CHECK_SPOD(spod_plan_qhat_bytes(plan, &hbytes));
  const size_t qbytes = sizeof(float) * (size_t)M * (size_t)nt;
  std::printf("M=%lld nt=%lld nfft=%lld L=%lld K=%lld q=%.3f GB qhat=%.3f GB\n", (long long)M,
              (long long)nt, (long long)nfft, (long long)L, (long long)K, qbytes / 1e9, hbytes / 1e9);
  std::fflush(stdout);

  float* q = nullptr;
  void* qhat = nullptr;
  double* mean = nullptr;
  void* ws = nullptr;
  CHECK_HIP(hipMalloc(&q, qbytes));
  CHECK_HIP(hipMalloc(&qhat, hbytes));
  CHECK_HIP(hipMalloc(&mean, sizeof(double) * (size_t)M));
  CHECK_HIP(hipMalloc(&ws, wsb > 0 ? wsb : 256));
  hipLaunchKernelGGL(fill_kernel, dim3(8192), dim3(256), 0, 0, q, (int64_t)(qbytes / 4), 12345u);
  CHECK_HIP(hipGetLastError());
  CHECK_HIP(hipDeviceSynchronize());

  hipEvent_t e0, e1;
  CHECK_HIP(hipEventCreate(&e0));
  CHECK_HIP(hipEventCreate(&e1));
  for (int64_t r = 0; r < reps; ++r) {
    CHECK_HIP(hipEventRecord(e0, 0));
    CHECK_SPOD(spod_blocks_fft(plan, q, SPOD_F32, qhat, mean, ws, wsb, nullptr));
    CHECK_HIP(hipEventRecord(e1, 0));
    CHECK_HIP(hipEventSynchronize(e1));
    float ms = 0.0f;
    CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
    std::printf("spod_blocks_fft %lld: %.3f ms, %.3f TB/s of algorithmic bytes\n", (long long)r, ms,
                (qbytes + hbytes) / (ms * 1e-3) / 1e12);
    std::fflush(stdout);
  }
  const size_t cbytes = size_t(1) << 30;
  if (qbytes >= cbytes && hbytes >= cbytes) {
    for (int r = 0; r < 3; ++r) {
      CHECK_HIP(hipEventRecord(e0, 0));
      hipLaunchKernelGGL(copy_kernel, dim3(8192), dim3(256), 0, 0, reinterpret_cast<const float4*>(q),
                         reinterpret_cast<float4*>(qhat), (int64_t)(cbytes / 16));
      CHECK_HIP(hipGetLastError());
      CHECK_HIP(hipEventRecord(e1, 0));
      CHECK_HIP(hipEventSynchronize(e1));
      float ms = 0.0f;
      CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
      std::printf("copy 1 GiB %d: %.3f ms, %.3f TB/s (read + write)\n", r, ms,
                  2.0 * cbytes / (ms * 1e-3) / 1e12);
      std::fflush(stdout);
    }
  }
  CHECK_HIP(hipDeviceSynchronize());
  spod_plan_destroy(plan);
  CHECK_HIP(hipFree(q));
  CHECK_HIP(hipFree(qhat));
  CHECK_HIP(hipFree(mean));
  CHECK_HIP(hipFree(ws));
  std::printf("done\n");
  return 0;
}
