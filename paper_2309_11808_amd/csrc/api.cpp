// extern "C" entry points of libspod: validation, plan lifetime, dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

namespace spod {

static thread_local std::string g_last_error;

// The status is returned even when the message cannot be stored (no memory
// for the string): nothing here throws.
spod_status fail(spod_status s, const char* msg) noexcept {
  try {
    g_last_error = spod_status_string(s);
    g_last_error += ": ";
    g_last_error += msg;
  } catch (...) {
  }
  return s;
}

spod_status fail(spod_status s, const std::string& msg) noexcept { return fail(s, msg.c_str()); }

spod_status hip_fail(hipError_t e, const char* where) noexcept {
  try {
    return fail(SPOD_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
  } catch (...) {
    return fail(SPOD_ERR_HIP, where);
  }
}

bool is_complex128(const Plan& p) { return p.prec == SPOD_PREC_FP64; }

size_t qhat_bytes(const Plan& p) {
  const size_t rows = (size_t)p.nfreq * (size_t)p.nblocks;
  if (p.qhat_packed) return rows * (size_t)pk_row_bytes(p.M);
  return rows * (size_t)p.M * (is_complex128(p) ? 16 : 8);
}

int64_t gram_split_for(const Plan& p, int64_t target) {
  // about `target` workgroups (one per slice and frequency; 8192 measured
  // best on the 1M-DOF workload: 32 slices x 257 frequencies), but keep at
  // least ~4 chunks of degrees of freedom per slice so the partial sums stay
  // cheap
  int64_t s = (target + p.nfreq - 1) / p.nfreq;
  int64_t cap = p.M / 512;
  if (cap < 1) cap = 1;
  if (s > cap) s = cap;
  if (s < 1) s = 1;
  return s;
}

static int64_t auto_gram_split(const Plan& p) {
  if (p.gram_split_opt > 0) return p.gram_split_opt;
  if (p.nblocks > SPOD_SMALL_NBLOCKS) {
    // L > 64: the block pairs of a frequency take several workgroups already
    // (four groups of 6 pairs each); about 4096 workgroups in all
    const int64_t nt16 = (p.nblocks + 15) / 16, np = nt16 * (nt16 + 1) / 2;
    const int64_t z = ((np + 5) / 6 + 3) / 4;
    return gram_split_for(p, std::max<int64_t>(1, 4096 / z));
  }
  return gram_split_for(p, 8192);
}

void plan_set_gram_split(Plan& p, int64_t s) {
  p.gram_split_opt = s;
  p.gram_split = (int)s;
  p.ws_bytes = workspace_bytes(p);
}

static void derive(Plan& p) {
  p.gram_dim = (int)((p.nblocks + 15) / 16 * 16);
  p.gram_split = (int)auto_gram_split(p);
  p.ws_bytes = workspace_bytes(p);
}

size_t workspace_bytes(const Plan& p) {
  size_t w = fft_workspace(p);
  size_t a = csd_workspace(p);
  size_t b = backward_workspace(p);
  size_t e = eig_workspace(p);
  if (a > w) w = a;
  if (b > w) w = b;
  if (e > w) w = e;
  return (w + 255) / 256 * 256;
}

void freeze(Plan& p) { p.frozen = true; }

Plan plan_rows(const Plan& p, int64_t row0, int64_t rows) {
  Plan c = p;
  c.nspace = rows;
  c.nvar = 1;
  c.M = rows;
  c.d_weights = p.d_weights + row0;
  c.d_sqrtw = p.d_sqrtw + row0;
  c.d_sqrtw32 = p.d_sqrtw32 + row0;
  derive(c);
  return c;
}

static bool is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

// Radices of n (8, 4, 2, 3, 5, 7, then the remaining primes in increasing
// order) with the odd stages' work-item shapes and table offsets; returns
// the odd stages' table entries, or -1 when n has more than 32 factors.
static int factor_radices(int64_t n, Radices& rad) {
  rad = Radices{};
  const int64_t n0 = n;
  for (int64_t f : {8, 4, 2, 3, 5, 7}) {
    while (n % f == 0 && rad.n < 32) {
      rad.r[rad.n++] = (int)f;
      n /= f;
    }
  }
  for (int64_t f = 11; n > 1 && rad.n < 32; f += 2) {
    while (n % f == 0 && rad.n < 32) {
      rad.r[rad.n++] = (int)f;
      n /= f;
    }
  }
  if (n != 1) {
    rad.n = 0;
    return -1;
  }
  // A stage costs a barrier, a pass through LDS and a twiddle product per
  // output besides its sums; for the smallest odd radices that costs more than
  // the longer direct sums of one merged stage: a 3 and a 5 become one radix-15
  // stage (8760 = 8 3 5 73: 30.8 -> 28.4 ms on 65,536 DOFs in 8 blocks), two
  // 3s one radix-9 stage.
  for (const int pr : {5, 3}) {
    for (;;) {
      int i3 = -1, ip = -1;
      for (int i = 0; i < rad.n; ++i) {
        if (rad.r[i] == 3 && i3 < 0) i3 = i;
        else if (rad.r[i] == pr && ip < 0) ip = i;
      }
      if (i3 < 0 || ip < 0) break;
      rad.r[i3] = 3 * pr;
      for (int i = ip; i + 1 < rad.n; ++i) rad.r[i] = rad.r[i + 1];
      --rad.n;
    }
  }
  // odd stages first, then the even ones (each group in its order): a first
  // stage of radix 8 over the whole length measured slower than the same
  // stage later (8760: 8 15 73 in 28.5 ms, 15 73 8 in 27.5 ms)
  {
    int rr[32], k = 0;
    for (int i = 0; i < rad.n; ++i)
      if (rad.r[i] % 2 == 1) rr[k++] = rad.r[i];
    for (int i = 0; i < rad.n; ++i)
      if (rad.r[i] % 2 == 0) rr[k++] = rad.r[i];
    for (int i = 0; i < rad.n; ++i) rad.r[i] = rr[i];
  }
  int odd_entries = 0;
  for (int i = 0; i < rad.n; ++i) {
    const int r = rad.r[i];
    if (r % 2 == 0) continue;
    rad.kpt[i] = general_odd_kpt(r, (int)(n0 / r));
    rad.toff[i] = odd_entries;
    odd_entries += general_odd_entries(r, rad.kpt[i]);
  }
  return odd_entries;
}

// The odd stages' tables T[g][j][c] = W_r^{(j + 1) k}, k = min(g + c G, (r-1)/2),
// from a twiddle table W_n^t of the transform length n.
static void odd_tables(const Radices& rad, int64_t n, const std::vector<double2>& tw,
                       const std::vector<float2>& tw32, std::vector<double2>& oddw,
                       std::vector<float2>& oddw32) {
  for (int i = 0; i < rad.n; ++i) {
    const int r = rad.r[i], kpt = rad.kpt[i];
    if (r % 2 == 0) continue;
    const int hm = (r - 1) / 2, G = (hm + 1 + kpt - 1) / kpt;
    size_t e = (size_t)rad.toff[i];
    for (int g = 0; g < G; ++g)
      for (int j = 1; j <= hm; ++j)
        for (int c = 0; c < kpt; ++c, ++e) {
          const int k = std::min(g + c * G, hm);
          const int64_t t = (n / r) * ((int64_t)j * k % r);
          oddw[e] = tw[t];
          oddw32[e] = tw32[t];
        }
  }
}

// Twiddles e^{-2 pi i j / n}, in long double and rounded once.
static void twiddles(int64_t n, std::vector<double2>& tw, std::vector<float2>& tw32) {
  tw.resize(n);
  tw32.resize(n);
  for (int64_t j = 0; j < n; ++j) {
    const long double a = 2.0L * 3.14159265358979323846264338327950288L * (long double)j / (long double)n;
    tw[j] = make_double2((double)cosl(a), (double)-sinl(a));
    tw32[j] = make_float2((float)cosl(a), (float)-sinl(a));
  }
}

// DFT of a real sequence, X[k] = sum_n x[n] e^{-2 pi i k n / N} for k < K, in
// long double: the same self-sorting mixed-radix stages as the device
// transform (decimation in frequency), N * (sum of the radices) operations.
static void host_dft(const std::vector<double>& x, const Radices& rad, int64_t K,
                     std::vector<double2>& out) {
  const int64_t N = (int64_t)x.size();
  std::vector<long double> ct(N), st(N);
  for (int64_t t = 0; t < N; ++t) {
    const long double a = 2.0L * 3.14159265358979323846264338327950288L * (long double)t / (long double)N;
    ct[t] = cosl(a);
    st[t] = -sinl(a);
  }
  std::vector<long double> xr(N), xi(N, 0.0L), yr(N), yi(N);
  for (int64_t i = 0; i < N; ++i) xr[i] = x[i];
  int64_t n = N, s = 1;
  for (int stg = 0; stg < rad.n; ++stg) {
    const int64_t r = rad.r[stg], m = n / r, wn = N / n;
    // y[q + s (r p + k)] = W_n^{p k} sum_j x[q + s (p + j m)] W_r^{j k}
    for (int64_t pp = 0; pp < m; ++pp)
      for (int64_t qq = 0; qq < s; ++qq)
        for (int64_t k = 0; k < r; ++k) {
          long double ar = 0.0L, ai = 0.0L;
          for (int64_t j = 0; j < r; ++j) {
            const int64_t t = (N / r) * ((j * k) % r);
            const int64_t idx = qq + s * (pp + j * m);
            ar += xr[idx] * ct[t] - xi[idx] * st[t];
            ai += xr[idx] * st[t] + xi[idx] * ct[t];
          }
          const int64_t t2 = (wn * pp * k) % N;
          const int64_t o = qq + s * (r * pp + k);
          yr[o] = ar * ct[t2] - ai * st[t2];
          yi[o] = ar * st[t2] + ai * ct[t2];
        }
    xr.swap(yr);
    xi.swap(yi);
    n = m;
    s *= r;
  }
  out.resize(K);
  for (int64_t k = 0; k < K; ++k) out[k] = make_double2((double)xr[k], (double)xi[k]);
}

static spod_status validate_shape(int64_t nt, int64_t nfft, int64_t noverlap, int64_t* L,
                                  int64_t* K) {
  if (nfft < 2) return fail(SPOD_ERR_INVALID_ARG, "nfft must be >= 2");
  if (noverlap < 0 || noverlap >= nfft)
    return fail(SPOD_ERR_INVALID_ARG, "noverlap must be in [0, nfft)");
  if (nt < nfft) return fail(SPOD_ERR_INVALID_ARG, "nt must be >= nfft");
  int64_t l = (nt - noverlap) / (nfft - noverlap);
  if (l < 2) return fail(SPOD_ERR_INVALID_ARG, "fewer than 2 blocks (L-1 normalisation)");
  if (L) *L = l;
  if (K) *K = nfft / 2 + 1;
  return SPOD_OK;
}

}  // namespace spod

using namespace spod;

extern "C" {

const char* spod_status_string(spod_status s) {
  switch (s) {
    case SPOD_OK: return "SPOD_OK";
    case SPOD_ERR_INVALID_ARG: return "SPOD_ERR_INVALID_ARG";
    case SPOD_ERR_UNSUPPORTED: return "SPOD_ERR_UNSUPPORTED";
    case SPOD_ERR_ALLOC: return "SPOD_ERR_ALLOC";
    case SPOD_ERR_HIP: return "SPOD_ERR_HIP";
    case SPOD_ERR_NUMERIC: return "SPOD_ERR_NUMERIC";
    case SPOD_ERR_WORKSPACE: return "SPOD_ERR_WORKSPACE";
    case SPOD_ERR_IO: return "SPOD_ERR_IO";
    case SPOD_ERR_INTERNAL: return "SPOD_ERR_INTERNAL";
  }
  return "SPOD_ERR_UNKNOWN";
}

const char* spod_last_error(void) { return g_last_error.c_str(); }

spod_status spod_shape(int64_t nt, int64_t nfft, int64_t noverlap, int64_t* nblocks,
                       int64_t* nfreq) {
  return validate_shape(nt, nfft, noverlap, nblocks, nfreq);
}

void spod_plan_destroy(spod_plan plan) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return;
  int cur = 0;
  if (hipGetDevice(&cur) == hipSuccess && cur != p->device) (void)hipSetDevice(p->device);
  (void)hipDeviceSynchronize();
  void* bufs[] = {p->d_window, p->d_window32, p->d_weights, p->d_sqrtw,
                  p->d_sqrtw32, p->d_tw64, p->d_tw32, p->d_what, p->d_oddw64, p->d_oddw32,
                  p->d_tw_a64, p->d_tw_a32, p->d_tw_b64, p->d_tw_b32, p->d_oddw_a64,
                  p->d_oddw_a32, p->d_oddw_b64, p->d_oddw_b32};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (cur != p->device) (void)hipSetDevice(cur);
  delete p;
}

spod_status spod_plan_create(int64_t nspace, int64_t nvar, int64_t nt, int64_t nfft,
                             int64_t noverlap, const double* window, const double* weights,
                             spod_plan* out) {
  return guarded([&]() -> spod_status {
    if (!out) return fail(SPOD_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (nspace < 1 || nvar < 1) return fail(SPOD_ERR_INVALID_ARG, "nspace and nvar must be >= 1");
    if (nspace > (int64_t(1) << 40) / nvar) return fail(SPOD_ERR_INVALID_ARG, "M too large");
    int64_t L = 0, K = 0;
    spod_status st = validate_shape(nt, nfft, noverlap, &L, &K);
    if (st != SPOD_OK) return st;
    const int64_t M = nspace * nvar;

    // host copies of window and weights, validated before any HIP call
    std::vector<double> w(nfft), W(M);
    double sw2 = 0.0;
    for (int64_t n = 0; n < nfft; ++n) {
      double v = window ? window[n]
                        : (double)(0.5L - 0.5L * cosl(2.0L * 3.14159265358979323846264338327950288L *
                                                      (long double)n / (long double)nfft));
      if (!std::isfinite(v)) return fail(SPOD_ERR_INVALID_ARG, "window has a non-finite value");
      w[n] = v;
      sw2 += v * v;
    }
    if (!(sw2 > 0.0) || !std::isfinite(sw2)) return fail(SPOD_ERR_INVALID_ARG, "window energy is zero");
    bool any = false;
    for (int64_t m = 0; m < M; ++m) {
      double v = weights ? weights[m] : 1.0 / (double)M;
      if (!std::isfinite(v) || v < 0.0)
        return fail(SPOD_ERR_INVALID_ARG, "weights must be finite and >= 0");
      any |= v > 0.0;
      W[m] = v;
    }
    if (!any) return fail(SPOD_ERR_INVALID_ARG, "weights are all zero");
    if (nfft < 8 || nfft > SPOD_LONG_MAX_NFFT)
      return fail(SPOD_ERR_UNSUPPORTED, "nfft must be in [8, 2^20]");

    Plan* p = new (std::nothrow) Plan();
    if (!p) return fail(SPOD_ERR_ALLOC, "plan");
    p->nspace = nspace;
    p->nvar = nvar;
    p->M = M;
    p->nt = nt;
    p->nfft = nfft;
    p->noverlap = noverlap;
    p->step = nfft - noverlap;
    p->nblocks = L;
    p->nfreq = K;
    p->general = !(is_pow2(nfft) && nfft <= 1024);
    const int odd_entries = std::max(0, factor_radices(nfft, p->radices));
    // above what one workgroup's LDS holds (complex64 above 20480, complex128
    // above 10240): the two-pass transform N = A B, A the largest divisor
    // <= sqrt(N) (both at most SPOD_LONG_MAX_FACTOR).  Its tables are built
    // for every general N above 1024; the precision and SPOD_OPT_GENERAL_PASSES
    // pick the path at launch.
    int odd_a = 0, odd_b = 0;
    if (p->general && nfft > 1024) {
      int64_t a = 1;
      for (int64_t d = 2; d * d <= nfft; ++d)
        if (nfft % d == 0) a = d;
      const int64_t b = nfft / a;
      bool ok = a >= 2 && b <= SPOD_LONG_MAX_FACTOR;
      if (ok) {
        odd_a = factor_radices(a, p->rad_a);
        odd_b = factor_radices(b, p->rad_b);
        for (const Radices* rr : {&p->rad_a, &p->rad_b})
          for (int i = 0; i < rr->n; ++i) ok = ok && rr->r[i] <= 1024;
      }
      if (!ok && nfft > SPOD_GENERAL_MAX_NFFT) {
        delete p;
        return fail(SPOD_ERR_UNSUPPORTED,
                    "nfft above 20480 must be a product A B of two factors <= 4096 "
                    "with prime factors <= 1024");
      }
      if (ok) {
        p->long_dft = true;
        p->long_a = (int)a;
        p->long_b = (int)b;
        // one workgroup per CU (each takes most of a CU's LDS), each with its
        // own slot of the intermediate in the workspace
        int dev = 0, cus = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess || cus < 1) {
          delete p;
          return e != hipSuccess ? hip_fail(e, "hipDeviceGetAttribute") : fail(SPOD_ERR_HIP, "no CUs");
        }
        p->long_grid = cus;
      }
    }
    p->kappa = 1.0 / std::sqrt((double)(L - 1) * sw2);
    // DFT of the window at every one-sided bin, What_k = sum_n w[n] e^{-2 pi i k n / N},
    // in long double with exact integer reduction of k*n mod N
    std::vector<double2> what(K);
    {
      long double sabs = 0.0L;
      for (int64_t n = 0; n < nfft; ++n) sabs += fabsl((long double)w[n]);
      std::vector<long double> ct(nfft), st(nfft);
      for (int64_t t = 0; t < nfft; ++t) {
        const long double a =
            2.0L * 3.14159265358979323846264338327950288L * (long double)t / (long double)nfft;
        ct[t] = cosl(a);
        st[t] = sinl(a);
      }
      int cnt = 0;
      // long blocks: the window's DFT by the host's mixed-radix transform
      // (N sum(r) operations instead of N K)
      std::vector<double2> what_fast;
      const bool fast = nfft > SPOD_GENERAL_MAX_NFFT;
      if (fast) host_dft(w, p->radices, K, what_fast);
      for (int64_t k = 0; k < K; ++k) {
        long double re = 0.0L, im = 0.0L;
        if (fast) {
          re = what_fast[k].x;
          im = what_fast[k].y;
        } else {
          int64_t t = 0;                    // (k * n) mod nfft
          for (int64_t n = 0; n < nfft; ++n) {
            re += (long double)w[n] * ct[t];
            im -= (long double)w[n] * st[t];
            t += k;
            if (t >= nfft) t -= nfft;
          }
        }
        what[k] = make_double2((double)re, (double)im);
        if (cnt >= 0 && sqrtl(re * re + im * im) > 1e-12L * sabs) {
          if (cnt == Plan::SPOD_MAX_MEAN_BINS) {
            cnt = -1;
          } else {
            p->mean_bin[cnt] = (int)k;
            p->what_re[cnt] = (double)re;
            p->what_im[cnt] = (double)im;
            ++cnt;
          }
        }
      }
      p->n_mean_bins = cnt;
    }
    derive(*p);

    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
      delete p;
      return hip_fail(e, "hipGetDevice");
    }
    // twiddles e^{-2 pi i j / N}, computed in long double and rounded once
    std::vector<double2> tw(nfft);
    std::vector<float2> tw32(nfft);
    // the FP32 weights are padded with zeros to a multiple of 128 (whole
    // superblocks of packed Fourier blocks)
    const int64_t Mpad = (M + PK_SB_DOFS - 1) / PK_SB_DOFS * PK_SB_DOFS;
    std::vector<float> w32(nfft), sq32(Mpad, 0.0f);
    std::vector<double> sq(M);
    for (int64_t j = 0; j < nfft; ++j) {
      long double a = 2.0L * 3.14159265358979323846264338327950288L * (long double)j / (long double)nfft;
      tw[j] = make_double2((double)cosl(a), (double)-sinl(a));
      tw32[j] = make_float2((float)cosl(a), (float)-sinl(a));
      w32[j] = (float)w[j];
    }
    for (int64_t m = 0; m < M; ++m) {
      sq[m] = std::sqrt(W[m]);
      sq32[m] = (float)sq[m];
    }
    // the odd stages' tables, from the same rounded twiddles
    std::vector<double2> oddw(std::max(odd_entries, 1));
    std::vector<float2> oddw32(oddw.size());
    for (int i = 0; i < p->radices.n; ++i) {
      const int r = p->radices.r[i], kpt = p->radices.kpt[i];
      if (r % 2 == 0) continue;
      const int hm = (r - 1) / 2, G = (hm + 1 + kpt - 1) / kpt;
      size_t e = (size_t)p->radices.toff[i];
      for (int g = 0; g < G; ++g)
        for (int j = 1; j <= hm; ++j)
          for (int c = 0; c < kpt; ++c, ++e) {
            const int k = std::min(g + c * G, hm);
            const int64_t t = (int64_t)(nfft / r) * ((int64_t)j * k % r);
            oddw[e] = tw[t];
            oddw32[e] = tw32[t];
          }
    }
    struct Up { void** dst; const void* src; size_t bytes; } ups[] = {
        {(void**)&p->d_window, w.data(), sizeof(double) * nfft},
        {(void**)&p->d_window32, w32.data(), sizeof(float) * nfft},
        {(void**)&p->d_weights, W.data(), sizeof(double) * M},
        {(void**)&p->d_sqrtw, sq.data(), sizeof(double) * M},
        {(void**)&p->d_sqrtw32, sq32.data(), sizeof(float) * Mpad},
        {(void**)&p->d_tw64, tw.data(), sizeof(double2) * nfft},
        {(void**)&p->d_tw32, tw32.data(), sizeof(float2) * nfft},
        {(void**)&p->d_what, what.data(), sizeof(double2) * K},
        {(void**)&p->d_oddw64, oddw.data(), sizeof(double2) * oddw.size()},
        {(void**)&p->d_oddw32, oddw32.data(), sizeof(float2) * oddw32.size()},
    };
    // the two-pass transform's tables of A and B
    std::vector<double2> tw_a, tw_b, oddw_a(std::max(odd_a, 1)), oddw_b(std::max(odd_b, 1));
    std::vector<float2> tw_a32, tw_b32, oddw_a32(oddw_a.size()), oddw_b32(oddw_b.size());
    if (p->long_dft) {
      twiddles(p->long_a, tw_a, tw_a32);
      twiddles(p->long_b, tw_b, tw_b32);
      odd_tables(p->rad_a, p->long_a, tw_a, tw_a32, oddw_a, oddw_a32);
      odd_tables(p->rad_b, p->long_b, tw_b, tw_b32, oddw_b, oddw_b32);
    }
    const size_t la = p->long_dft ? (size_t)p->long_a : 0, lb = p->long_dft ? (size_t)p->long_b : 0;
    Up ups_long[] = {
        {(void**)&p->d_tw_a64, tw_a.data(), sizeof(double2) * la},
        {(void**)&p->d_tw_a32, tw_a32.data(), sizeof(float2) * la},
        {(void**)&p->d_tw_b64, tw_b.data(), sizeof(double2) * lb},
        {(void**)&p->d_tw_b32, tw_b32.data(), sizeof(float2) * lb},
        {(void**)&p->d_oddw_a64, oddw_a.data(), p->long_dft ? sizeof(double2) * oddw_a.size() : 0},
        {(void**)&p->d_oddw_a32, oddw_a32.data(), p->long_dft ? sizeof(float2) * oddw_a32.size() : 0},
        {(void**)&p->d_oddw_b64, oddw_b.data(), p->long_dft ? sizeof(double2) * oddw_b.size() : 0},
        {(void**)&p->d_oddw_b32, oddw_b32.data(), p->long_dft ? sizeof(float2) * oddw_b32.size() : 0},
    };
    for (auto& u : ups_long) {
      if (u.bytes == 0) continue;
      e = hipMalloc(u.dst, u.bytes);
      if (e != hipSuccess) {
        spod_plan_destroy(reinterpret_cast<spod_plan>(p));
        return e == hipErrorOutOfMemory ? fail(SPOD_ERR_ALLOC, "plan tables")
                                        : hip_fail(e, "hipMalloc");
      }
      e = hipMemcpy(*u.dst, u.src, u.bytes, hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        spod_plan_destroy(reinterpret_cast<spod_plan>(p));
        return hip_fail(e, "hipMemcpy");
      }
    }
    for (auto& u : ups) {
      e = hipMalloc(u.dst, u.bytes);
      if (e != hipSuccess) {
        spod_plan_destroy(reinterpret_cast<spod_plan>(p));
        return e == hipErrorOutOfMemory ? fail(SPOD_ERR_ALLOC, "plan tables")
                                        : hip_fail(e, "hipMalloc");
      }
      e = hipMemcpy(*u.dst, u.src, u.bytes, hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        spod_plan_destroy(reinterpret_cast<spod_plan>(p));
        return hip_fail(e, "hipMemcpy");
      }
    }
    *out = reinterpret_cast<spod_plan>(p);
    return SPOD_OK;
  });
}

spod_status spod_plan_set_precision(spod_plan plan, spod_precision prec) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return fail(SPOD_ERR_INVALID_ARG, "plan is NULL");
  if (p->frozen) return fail(SPOD_ERR_INVALID_ARG, "plan already used");
  if (prec != SPOD_PREC_FP64 && prec != SPOD_PREC_FP32 && prec != SPOD_PREC_BF16X4 &&
      prec != SPOD_PREC_FP16X4)
    return fail(SPOD_ERR_INVALID_ARG, "unknown precision");
  if (prec == SPOD_PREC_FP64 && p->qhat_packed)
    return fail(SPOD_ERR_UNSUPPORTED, "packed Fourier blocks need a complex64 precision form");
  p->prec = prec;
  derive(*p);
  return SPOD_OK;
}

spod_status spod_plan_set_option(spod_plan plan, spod_option opt, int64_t value) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return fail(SPOD_ERR_INVALID_ARG, "plan is NULL");
  if (p->frozen) return fail(SPOD_ERR_INVALID_ARG, "plan already used");
  switch (opt) {
    case SPOD_OPT_MAX_SWEEPS:
      if (value < 0 || value > 1000) return fail(SPOD_ERR_INVALID_ARG, "max sweeps in [0, 1000]");
      p->max_sweeps = (int)value;
      break;
    case SPOD_OPT_GRAM_SPLIT:
      if (value < 0 || value > 65536) return fail(SPOD_ERR_INVALID_ARG, "gram split in [0, 65536]");
      p->gram_split_opt = value;
      break;
    case SPOD_OPT_FFT_TILE:
      if (value != 0 && value != 16 && value != 32)
        return fail(SPOD_ERR_INVALID_ARG, "fft tile must be 0, 16 or 32");
      p->fft_tile_opt = value;
      break;
    case SPOD_OPT_MODES_KERNEL:
      if (value != 0 && value != 1)
        return fail(SPOD_ERR_INVALID_ARG, "modes kernel must be 0 (vector ALU) or 1 (matrix cores)");
      p->modes_mfma = value == 1;
      break;
    case SPOD_OPT_GENERAL_PASSES:
      if (value != 0 && value != 1 && value != 2)
        return fail(SPOD_ERR_INVALID_ARG, "general passes must be 0, 1 or 2");
      if (value == 2 && !p->long_dft)
        return fail(SPOD_ERR_UNSUPPORTED,
                    "two passes need nfft > 1024, not a power of two, with two factors <= 4096");
      p->general_passes = (int)value;
      break;
    case SPOD_OPT_QHAT_FORMAT:
      if (value != SPOD_QHAT_COMPLEX && value != SPOD_QHAT_BFP20)
        return fail(SPOD_ERR_INVALID_ARG, "qhat format must be SPOD_QHAT_COMPLEX or SPOD_QHAT_BFP20");
      if (value == SPOD_QHAT_BFP20 && (p->prec == SPOD_PREC_FP64 || p->general))
        return fail(SPOD_ERR_UNSUPPORTED,
                    "packed Fourier blocks need a complex64 precision form and a power-of-two "
                    "nfft <= 1024");
      p->qhat_packed = value == SPOD_QHAT_BFP20;
      break;
    default:
      return fail(SPOD_ERR_INVALID_ARG, "unknown option");
  }
  derive(*p);
  return SPOD_OK;
}

spod_status spod_plan_qhat_bytes(spod_plan plan, size_t* bytes) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return fail(SPOD_ERR_INVALID_ARG, "plan is NULL");
  if (!bytes) return fail(SPOD_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = qhat_bytes(*p);
  return SPOD_OK;
}

spod_status spod_plan_query(spod_plan plan, int64_t* nblocks, int64_t* nfreq,
                            size_t* workspace) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return fail(SPOD_ERR_INVALID_ARG, "plan is NULL");
  if (nblocks) *nblocks = p->nblocks;
  if (nfreq) *nfreq = p->nfreq;
  if (workspace) *workspace = p->ws_bytes;
  return SPOD_OK;
}

static spod_status check_ws(const Plan& p, void* ws, size_t ws_bytes, size_t need) {
  if (need == 0) return SPOD_OK;
  if (!ws || ws_bytes < need) {
    char msg[64];
    std::snprintf(msg, sizeof msg, "workspace of %zu bytes required", need);
    return fail(SPOD_ERR_WORKSPACE, msg);
  }
  (void)p;
  return SPOD_OK;
}

static spod_status enter(Plan* p) {
  if (!p) return fail(SPOD_ERR_INVALID_ARG, "plan is NULL");
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (cur != p->device) return fail(SPOD_ERR_INVALID_ARG, "plan belongs to another device");
  freeze(*p);
  return SPOD_OK;
}

spod_status spod_blocks_fft(spod_plan plan, const void* q, spod_dtype dtype, void* qhat,
                            double* mean, void* ws, size_t ws_bytes, spod_stream stream) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  spod_status st = enter(p);
  if (st != SPOD_OK) return st;
  if (!q || !qhat) return fail(SPOD_ERR_INVALID_ARG, "q and qhat are required");
  if (dtype != SPOD_F32 && dtype != SPOD_F64) return fail(SPOD_ERR_INVALID_ARG, "dtype");
  if (p->qhat_packed && (uintptr_t)qhat % 16 != 0)
    return fail(SPOD_ERR_INVALID_ARG, "packed qhat must be 16-byte aligned");
  if (!mean) {
    st = check_ws(*p, ws, ws_bytes, fft_workspace(*p));
    if (st != SPOD_OK) return st;
  }
  return launch_blocks_fft(*p, q, dtype, qhat, mean, ws, (hipStream_t)stream);
}

spod_status spod_csd(spod_plan plan, const void* qhat, void* gram, void* ws, size_t ws_bytes,
                     spod_stream stream) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  spod_status st = enter(p);
  if (st != SPOD_OK) return st;
  if (!qhat || !gram) return fail(SPOD_ERR_INVALID_ARG, "qhat and gram are required");
  if (p->qhat_packed && (uintptr_t)qhat % 16 != 0)
    return fail(SPOD_ERR_INVALID_ARG, "packed qhat must be 16-byte aligned");
  st = check_ws(*p, ws, ws_bytes, csd_workspace(*p));
  if (st != SPOD_OK) return st;
  return launch_csd(*p, qhat, gram, ws, (hipStream_t)stream);
}

spod_status spod_csd_noalloc(spod_plan plan, const void* qhat, void* gram, int64_t* slices,
                             spod_stream stream) {
  return guarded([&]() -> spod_status {
    Plan* p = reinterpret_cast<Plan*>(plan);
    spod_status st = enter(p);
    if (st != SPOD_OK) return st;
    if (!qhat || !gram) return fail(SPOD_ERR_INVALID_ARG, "qhat and gram are required");
    if (p->qhat_packed && (uintptr_t)qhat % 16 != 0)
      return fail(SPOD_ERR_INVALID_ARG, "packed qhat must be 16-byte aligned");
    if (slices) *slices = csd_noalloc_split(*p);
    return launch_csd_noalloc(*p, qhat, gram, (hipStream_t)stream);
  });
}

spod_status spod_eig(spod_plan plan, const void* gram, double* lam, void* psi, int32_t* info,
                     void* ws, size_t ws_bytes, spod_stream stream) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  spod_status st = enter(p);
  if (st != SPOD_OK) return st;
  if (!gram || !lam || !psi) return fail(SPOD_ERR_INVALID_ARG, "gram, lam and psi are required");
  st = check_ws(*p, ws, ws_bytes, eig_workspace(*p));
  if (st != SPOD_OK) return st;
  return launch_eig(*p, gram, lam, psi, info, ws, (hipStream_t)stream);
}

spod_status spod_modes(spod_plan plan, const void* qhat, const double* lam, const void* psi,
                       int64_t n_modes, void* phi, int32_t* n_valid, void* ws, size_t ws_bytes,
                       spod_stream stream) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  spod_status st = enter(p);
  if (st != SPOD_OK) return st;
  if (!qhat || !lam || !psi || !phi)
    return fail(SPOD_ERR_INVALID_ARG, "qhat, lam, psi and phi are required");
  if (n_modes < 1 || n_modes > p->nblocks)
    return fail(SPOD_ERR_INVALID_ARG, "n_modes must be in [1, nblocks]");
  if (p->qhat_packed && (uintptr_t)qhat % 16 != 0)
    return fail(SPOD_ERR_INVALID_ARG, "packed qhat must be 16-byte aligned");
  (void)ws_bytes;
  return launch_modes(*p, qhat, lam, psi, (int)n_modes, phi, n_valid, ws, (hipStream_t)stream);
}

spod_status spod_backward(spod_plan plan, const void* q, spod_dtype dtype, const void* qhat,
                          const double* lam, const void* psi, const double* g_lam,
                          const void* g_phi, int64_t n_modes, const int32_t* bins,
                          int64_t n_bins, void* g_qhat, void* g_q, void* ws, size_t ws_bytes,
                          spod_stream stream) {
  return guarded([&]() -> spod_status {
    Plan* p = reinterpret_cast<Plan*>(plan);
    if (!p) return fail(SPOD_ERR_INVALID_ARG, "plan is NULL");
    if (!lam || !psi || !g_qhat || !g_q)
      return fail(SPOD_ERR_INVALID_ARG, "lam, psi, g_qhat and g_q are required");
    if (!qhat && !q) return fail(SPOD_ERR_INVALID_ARG, "q is required when qhat is NULL");
    if (dtype != SPOD_F32 && dtype != SPOD_F64) return fail(SPOD_ERR_INVALID_ARG, "dtype");
    if (g_phi && (n_modes < 1 || n_modes > p->nblocks))
      return fail(SPOD_ERR_INVALID_ARG, "n_modes must be in [1, nblocks]");
    if (bins) {
      if (n_bins < 1 || n_bins > p->nfreq)
        return fail(SPOD_ERR_INVALID_ARG, "n_bins must be in [1, nfreq]");
      for (int64_t i = 0; i < n_bins; ++i) {
        if (bins[i] < 0 || bins[i] >= p->nfreq || (i > 0 && bins[i] <= bins[i - 1]))
          return fail(SPOD_ERR_INVALID_ARG, "bins must be strictly increasing in [0, nfreq)");
      }
      if (qhat && qhat == g_qhat)
        return fail(SPOD_ERR_INVALID_ARG, "g_qhat may alias qhat only without a bin selection");
    }
    if (p->nfft < 16) return fail(SPOD_ERR_UNSUPPORTED, "backward needs nfft >= 16");
    if (!p->general && p->step != p->nfft && p->step != p->nfft / 2 && p->step != p->nfft / 4)
      return fail(SPOD_ERR_UNSUPPORTED, "backward needs a hop of nfft/4, nfft/2 or nfft");
    if (p->nblocks > 64) return fail(SPOD_ERR_UNSUPPORTED, "nblocks > 64");
    if (p->qhat_packed && qhat)
      return fail(SPOD_ERR_UNSUPPORTED,
                  "packed Fourier blocks: pass qhat = NULL (the blocks are recomputed)");
    spod_status st = enter(p);
    if (st != SPOD_OK) return st;
    st = check_ws(*p, ws, ws_bytes, backward_workspace(*p));
    if (st != SPOD_OK) return st;
    // the adjoint works on complex blocks (g_qhat), whatever the plan stores
    Plan c = *p;
    c.qhat_packed = false;
    return launch_backward(c, q, dtype, qhat, lam, psi, g_lam, g_phi, g_phi ? (int)n_modes : 0,
                           bins, bins ? (int)n_bins : (int)p->nfreq, g_qhat, g_q, ws,
                           (hipStream_t)stream);
  });
}

static spod_status coeff_sel(const Plan& p, int64_t n_modes, const int32_t* bins, int64_t n_bins,
                             int64_t n_r, CoeffSel* cs) {
  if (n_modes < 1 || n_modes > p.nblocks)
    return fail(SPOD_ERR_INVALID_ARG, "n_modes must be in [1, nblocks]");
  if (n_r < 1 || n_r > n_modes) return fail(SPOD_ERR_INVALID_ARG, "n_r must be in [1, n_modes]");
  if (!bins) return fail(SPOD_ERR_INVALID_ARG, "bins is required");
  if (n_bins < 1 || n_bins > p.nfreq)
    return fail(SPOD_ERR_INVALID_ARG, "n_bins must be in [1, nfreq]");
  for (int64_t i = 0; i < n_bins; ++i)
    if (bins[i] < 0 || bins[i] >= p.nfreq || (i > 0 && bins[i] <= bins[i - 1]))
      return fail(SPOD_ERR_INVALID_ARG, "bins must be strictly increasing in [0, nfreq)");
  if (n_bins * n_r > CoeffSel::MAX_R)
    return fail(SPOD_ERR_UNSUPPORTED, "n_bins * n_r above 1024 retained modes");
  cs->n_bins = (int)n_bins;
  cs->n_r = (int)n_r;
  cs->n_modes = (int)n_modes;
  for (int64_t i = 0; i < n_bins; ++i) cs->bin[i] = bins[i];
  return SPOD_OK;
}

spod_status spod_coeffs_query(spod_plan plan, int64_t n_bins, int64_t n_r, size_t* workspace) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return fail(SPOD_ERR_INVALID_ARG, "plan is NULL");
  if (n_bins < 1 || n_r < 1 || n_bins * n_r > CoeffSel::MAX_R)
    return fail(SPOD_ERR_INVALID_ARG, "n_bins * n_r must be in [1, 1024]");
  if (workspace) *workspace = coeff_layout(*p, (int)(n_bins * n_r)).bytes;
  return SPOD_OK;
}

spod_status spod_coeffs(spod_plan plan, const void* q, spod_dtype dtype, const double* mean,
                        const void* phi, int64_t n_modes, const int32_t* bins, int64_t n_bins,
                        int64_t n_r, void* a, int32_t* info, void* ws, size_t ws_bytes,
                        spod_stream stream) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return fail(SPOD_ERR_INVALID_ARG, "plan is NULL");
  if (!q || !mean || !phi || !a || !info)
    return fail(SPOD_ERR_INVALID_ARG, "q, mean, phi, a and info are required");
  if (dtype != SPOD_F32 && dtype != SPOD_F64) return fail(SPOD_ERR_INVALID_ARG, "dtype");
  CoeffSel cs;
  spod_status st = coeff_sel(*p, n_modes, bins, n_bins, n_r, &cs);
  if (st != SPOD_OK) return st;
  st = enter(p);
  if (st != SPOD_OK) return st;
  st = check_ws(*p, ws, ws_bytes, coeff_layout(*p, cs.n_bins * cs.n_r).bytes);
  if (st != SPOD_OK) return st;
  return launch_coeffs(*p, q, dtype, mean, phi, cs, a, info, ws, (hipStream_t)stream);
}

spod_status spod_reconstruct(spod_plan plan, const void* phi, int64_t n_modes, const int32_t* bins,
                             int64_t n_bins, int64_t n_r, const void* a, const double* mean,
                             void* q_rec, spod_dtype dtype, spod_stream stream) {
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return fail(SPOD_ERR_INVALID_ARG, "plan is NULL");
  if (!phi || !a || !mean || !q_rec)
    return fail(SPOD_ERR_INVALID_ARG, "phi, a, mean and q_rec are required");
  if (dtype != SPOD_F32 && dtype != SPOD_F64) return fail(SPOD_ERR_INVALID_ARG, "dtype");
  CoeffSel cs;
  spod_status st = coeff_sel(*p, n_modes, bins, n_bins, n_r, &cs);
  if (st != SPOD_OK) return st;
  st = enter(p);
  if (st != SPOD_OK) return st;
  return launch_reconstruct(*p, phi, cs, a, mean, q_rec, dtype, (hipStream_t)stream);
}

}  // extern "C"
