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
// of T complex values.  The factor 1/2 and the DFT scale kappa ride on the
// window.
#include <hip/hip_runtime.h>

#include "fft_core.h"
#include "internal.h"

namespace spod {

// ---------------------------------------------------------------------------
// temporal mean, accumulated in FP64: one 64-lane wavefront per row
// ---------------------------------------------------------------------------
// A 16-byte-aligned row is read as 16-byte non-temporal vectors, four per
// lane in flight, into four FP64 partial sums (the row is read once here and once
// more by the transform, far beyond any cache); the rest of the row, or a
// whole unaligned row, element by element.
template <typename TIN>
__global__ __launch_bounds__(256) void mean_kernel(const TIN* __restrict__ q, double* __restrict__ mean,
                                                   int64_t M, int64_t nt) {
  typedef TIN vec_t __attribute__((ext_vector_type(16 / sizeof(TIN))));
  constexpr int V = 16 / (int)sizeof(TIN);
  const int lane = threadIdx.x & 63;
  const int64_t m = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (m >= M) return;
  const TIN* row = q + m * nt;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int64_t t0 = 0;
  if ((reinterpret_cast<uintptr_t>(row) & 15) == 0) {   // the same for the whole wavefront
    const vec_t* rv = reinterpret_cast<const vec_t*>(row);
    const int64_t nv = nt / V;
    int64_t i = lane;
    for (; i + 192 < nv; i += 256) {
      vec_t a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = __builtin_nontemporal_load(rv + i + 64 * u);
#pragma unroll
      for (int u = 0; u < 4; u += 2)
#pragma unroll
        for (int e = 0; e < V; e += 2) {
          s0 += (double)a[u][e];
          s1 += (double)a[u][e + 1];
          s2 += (double)a[u + 1][e];
          s3 += (double)a[u + 1][e + 1];
        }
    }
    for (; i < nv; i += 64) {
      const vec_t a = __builtin_nontemporal_load(rv + i);
#pragma unroll
      for (int e = 0; e < V; e += 2) {
        s0 += (double)a[e];
        s1 += (double)a[e + 1];
      }
    }
    t0 = nv * V;
  }
  for (int64_t t = t0 + lane; t < nt; t += 64) s0 += (double)row[t];
  double s = (s0 + s1) + (s2 + s3);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) mean[m] = s / (double)nt;
}

// Streaming stores of two adjacent complex values (16-byte aligned address):
// the blocks are written once and read by a later kernel, so they bypass the
// caches on the way out.
__device__ __forceinline__ void store_pair(float2* o, float2 a, float2 b) {
  typedef float v4 __attribute__((ext_vector_type(4)));
  const v4 v = {a.x, a.y, b.x, b.y};
  __builtin_nontemporal_store(v, reinterpret_cast<v4*>(o));
}
__device__ __forceinline__ void store_pair(double2* o, double2 a, double2 b) {
  typedef double v2 __attribute__((ext_vector_type(2)));
  const v2 va = {a.x, a.y}, vb = {b.x, b.y};
  __builtin_nontemporal_store(va, reinterpret_cast<v2*>(o));
  __builtin_nontemporal_store(vb, reinterpret_cast<v2*>(o) + 1);
}

// Sum over the P lanes of one transform (P a power of two <= 64).
template <int P>
__device__ __forceinline__ double group_sum(double x) {
  static_assert(P <= 64, "a transform must fit in one wavefront");
#pragma unroll
  for (int o = P / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, P);
  return x;
}

// ---------------------------------------------------------------------------
// windowed block transform
// ---------------------------------------------------------------------------
// A workgroup owns a tile of T = 2*NPAIR degrees of freedom and the blocks
// [l0, l1).  SHIFT = hop / P when the hop between blocks is a whole number of
// lane strides (e.g. 4 for 50% overlap): the raw samples of elements
// SHIFT..7 of block l are elements 0..7-SHIFT of block l+1 and stay in
// registers, and only SHIFT new samples per lane are loaded (prefetched one
// block ahead).  SHIFT = 0 means "not a whole number": every block is loaded
// in full.
//
// FUSED: the temporal mean is removed in the same pass.  The workgroup covers
// all L blocks; it transforms w (x - mu0) with mu0 the mean of the first block,
// accumulates sum(x - mu0) over every sample (blocks and the dropped tail) in
// FP64, and at the end subtracts kappa (mu - mu0) What_k from the bins where
// What_k != 0 (the DFT is linear: DFT(w (x - mu)) = DFT(w (x - mu0)) -
// (mu - mu0) What).  mu0 keeps the transform's input of the order of the
// fluctuations, so the FP32 transform does not lose the precision a large
// mean would cost.  Not FUSED: mean[] was computed by mean_kernel.
template <int NF, typename TC, typename TIN, int NPAIR, int SHIFT, bool FUSED, bool PACK = false>
__device__ __forceinline__ void blocks_fft_body(
    const TIN* __restrict__ q, double* __restrict__ mean, const double* __restrict__ window,
    const cpx_t<TC>* __restrict__ tw, cpx_t<TC>* __restrict__ qhat, int64_t M, int64_t ldq,
    int64_t nt, int step, int L, int bpw, TC kappa, const MeanBins& mb,
    const int* __restrict__ sel, int nsel, int64_t tile, int chunk) {
  using C = cpx_t<TC>;
  constexpr int P = NF / 8;              // lanes per transform
  constexpr int T = 2 * NPAIR;           // degrees of freedom per tile
  constexpr int NTH = NPAIR * P;
  constexpr int LDP = NF + NF / 8 + 1;   // padded LDS row
  constexpr int K = NF / 2 + 1;
  constexpr int NEWR = SHIFT == 0 ? 8 : SHIFT;   // freshly loaded elements per block (after the first)
  static_assert(!FUSED || SHIFT > 0, "the fused mean needs a whole-stride hop");
  // complex64: the twiddle table is copied to LDS (4 KB at N = 512), so
  // twiddle reads do not share the vector-memory counter with the prefetch
  constexpr bool TWL = sizeof(TC) == 4;
  __shared__ C lds[NPAIR * LDP];
  __shared__ C twl[TWL ? NF : 1];
  __shared__ double corr[FUSED ? T : 1];
  __shared__ int ksel[K];                // output row s holds frequency ksel[s] (sel != NULL)

  const int tid = threadIdx.x;
  const int f = tid / P;                 // transform (pair) index in the tile
  const int j = tid % P;                 // lane within the transform
  const int64_t m0 = tile * T;
  const int64_t ma = m0 + 2 * f, mb_ = ma + 1;
  const bool va = ma < M, vb = mb_ < M;
  // a row past M reads a real row instead (row a of its pair, else the last
  // row): its transform is never stored, and it cannot carry another row's
  // NaN or infinity into a stored spectrum of its pair
  const TIN* ra = q + (va ? ma : M - 1) * nt;
  const TIN* rb = q + (vb ? mb_ : (va ? ma : M - 1)) * nt;
  C* buf = lds + f * LDP;
  // two adjacent complex values per 16-byte aligned store (complex64 needs an
  // even row stride ldq)
  const bool pair_ok = ((uintptr_t)qhat % 16 == 0) && (sizeof(TC) == 8 || (ldq & 1) == 0);
  if (sel)
    for (int i = tid; i < nsel; i += NTH) ksel[i] = sel[i];

  // the window carries kappa / 2 (the DFT scale and the 1/2 of the
  // two-for-one separation), so the separated spectra need no scaling
  TC w[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) w[r] = (TC)(window[j + r * P] * (0.5 * (double)kappa));
  const C* twp = tw;
  if constexpr (TWL) {
    for (int i = tid; i < NF; i += NTH) twl[i] = tw[i];
    twp = twl;
    __syncthreads();
  }

  const int l0 = chunk * bpw;
  const int l1 = min(L, l0 + bpw);
  TIN xa[8], xb[8], na[8], nb[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int64_t t = (int64_t)l0 * step + j + r * P;
    xa[r] = ra[t];
    xb[r] = rb[t];
  }
  double mua, mub;
  double sa = 0.0, sb = 0.0;             // FUSED: sums of (x - mu0) over this lane's samples
  if constexpr (FUSED) {
    double pa = 0.0, pb = 0.0;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      pa += (double)xa[r];
      pb += (double)xb[r];
    }
    mua = group_sum<P>(pa) / NF;
    mub = group_sum<P>(pb) / NF;
    if constexpr (sizeof(TC) == 4 && sizeof(TIN) == 4) {
      // mu0 is any constant close to the mean: rounded to float, x - mu0 is
      // a single float subtraction with the same (correctly rounded) result
      // as the FP64 difference rounded to float
      mua = (double)(float)mua;
      mub = (double)(float)mub;
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      sa += (double)xa[r] - mua;
      sb += (double)xb[r] - mub;
    }
  } else {
    mua = va ? mean[ma] : 0.0;
    mub = vb ? mean[mb_] : 0.0;
  }

  for (int l = l0; l < l1; ++l) {
    // prefetch the samples block l+1 needs that block l does not hold; the
    // last block re-reads its own (in-range) samples so the loads stay
    // unconditional and in flight during the transform
    const bool more = l + 1 < l1;
    const int64_t tn = (int64_t)(more ? l + 1 : l) * step + j;
#pragma unroll
    for (int r = 8 - NEWR; r < 8; ++r) {
      na[r] = __builtin_nontemporal_load(ra + tn + r * P);     // q is read once
      nb[r] = __builtin_nontemporal_load(rb + tn + r * P);
    }
    __builtin_amdgcn_sched_barrier(0);

    C v[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      TC a, b;
      if constexpr (FUSED && sizeof(TC) == 4 && sizeof(TIN) == 4) {
        a = xa[r] - (float)mua;
        b = xb[r] - (float)mub;
      } else {
        a = (TC)((double)xa[r] - mua);
        b = (TC)((double)xb[r] - mub);
      }
      v[r] = C{a * w[r], b * w[r]};
    }
    stockham<NF, 1>(v, buf, j, twp);
#pragma unroll
    for (int r = 0; r < 8; ++r) buf[pad8(j + r * P)] = v[r];
    if (j == 0) buf[pad8(NF)] = v[0];      // Z[N] = Z[0]: the partner of k = 0 is pad8(N - 0)
    __syncthreads();

    // take in the prefetched samples of block l+1 now, before this block's
    // stores are issued: the vector-memory counter also counts stores, so a
    // wait placed after the store loop would wait for every store as well.
    // The shift is unconditional (after the last block the registers are
    // dead): loads used only under a branch get sunk into it, past the
    // transform, which would undo the prefetch.
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      if (r < 8 - NEWR) {
        xa[r] = xa[r + NEWR];
        xb[r] = xb[r + NEWR];
      } else {
        xa[r] = na[r];
        xb[r] = nb[r];
      }
    }
    if constexpr (FUSED) {
      if (more) {            // uniform: the last block's re-read samples are not new
#pragma unroll
        for (int r = 8 - NEWR; r < 8; ++r) {
          sa += (double)xa[r] - mua;
          sb += (double)xb[r] - mub;
        }
      }
    }
    // an empty asm that reads the new samples pins their arrival (the wait
    // on the prefetch) here, ahead of the store loop
#pragma unroll
    for (int r = 8 - NEWR; r < 8; ++r) asm volatile("" ::"v"(xa[r]), "v"(xb[r]));

    // separate the two real spectra and write qhat[s][l][m0 .. m0+T), where
    // output row s holds frequency k = s (or ksel[s] for a bin selection).
    // One thread per (row, pair): X_a = (A + conj B) / 2 and
    // X_b = (A - conj B) / (2i) come from the same two LDS reads, and the two
    // adjacent degrees of freedom are written with one 16-byte streaming store
    // (or, packed, as their 20-bit mantissas: 8 consecutive threads form a
    // group of 16 degrees of freedom and share its exponent).
    if constexpr (PACK) {
      // one thread per quarter group (two pairs, 4 degrees of freedom); the
      // 4 quarters of a group are an aligned quad of lanes.  Degrees of
      // freedom past M are stored as zeros (the separation of a pair with one
      // real row leaves rounding noise in the other).
      constexpr int NQ = NPAIR / 2;
      for (int idx = tid; idx < nsel * NQ; idx += NTH) {
        const int fq = idx % NQ;
        const int s = idx / NQ;
        const int k = sel ? ksel[s] : s;
        float v[8];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const C* row = lds + (2 * fq + h) * LDP;
          const C A = row[pad8(k)];
          const C Bc = row[pad8((NF - k) & (NF - 1))];
          const int64_t m = m0 + 4 * fq + 2 * h;
          const bool ka = m < M, kb = m + 1 < M;
          v[4 * h] = ka ? (float)(A.x + Bc.x) : 0.0f;
          v[4 * h + 1] = ka ? (float)(A.y - Bc.y) : 0.0f;
          v[4 * h + 2] = kb ? (float)(A.y + Bc.y) : 0.0f;
          v[4 * h + 3] = kb ? (float)(Bc.x - A.x) : 0.0f;
        }
        // ldq is the packed row length in bytes; tiles cover whole superblocks
        const int64_t m = m0 + 4 * fq;
        char* sb = reinterpret_cast<char*>(qhat) + ((int64_t)s * L + l) * ldq +
                   (m / PK_SB_DOFS) * PK_SB_BYTES;
        pk_store_quarter(sb, (int)((m % PK_SB_DOFS) >> 4), (int)((m & 15) >> 2), v);
      }
    } else if (!sel && pair_ok && m0 + T <= M) {
      // every frequency, a whole tile with 16-byte stores: thread tid keeps
      // its pair (tid % NPAIR) and steps over the rows s = tid / NPAIR + i SR
      constexpr int SR = NTH / NPAIR;
      const int f2 = tid % NPAIR;
      const C* row = lds + f2 * LDP;
      int s = tid / NPAIR;
      int ia = pad8(s), ib = pad8(NF - s);
      C* o = qhat + ((int64_t)s * L + l) * ldq + m0 + 2 * f2;
      const int64_t ostep = (int64_t)SR * L * ldq;
      for (; s < nsel; s += SR, o += ostep) {
        const C A = row[ia];
        const C Bc = row[ib];
        store_pair(o, C{A.x + Bc.x, A.y - Bc.y}, C{A.y + Bc.y, Bc.x - A.x});
        if constexpr (SR % 8 == 0) {         // pad8 is linear in steps of 8
          ia += SR + SR / 8;
          ib -= SR + SR / 8;
        } else {
          ia = pad8(s + SR);
          ib = pad8(NF - s - SR);
        }
      }
    } else {
      for (int idx = tid; idx < nsel * NPAIR; idx += NTH) {
        const int f2 = idx % NPAIR;
        const int s = idx / NPAIR;
        const int k = sel ? ksel[s] : s;
        const C* row = lds + f2 * LDP;
        const C A = row[pad8(k)];
        const C Bc = row[pad8((NF - k) & (NF - 1))];
        const C Xa = C{A.x + Bc.x, A.y - Bc.y};
        const C Xb = C{A.y + Bc.y, Bc.x - A.x};
        const int64_t m = m0 + 2 * f2;
        C* o = qhat + (int64_t)l * ldq + (int64_t)s * L * ldq + m;
        if (pair_ok && m + 1 < M) {
          store_pair(o, Xa, Xb);
        } else {
          if (m < M) o[0] = Xa;
          if (m + 1 < M) o[1] = Xb;
        }
      }
    }
    __syncthreads();

  }

  if constexpr (FUSED) {
    // snapshots after the last block only enter the mean
    for (int64_t t = (int64_t)(L - 1) * step + NF + j; t < nt; t += P) {
      if (va) sa += (double)ra[t] - mua;
      if (vb) sb += (double)rb[t] - mub;
    }
    sa = group_sum<P>(sa);
    sb = group_sum<P>(sb);
    const double da = sa / (double)nt, db = sb / (double)nt;   // mu - mu0
    if (j == 0) {
      if (va) mean[ma] = mua + da;
      if (vb) mean[mb_] = mub + db;
      corr[2 * f] = da * (double)kappa;
      corr[2 * f + 1] = db * (double)kappa;
    }
    __syncthreads();
    if constexpr (PACK) {
      // decode, correct and re-encode the groups of the mean bins' rows (the
      // group exponent may change); one thread per quarter group as in the
      // stores
      constexpr int NQ = NPAIR / 2;
      for (int idx = tid; idx < mb.n * L * NQ; idx += NTH) {
        const int fq = idx % NQ;
        const int l = (idx / NQ) % L;
        const int s = idx / (NQ * L);
        const int64_t m = m0 + 4 * fq;
        char* sb = reinterpret_cast<char*>(qhat) + ((int64_t)mb.k[s] * L + l) * ldq +
                   (m / PK_SB_DOFS) * PK_SB_BYTES;
        const int g = (int)((m % PK_SB_DOFS) >> 4), c = (int)((m & 15) >> 2);
        const char* grp = sb + PK_HDR_BYTES + PK_GROUP_BYTES * g;
        typedef unsigned int v4u __attribute__((ext_vector_type(4)));
        const v4u hw = *reinterpret_cast<const v4u*>(grp + 16 * c);
        const uint32_t nib = *reinterpret_cast<const uint32_t*>(grp + 64 + 4 * c);
        const float scale = pk_scale((int)(signed char)sb[g]);
        float v[8];
        pk_decode4(hw[0], hw[1], nib & 0xffffu, scale, v);
        pk_decode4(hw[2], hw[3], nib >> 16, scale, v + 4);
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          const double cd = corr[4 * fq + d];
          const bool live = m + d < M;
          v[2 * d] = live ? (float)((double)v[2 * d] - cd * mb.wr[s]) : 0.0f;
          v[2 * d + 1] = live ? (float)((double)v[2 * d + 1] - cd * mb.wi[s]) : 0.0f;
        }
        // every lane of the group has read its quarter (and the exponent)
        // before any lane overwrites them (the quad runs in lockstep)
        __builtin_amdgcn_wave_barrier();
        pk_store_quarter(sb, g, c, v);
      }
    } else {
      for (int idx = tid; idx < mb.n * L * T; idx += NTH) {
        const int d = idx % T;
        const int l = (idx / T) % L;
        const int s = idx / (T * L);
        const int64_t m = m0 + d;
        if (m >= M) continue;
        C* o = qhat + ((int64_t)mb.k[s] * L + l) * ldq + m;
        const C raw = *o;
        const double c = corr[d];
        *o = C{(TC)((double)raw.x - c * mb.wr[s]), (TC)((double)raw.y - c * mb.wi[s])};
      }
    }
  }
}

// PACK: qhat in the packed 20-bit layout (ldq = bytes of a packed row).
template <int NF, typename TC, typename TIN, int NPAIR, int SHIFT, bool FUSED, bool PACK>
__global__ __launch_bounds__(NPAIR*(NF / 8)) void blocks_fft_kernel(
    const TIN* __restrict__ q, double* __restrict__ mean, const double* __restrict__ window,
    const cpx_t<TC>* __restrict__ tw, cpx_t<TC>* __restrict__ qhat, int64_t M, int64_t ldq,
    int64_t nt, int step, int L, int bpw, TC kappa, MeanBins mb, const int* __restrict__ sel,
    int nsel) {
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  blocks_fft_body<NF, TC, TIN, NPAIR, SHIFT, FUSED, PACK>(q, mean, window, tw, qhat, M, ldq, nt, step,
                                                          L, bpw, kappa, mb, sel, nsel, tile,
                                                          blockIdx.y);
}

// Grouped launch over the problems of a batch that share N_f, precision, input
// type and hop: workgroup b belongs to the last item whose first workgroup is
// <= b, and transforms that item's tile b - start (all blocks, fused mean).
// PERSIST: persistent workgroups that take units (tiles) from the queue; a
// separate instantiation, so the loop's register needs do not reach the
// one-unit-per-workgroup kernel.
template <int NF, typename TC, typename TIN, int NPAIR, int SHIFT, bool PERSIST>
__global__ __launch_bounds__(NPAIR*(NF / 8)) void blocks_fft_batch_kernel(const FftItem* __restrict__ items,
                                                                          int n, int units, int* queue) {
  __shared__ int slot;
  for (int b = next_unit(PERSIST ? queue : nullptr, &slot, true); b < units;
       b = next_unit(PERSIST ? queue : nullptr, &slot, false)) {
    const FftItem& it = items[find_item(items, n, b)];
    blocks_fft_body<NF, TC, TIN, NPAIR, SHIFT, true>(
        static_cast<const TIN*>(it.q), it.mean, it.window, static_cast<const cpx_t<TC>*>(it.tw),
        static_cast<cpx_t<TC>*>(it.qhat), it.M, it.ldq, it.nt, it.step, it.L, it.L, (TC)it.kappa,
        it.mb, nullptr, NF / 2 + 1, (int64_t)b - it.start, 0);
    if constexpr (!PERSIST) break;
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
template <int NF, typename TC, typename TIN, int NPAIR, int SHIFT, bool FUSED>
static void launch_fft_kernel(const Plan& p, dim3 grid, const TIN* q, double* mean, const void* tw,
                              void* qhat, int bpw, const MeanBins& mb, const FftSel& fs,
                              hipStream_t st) {
  using C = cpx_t<TC>;
  constexpr int P = NF / 8;
  const int nsel = fs.d_sel ? fs.nsel : (int)p.nfreq;
  if constexpr (sizeof(TC) == 4) {
    if (p.qhat_packed) {
      hipLaunchKernelGGL((blocks_fft_kernel<NF, TC, TIN, NPAIR, SHIFT, FUSED, true>), grid,
                         dim3(NPAIR * P), 0, st, q, mean, p.d_window, static_cast<const C*>(tw),
                         static_cast<C*>(qhat), (int64_t)p.M, pk_row_bytes(p.M), (int64_t)p.nt,
                         (int)p.step, (int)p.nblocks, bpw, (TC)p.kappa, mb, fs.d_sel, nsel);
      return;
    }
  }
  hipLaunchKernelGGL((blocks_fft_kernel<NF, TC, TIN, NPAIR, SHIFT, FUSED, false>), grid,
                     dim3(NPAIR * P), 0, st, q, mean, p.d_window, static_cast<const C*>(tw),
                     static_cast<C*>(qhat), (int64_t)p.M, (int64_t)p.M, (int64_t)p.nt, (int)p.step,
                     (int)p.nblocks, bpw, (TC)p.kappa, mb, fs.d_sel, nsel);
}

template <int NF, typename TC, typename TIN, int BASE>
static spod_status launch_fft_shape(const Plan& p, const TIN* q, double* mean, void* qhat,
                                    hipStream_t st, bool fused, const FftSel& fs) {
  using S = FftShape<NF, BASE>;
  constexpr int P = S::P, NPAIR = S::NPAIR, T = S::T;
  static_assert(PK_SB_DOFS % T == 0, "tiles must tile the packed superblocks");
  // packed blocks: the tiles cover whole superblocks (their padding is written as zeros)
  const int64_t ntiles = p.qhat_packed ? pk_superblocks(p.M) * (PK_SB_DOFS / T) : (p.M + T - 1) / T;
  if (ntiles > 0x7fffffff) return fail(SPOD_ERR_UNSUPPORTED, "too many tiles");
  const int L = (int)p.nblocks;
  const void* tw = sizeof(TC) == 4 ? (const void*)p.d_tw32 : (const void*)p.d_tw64;
  MeanBins mb{};
  // the correction is applied to the output row of each mean bin (bins outside
  // a selection are not written at all)
  mb.n = 0;
  for (int i = 0; fused && i < p.n_mean_bins; ++i) {
    const int row = fs.d_sel ? fs.h_slot[p.mean_bin[i]] : p.mean_bin[i];
    if (row < 0) continue;
    mb.k[mb.n] = row;
    mb.wr[mb.n] = p.what_re[i];
    mb.wi[mb.n] = p.what_im[i];
    ++mb.n;
  }
  const int shift = (p.step % P == 0) ? (int)(p.step / P) : 0;
  if (fused) {
    if constexpr (P <= 64) {
      dim3 grid((unsigned)ntiles, 1);
      switch (shift) {
        case 2: launch_fft_kernel<NF, TC, TIN, NPAIR, 2, true>(p, grid, q, mean, tw, qhat, L, mb, fs, st); break;
        case 4: launch_fft_kernel<NF, TC, TIN, NPAIR, 4, true>(p, grid, q, mean, tw, qhat, L, mb, fs, st); break;
        case 8: launch_fft_kernel<NF, TC, TIN, NPAIR, 8, true>(p, grid, q, mean, tw, qhat, L, mb, fs, st); break;
        default: return fail(SPOD_ERR_UNSUPPORTED, "fused transform needs hop = N/4, N/2 or N");
      }
    } else {
      return fail(SPOD_ERR_UNSUPPORTED, "fused transform needs nfft <= 512");
    }
  } else {
    // split the blocks over workgroups only when the tiles alone cannot fill the GPU
    int64_t chunks = 1;
    if (ntiles < 4096) chunks = (4096 + ntiles - 1) / ntiles;
    if (chunks > L) chunks = L;
    const int bpw = (int)((L + chunks - 1) / chunks);
    chunks = (L + bpw - 1) / bpw;
    dim3 grid((unsigned)ntiles, (unsigned)chunks);
    if (shift == 4)
      launch_fft_kernel<NF, TC, TIN, NPAIR, 4, false>(p, grid, q, mean, tw, qhat, bpw, mb, fs, st);
    else
      launch_fft_kernel<NF, TC, TIN, NPAIR, 0, false>(p, grid, q, mean, tw, qhat, bpw, mb, fs, st);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPOD_OK : hip_fail(e, "blocks_fft_kernel");
}

template <int NF, typename TC, typename TIN>
static spod_status launch_fft_nf(const Plan& p, const TIN* q, double* mean, void* qhat,
                                 hipStream_t st, bool fused, const FftSel& fs) {
  // Default tile (measured on 393,216 DOFs, 50% overlap): 16 degrees of
  // freedom at N >= 512 (512 threads, two workgroups share a CU, so one's
  // stores overlap the other's transform), 32 for shorter transforms (more
  // work per workgroup; up to 18% faster at N = 128 for complex128).
  // SPOD_OPT_FFT_TILE = 16 or 32 overrides.
  const bool wide = p.fft_tile_opt == 32 || (p.fft_tile_opt == 0 && NF <= 256);
  if (wide && FftShape<NF, 16>::NPAIR != FftShape<NF, 8>::NPAIR)
    return launch_fft_shape<NF, TC, TIN, 16>(p, q, mean, qhat, st, fused, fs);
  return launch_fft_shape<NF, TC, TIN, 8>(p, q, mean, qhat, st, fused, fs);
}

template <typename TC, typename TIN>
static spod_status launch_fft_t(const Plan& p, const TIN* q, double* mean, void* qhat,
                                hipStream_t st, bool fused, const FftSel& fs) {
  switch (p.nfft) {
    case 8: return launch_fft_nf<8, TC, TIN>(p, q, mean, qhat, st, fused, fs);
    case 16: return launch_fft_nf<16, TC, TIN>(p, q, mean, qhat, st, fused, fs);
    case 32: return launch_fft_nf<32, TC, TIN>(p, q, mean, qhat, st, fused, fs);
    case 64: return launch_fft_nf<64, TC, TIN>(p, q, mean, qhat, st, fused, fs);
    case 128: return launch_fft_nf<128, TC, TIN>(p, q, mean, qhat, st, fused, fs);
    case 256: return launch_fft_nf<256, TC, TIN>(p, q, mean, qhat, st, fused, fs);
    case 512: return launch_fft_nf<512, TC, TIN>(p, q, mean, qhat, st, fused, fs);
    case 1024: return launch_fft_nf<1024, TC, TIN>(p, q, mean, qhat, st, fused, fs);
  }
  return fail(SPOD_ERR_UNSUPPORTED, "nfft");
}

// ---------------------------------------------------------------------------
// grouped launch for a batch: fused mean, hop N/2, nfft <= 512.  Tile: 16 or
// 32 degrees of freedom, or 0 for the single-problem default (32 up to
// N = 256, else 16).  A tile's results do not depend on the tile size (the
// pairs are the same adjacent DOFs), so every choice is bit-identical to the
// single-problem path.
// ---------------------------------------------------------------------------
template <int NF, int BASE>
using GroupShape = FftShape<NF, BASE>;

constexpr int group_base(int nf, int tile) { return tile == 32 ? 16 : (tile == 16 ? 8 : (nf <= 256 ? 16 : 8)); }

template <int NF, typename TC, typename TIN, int BASE>
static spod_status fft_group_shape(const FftItem* d, int n, int wgs, int* queue, hipStream_t st) {
  using S = GroupShape<NF, BASE>;
  if (queue) {
    const void* k = reinterpret_cast<const void*>(&blocks_fft_batch_kernel<NF, TC, TIN, S::NPAIR, 4, true>);
    hipLaunchKernelGGL((blocks_fft_batch_kernel<NF, TC, TIN, S::NPAIR, 4, true>),
                       dim3((unsigned)persistent_grid(k, S::NPAIR * S::P, 0, wgs)),
                       dim3(S::NPAIR * S::P), 0, st, d, n, wgs, queue);
  } else {
    hipLaunchKernelGGL((blocks_fft_batch_kernel<NF, TC, TIN, S::NPAIR, 4, false>), dim3((unsigned)wgs),
                       dim3(S::NPAIR * S::P), 0, st, d, n, wgs, queue);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPOD_OK : hip_fail(e, "blocks_fft_batch_kernel");
}

template <int NF, typename TC, typename TIN>
static spod_status fft_group_nf(int tile, const FftItem* d, int n, int wgs, int* queue, hipStream_t st) {
  if (group_base(NF, tile) == 16) return fft_group_shape<NF, TC, TIN, 16>(d, n, wgs, queue, st);
  return fft_group_shape<NF, TC, TIN, 8>(d, n, wgs, queue, st);
}

template <typename TC, typename TIN>
static spod_status fft_group_t(int nfft, int tile, const FftItem* d, int n, int wgs, int* queue,
                               hipStream_t st) {
  switch (nfft) {
    case 16: return fft_group_nf<16, TC, TIN>(tile, d, n, wgs, queue, st);
    case 32: return fft_group_nf<32, TC, TIN>(tile, d, n, wgs, queue, st);
    case 64: return fft_group_nf<64, TC, TIN>(tile, d, n, wgs, queue, st);
    case 128: return fft_group_nf<128, TC, TIN>(tile, d, n, wgs, queue, st);
    case 256: return fft_group_nf<256, TC, TIN>(tile, d, n, wgs, queue, st);
    case 512: return fft_group_nf<512, TC, TIN>(tile, d, n, wgs, queue, st);
  }
  return fail(SPOD_ERR_UNSUPPORTED, "grouped transform: nfft");
}

int fft_group_tile(int nfft, spod_precision prec, int tile) {
  (void)prec;
  switch (nfft) {
#define SPOD_TILE(NF) \
    case NF: return group_base(NF, tile) == 16 ? GroupShape<NF, 16>::T : GroupShape<NF, 8>::T;
    SPOD_TILE(16) SPOD_TILE(32) SPOD_TILE(64) SPOD_TILE(128) SPOD_TILE(256) SPOD_TILE(512)
#undef SPOD_TILE
  }
  return 0;
}

spod_status launch_fft_group(int nfft, spod_precision prec, spod_dtype dtype, int shift, int tile,
                             const FftItem* d_items, int n, int wgs, int* queue, hipStream_t st) {
  if (shift != 4) return fail(SPOD_ERR_UNSUPPORTED, "grouped transform: hop must be nfft/2");
  const bool c128 = prec == SPOD_PREC_FP64;
  if (dtype == SPOD_F32)
    return c128 ? fft_group_t<double, float>(nfft, tile, d_items, n, wgs, queue, st)
                : fft_group_t<float, float>(nfft, tile, d_items, n, wgs, queue, st);
  return c128 ? fft_group_t<double, double>(nfft, tile, d_items, n, wgs, queue, st)
              : fft_group_t<float, double>(nfft, tile, d_items, n, wgs, queue, st);
}

// the mean (when the caller passes no buffer for it), then, for the two-pass
// transform, its scratch
size_t fft_workspace(const Plan& p) {
  const size_t mean = (sizeof(double) * (size_t)p.M + 255) / 256 * 256;
  return mean + long_scratch_bytes(p);
}

spod_status launch_blocks_fft(const Plan& p, const void* q, spod_dtype dtype, void* qhat,
                              double* mean, void* ws, hipStream_t st, const FftSel& fs) {
  // the mean goes to the caller's buffer, or to the start of the workspace
  double* mu = mean ? mean : static_cast<double*>(ws);
  if (p.qhat_packed && (p.general || fs.d_sel || is_complex128(p)))
    return fail(SPOD_ERR_UNSUPPORTED, "packed Fourier blocks: complex64, power-of-two nfft, all bins");
  if (p.general) {
    if (fs.d_sel) return fail(SPOD_ERR_UNSUPPORTED, "frequency selection needs a power-of-two nfft");
    const int64_t mgrid = (p.M + 3) / 4;
    if (dtype == SPOD_F32)
      hipLaunchKernelGGL(mean_kernel<float>, dim3((unsigned)mgrid), dim3(256), 0, st,
                         (const float*)q, mu, (int64_t)p.M, (int64_t)p.nt);
    else
      hipLaunchKernelGGL(mean_kernel<double>, dim3((unsigned)mgrid), dim3(256), 0, st,
                         (const double*)q, mu, (int64_t)p.M, (int64_t)p.nt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "mean_kernel");
    if (long_scratch_bytes(p) > 0) {
      if (!ws) return fail(SPOD_ERR_WORKSPACE, "the two-pass transform needs the plan's workspace");
      char* scratch = static_cast<char*>(ws) + (sizeof(double) * (size_t)p.M + 255) / 256 * 256;
      return launch_blocks_dft_long(p, q, dtype, mu, qhat, scratch, st);
    }
    return launch_blocks_dft_general(p, q, dtype, mu, qhat, st);
  }
  // single pass when the window's DFT has few non-zero bins and the hop is a
  // whole number of lane strides; otherwise a separate FP64 mean pass first
  const int P = (int)(p.nfft / 8);
  const int shift = (p.step % P == 0) ? (int)(p.step / P) : 0;
  // (the per-transform sums are wavefront shuffles: one transform must fit in
  // one wavefront, P <= 64)
  const bool fused = p.n_mean_bins >= 0 && P <= 64 && (shift == 2 || shift == 4 || shift == 8);
  if (!fused) {
    const int64_t mgrid = (p.M + 3) / 4;
    if (dtype == SPOD_F32)
      hipLaunchKernelGGL(mean_kernel<float>, dim3((unsigned)mgrid), dim3(256), 0, st,
                         (const float*)q, mu, (int64_t)p.M, (int64_t)p.nt);
    else
      hipLaunchKernelGGL(mean_kernel<double>, dim3((unsigned)mgrid), dim3(256), 0, st,
                         (const double*)q, mu, (int64_t)p.M, (int64_t)p.nt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "mean_kernel");
  }
  const bool c128 = is_complex128(p);
  if (dtype == SPOD_F32)
    return c128 ? launch_fft_t<double, float>(p, (const float*)q, mu, qhat, st, fused, fs)
                : launch_fft_t<float, float>(p, (const float*)q, mu, qhat, st, fused, fs);
  return c128 ? launch_fft_t<double, double>(p, (const double*)q, mu, qhat, st, fused, fs)
              : launch_fft_t<float, double>(p, (const double*)q, mu, qhat, st, fused, fs);
}

}  // namespace spod
