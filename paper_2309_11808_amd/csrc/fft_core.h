// Length-N_f complex FFT held in registers and LDS, shared by the forward
// block transform and its adjoint.
//
// Stockham autosort, radix 8 in registers with exchanges through LDS: lane j
// of the P = N_f/8 lanes of a transform holds elements j + r*P, r = 0..7, in
// natural order before and after.  Forward sign e^{-2 pi i k n / N_f}.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace spod {

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

// LDS layout of one transform: element i at pad(i) = i + i/8, which spreads the
// stride-8 writes of the first radix-8 stage over all banks; rows (one per
// transform) are LDP = pad(N) + 1 elements apart so that reading the same
// frequency of consecutive rows also spreads over the banks.
__device__ __forceinline__ int pad8(int i) { return i + (i >> 3); }

// Exchange barrier: when a transform lives inside one wavefront (P <= 64) its
// lanes only need a wavefront-level barrier; otherwise the workgroup's.
template <bool WAVE>
__device__ __forceinline__ void xbarrier() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
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
      for (int q = 0; q < RS; ++q) buf[pad8(base + q * NS)] = x[q];
    }
  }
  if constexpr (!LAST) {
    xbarrier<(P <= 64)>();
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = buf[pad8(j + r * P)];
    xbarrier<(P <= 64)>();
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

// Transforms per workgroup: at least a full wavefront of lanes, at most 512
// threads by default (more threads cap the registers per lane at 128).
template <int NF, int BASE>
struct FftShape {
  static constexpr int P = NF / 8;
  static constexpr int NPAIR0 = (BASE * P < 64) ? (64 / P) : BASE;
  static constexpr int NPAIR = (NPAIR0 * P > 1024) ? (1024 / P) : NPAIR0;
  static constexpr int T = 2 * NPAIR;
};

}  // namespace spod
