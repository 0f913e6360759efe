// Batched complex FFT in LDS and the sine transform built on it.
//
// Sine transform (Sec. 4.3): X_k = sum_{i=1}^{n-1} x_i sin(pi k i / n),
// k = 1..n-1.  Two real sequences a, b of the same length are packed as the
// odd extension z of length L = 2n:
//     z_0 = z_n = 0,  z_i = a_i + i b_i,  z_{2n-i} = -(a_i + i b_i),
// and one forward DFT Z_k = sum_m z_m exp(-2 pi i k m / L) gives
//     Z_k = -2i A_k + 2 B_k,  i.e.  A_k = -Im(Z_k)/2,  B_k = Re(Z_k)/2.
// The transform is its own inverse up to 2/n, so the same routine serves
// the analysis and the synthesis sums of Sec. 4.3.
//
// The DFT is a Stockham autosort FFT over radices 4 and 2, with the radix-3
// stage of L = 3*2^k placed last, so that the span Ns of every stage is a
// power of two and all index arithmetic is shifts and masks.  At a stage of
// radix R, butterfly j reads x[j + r L/R], twiddles element r by
// w_L^(r (j mod Ns) L/(Ns R)), takes an R-point DFT and writes
// y[(j div Ns) Ns R + (j mod Ns) + r Ns].  The stage loop is a runtime loop
// (compact code), each stage runs in place on one LDS buffer: every thread
// reads the inputs of its butterflies, the block synchronises, every thread
// writes its outputs, the block synchronises.  Twiddles w_L^m, m < L/2, come
// from an LDS copy of a host-built FP64 table (w^(m + L/2) = -w^m).
// A block transforms one or two sequences (nseq <= 2) of length L <= 2048.
#pragma once

#include "cgp_internal.hpp"

namespace cgp {

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

template <typename T, int R>
__device__ __forceinline__ void small_dft(cplx<T>* v) {
  if constexpr (R == 2) {
    cplx<T> a = v[0], b = v[1];
    v[0] = {a.x + b.x, a.y + b.y};
    v[1] = {a.x - b.x, a.y - b.y};
  } else if constexpr (R == 4) {
    cplx<T> s02 = {v[0].x + v[2].x, v[0].y + v[2].y};
    cplx<T> d02 = {v[0].x - v[2].x, v[0].y - v[2].y};
    cplx<T> s13 = {v[1].x + v[3].x, v[1].y + v[3].y};
    cplx<T> d13 = {v[1].x - v[3].x, v[1].y - v[3].y};
    v[0] = {s02.x + s13.x, s02.y + s13.y};
    v[2] = {s02.x - s13.x, s02.y - s13.y};
    // -i * d13 = (d13.y, -d13.x)
    v[1] = {d02.x + d13.y, d02.y - d13.x};
    v[3] = {d02.x - d13.y, d02.y + d13.x};
  } else {  // R == 3, w = exp(-2 pi i / 3) = -1/2 - i sqrt(3)/2
    const T h = T(0.8660254037844386467637231707529362);
    cplx<T> a0 = v[0], s = {v[1].x + v[2].x, v[1].y + v[2].y};
    cplx<T> d = {v[1].x - v[2].x, v[1].y - v[2].y};
    cplx<T> t = {a0.x - T(0.5) * s.x, a0.y - T(0.5) * s.y};
    v[0] = {a0.x + s.x, a0.y + s.y};
    v[1] = {t.x + h * d.y, t.y - h * d.x};
    v[2] = {t.x - h * d.y, t.y + h * d.x};
  }
}

// w_L^m from the half table (m < L).
template <typename T>
__device__ __forceinline__ cplx<T> twiddle(const cplx<T>* tw, int m, int half) {
  if (m < half) return tw[m];
  const cplx<T> w = tw[m - half];
  return {-w.x, -w.y};
}

// One in-place stage of radix R over nseq sequences of length L in `buf`.
// Thread `tid` owns butterflies b = tid + NT q (q < MAXB).
template <typename T, int R, int MAXB>
__device__ __forceinline__ void fft_stage(cplx<T>* buf, int nseq, int L, int lns,
                                          int twscale, const cplx<T>* tw) {
  const int LR = L / R;
  const int nb = nseq * LR;
  const int ns = 1 << lns;
  constexpr int NT = kThreads;
  cplx<T> v[MAXB][R];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int b = threadIdx.x + NT * q;
    if (b < nb) {
      const int p = b >= LR ? 1 : 0;
      const int j = b - p * LR;
      const int k = j & (ns - 1);
      const cplx<T>* src = buf + p * L + j;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = src[r * LR];
      if (k != 0) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], twiddle(tw, r * k * twscale, L >> 1));
      }
      small_dft<T, R>(v[q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int b = threadIdx.x + NT * q;
    if (b < nb) {
      const int p = b >= LR ? 1 : 0;
      const int j = b - p * LR;
      const int k = j & (ns - 1);
      cplx<T>* dst = buf + p * L + ((j >> lns) << lns) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * ns] = v[q][r];
    }
  }
  __syncthreads();
}

// Forward DFT of nseq (1 or 2) sequences of length L held back to back in
// `buf` (LDS), in place.  nseq * L <= 2 * blockDim.x * 4 is required (at most
// four radix-2 butterflies per thread).  Every thread of the block must call
// it; it begins and ends with a barrier.
template <typename T>
__device__ __forceinline__ void fft_lds(cplx<T>* buf, int nseq, int L, int nst, const int* rad,
                                        const int* lns,
                        const int* tws, const cplx<T>* tw) {
  __syncthreads();
#pragma unroll 1
  for (int s = 0; s < nst; ++s) {
    const int R = rad[s];
    if (R == 4) fft_stage<T, 4, 2>(buf, nseq, L, lns[s], tws[s], tw);
    else if (R == 2) fft_stage<T, 2, 4>(buf, nseq, L, lns[s], tws[s], tw);
    else fft_stage<T, 3, 3>(buf, nseq, L, lns[s], tws[s], tw);
  }
}

// Copy the half twiddle table (L/2 values) from global memory to LDS.
template <typename T>
__device__ __forceinline__ void load_twiddles(cplx<T>* dst, const cplx<T>* __restrict__ src,
                                              int L) {
  for (int m = threadIdx.x; m < (L >> 1); m += kThreads) dst[m] = src[m];
}

}  // namespace cgp
