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
// The DFT is a Stockham autosort FFT over radices {4, 3, 2} (L = 2^k or
// 3*2^k): at a stage of radix R with span Ns (product of earlier radices),
// butterfly j reads x[j + r L/R], twiddles element r by w_L^(r (j mod Ns) L/(Ns R)),
// takes an R-point DFT and writes y[(j div Ns) Ns R + (j mod Ns) + r Ns].
// Twiddles w_L^m = exp(-2 pi i m / L) come from a host-built FP64 table.
// Ping-pong LDS buffers; one barrier per stage; all threads of the block
// share the butterflies of all sequences.
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
    // u = -i h d = (h d.y, -h d.x)
    v[0] = {a0.x + s.x, a0.y + s.y};
    v[1] = {t.x + h * d.y, t.y - h * d.x};
    v[2] = {t.x - h * d.y, t.y + h * d.x};
  }
}

template <typename T, int R>
__device__ __forceinline__ void fft_stage(const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out,
                                          int nseq, int L, int Ns, const cplx<T>* __restrict__ tw) {
  const int LR = L / R;
  const int total = nseq * LR;
  const int twscale = L / (Ns * R);
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int p = t / LR;
    const int j = t - p * LR;
    const int k = j % Ns;
    const cplx<T>* src = in + p * L;
    cplx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[j + r * LR];
    if (k != 0) {
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[r * k * twscale]);
    }
    small_dft<T, R>(v);
    cplx<T>* dst = out + p * L + (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[r * Ns] = v[r];
  }
}

// Forward DFT of nseq sequences of length L held back to back in `a`.
// `b` is scratch of the same size.  Returns the buffer holding the result.
// Must be called by every thread of the block; begins and ends with a barrier.
template <typename T>
__device__ cplx<T>* fft_lds(cplx<T>* a, cplx<T>* b, int nseq, int L, int nst, const int* rad,
                            const cplx<T>* __restrict__ tw) {
  __syncthreads();
  int Ns = 1;
  for (int s = 0; s < nst; ++s) {
    const int R = rad[s];
    if (R == 4) fft_stage<T, 4>(a, b, nseq, L, Ns, tw);
    else if (R == 2) fft_stage<T, 2>(a, b, nseq, L, Ns, tw);
    else fft_stage<T, 3>(a, b, nseq, L, Ns, tw);
    __syncthreads();
    cplx<T>* t = a; a = b; b = t;
    Ns *= R;
  }
  return a;
}

}  // namespace cgp
