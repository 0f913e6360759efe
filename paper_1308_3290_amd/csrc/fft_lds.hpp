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
// The DFT is a Stockham autosort FFT over radices 8, 4 and 2 with the
// radix-3 stage of L = 3*2^k placed last, so that the span Ns of every stage
// is a power of two and all index arithmetic is shifts and masks.  Shorter
// transforms use radix 4 (one radix-8 or radix-2 stage first when the power
// of two is odd): a block then has L/4 butterflies per sequence in flight,
// enough to occupy its four SIMDs.  Long enough ones have enough
// butterflies at radix 8, which needs fewer stages (each stage moves the
// whole sequence through LDS once); where that starts depends on the
// sequences per block (stage_plan).  At a stage
// of radix R, butterfly j reads x[j + r L/R], twiddles element r by
// w_L^(r (j mod Ns) L/(Ns R)), takes an R-point DFT and writes
// y[(j div Ns) Ns R + (j mod Ns) + r Ns].  Stages ping-pong between two LDS
// buffers with one barrier each; the stage loop is a runtime loop (compact
// code).  Twiddles come from per-stage tables built on the host in FP64:
// stage s keeps, for r = 1..R-1, the values w^(r k L/(Ns R)) for k < Ns
// contiguously in k, so that neighbouring butterflies read neighbouring
// entries.  A block transforms one or two sequences (nseq <= 2) with
// nseq * L <= 2048.
//
// LDS layout: element i of sequence p sits at p * lpad(L) + pad(i), with one
// padding slot after every 8 elements, which spreads the stride-8 and
// stride-64 write patterns of the first stages over all LDS banks.
#pragma once

#include "cgp_internal.hpp"

namespace cgp {

__host__ __device__ constexpr int pad(int i) { return i + (i >> 3); }
__host__ __device__ constexpr int lpad(int L) { return L + (L >> 3); }

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }

// 4-point DFT of v[0], v[S], v[2S], v[3S] in place, natural order.
template <typename T, int S>
__device__ __forceinline__ void dft4s(cplx<T>* v) {
  const cplx<T> s02 = cadd(v[0], v[2 * S]), d02 = csub(v[0], v[2 * S]);
  const cplx<T> s13 = cadd(v[S], v[3 * S]), e = csub(v[S], v[3 * S]);
  const cplx<T> d13 = {e.y, -e.x};  // -i (v1 - v3)
  v[0] = cadd(s02, s13);
  v[2 * S] = csub(s02, s13);
  v[S] = cadd(d02, d13);
  v[3 * S] = csub(d02, d13);
}

template <typename T, int R>
__device__ __forceinline__ void small_dft(cplx<T>* v) {
  if constexpr (R == 2) {
    const cplx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    dft4s<T, 1>(v);
  } else if constexpr (R == 8) {
    // n = 2 n1 + n2, k = k1 + 4 k2: two 4-point DFTs, twiddles w8^(n2 k1), 2-point DFTs
    const T h = T(0.70710678118654752440084436210484904);
    dft4s<T, 2>(v);
    dft4s<T, 2>(v + 1);
    v[3] = cmul(v[3], cplx<T>{h, -h});
    v[5] = cplx<T>{v[5].y, -v[5].x};
    v[7] = cmul(v[7], cplx<T>{-h, -h});
    cplx<T> o[8];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      o[k1] = cadd(v[2 * k1], v[2 * k1 + 1]);
      o[k1 + 4] = csub(v[2 * k1], v[2 * k1 + 1]);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = o[k];
  } else {  // R == 3, w = exp(-2 pi i / 3) = -1/2 - i sqrt(3)/2
    const T h = T(0.8660254037844386467637231707529362);
    const cplx<T> a0 = v[0], s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
    const cplx<T> t = {a0.x - T(0.5) * s.x, a0.y - T(0.5) * s.y};
    v[0] = cadd(a0, s);
    v[1] = {t.x + h * d.y, t.y - h * d.x};
    v[2] = {t.x - h * d.y, t.y + h * d.x};
  }
}

// One stage of radix R (span Ns = 2^lns) over nseq sequences of length L,
// from `in` to `out` (padded layout); `tw` is this stage's twiddle table
// ((R-1) x Ns).  Thread t of NT owns butterflies b = t + NT q, q < MAXB.
template <typename T, int R, int MAXB, int NT>
__device__ __forceinline__ void fft_stage(const cplx<T>* in, cplx<T>* out, int nseq, int L,
                                          int lns, const cplx<T>* tw) {
  const int LR = L / R;
  const int nb = nseq * LR;
  const int ns = 1 << lns;
  const int LP = lpad(L);
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int b = CGP_TID + NT * q;
    if (b < nb) {
      const int p = b / LR;
      const int j = b - p * LR;
      const int k = j & (ns - 1);
      const cplx<T>* src = in + p * LP;
      cplx<T> v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = src[pad(j + r * LR)];
      if (lns > 0) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[(r - 1) * ns + k]);
      }
      small_dft<T, R>(v);
      cplx<T>* dst = out + p * LP;
      const int o = ((j >> lns) << lns) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[pad(o + r * ns)] = v[r];
    }
  }
  __syncthreads();
}

// Stage word: radix (bits 0-3), log2 span (bits 4-8), twiddle offset (bits 9+).
__host__ __device__ constexpr int stage_word(int R, int lns, int two) {
  return R | (lns << 4) | (two << 9);
}

// Stage plan of a complex FFT of length L = 2^k or 3*2^k.  L < wide: for odd
// k one radix-8 stage first (radix 2 when k = 1), then radix 4.  L >= wide:
// radix 8 while possible, then 4, then 2.  The radix 3 comes last, so that
// every stage's span Ns (the product of the earlier radices) is a power of
// two.  `wide` is where a block has enough radix-8 butterflies per stage to
// keep its four SIMDs busy: kWideRows for the row transforms (two or three
// sequences per 512-thread block), kWideCols for the column transform (one
// sequence per 256-thread block: L/8 >= 256 from L = 2048 on).  The first
// stage has no twiddles (Ns = 1).  Stage s has radix R[s], span 2^lns[s] and
// its twiddle table ((R-1) x Ns values) at off[s]; ntw is the total table
// size.  Shared by the host (tables, stage words) and the compile-time
// transforms below.
struct StagePlan {
  int n = 0, ntw = 0;
  int R[kMaxStages] = {}, lns[kMaxStages] = {}, off[kMaxStages] = {};
};

constexpr int kWideRows = 1024;
constexpr int kWideCols = 2048;

__host__ __device__ constexpr StagePlan stage_plan(int L, int wide_from = kWideRows) {
  StagePlan p{};
  int rest = L, ns = 1, lg = 0, e = 0;
  while (rest % 2 == 0) {
    rest /= 2;
    ++e;
  }
  const bool wide = L >= wide_from;
  while (e > 0 && p.n < kMaxStages) {
    // log2 of this stage's radix
    const int lr = wide ? (e >= 3 ? 3 : e) : ((e & 1) ? (e >= 3 ? 3 : 1) : 2);
    const int R = 1 << lr;
    p.R[p.n] = R;
    p.lns[p.n] = lg;
    p.off[p.n] = p.ntw;
    p.ntw += (R - 1) * ns;
    ns *= R;
    lg += lr;
    e -= lr;
    ++p.n;
  }
  if (rest == 3 && p.n < kMaxStages) {
    p.R[p.n] = 3;
    p.lns[p.n] = lg;
    p.off[p.n] = p.ntw;
    p.ntw += 2 * ns;
    ++p.n;
  }
  return p;
}

// Forward DFT of nseq sequences of length L held back to back in buffer a
// (LDS, padded layout; nseq L <= 2048 for 256 threads, <= 3072 for 512); b
// is scratch of the same size.  Returns the
// buffer holding the result.  Every thread of the block (NT threads) must
// call it; it begins and ends with a barrier.
template <typename T, int NT = kThreads>
__device__ __forceinline__ cplx<T>* fft_lds(cplx<T>* a, cplx<T>* b, int nseq, int L, int nst,
                                            const int* words, const cplx<T>* tw) {
  int w[kMaxStages];
#pragma unroll
  for (int s = 0; s < kMaxStages; ++s) w[s] = words[s];
  __syncthreads();
#pragma unroll 1
  for (int s = 0; s < nst; ++s) {
    const int word = w[s];
    const int R = word & 15, lns = (word >> 4) & 31;
    const cplx<T>* t = tw + (word >> 9);
    if (R == 8) fft_stage<T, 8, 1, NT>(a, b, nseq, L, lns, t);
    else if (R == 4) fft_stage<T, 4, 2, NT>(a, b, nseq, L, lns, t);
    else if (R == 2) fft_stage<T, 2, 4, NT>(a, b, nseq, L, lns, t);
    else fft_stage<T, 3, 3, NT>(a, b, nseq, L, lns, t);
    cplx<T>* x = a;
    a = b;
    b = x;
  }
  return a;
}

// ---------------------------------------------------------------------------
// Compile-time transforms for the common lengths.  The stage plan, strides
// and twiddle offsets are constants, so that every LDS address of a butterfly
// is a per-thread base plus an immediate offset: the padded index of
// j + r L/R is pad(j) + r lpad(L/R) (L/R is a multiple of 8), and that of the
// output o + r Ns is pad(o) + r Ns + floor(r Ns / 8).  The latter holds for
// every power-of-two span: o is a multiple of Ns R plus k < Ns, so o + r Ns
// crosses a multiple of 8 exactly where r Ns does.
// ---------------------------------------------------------------------------
// Twiddles in registers (RT = true below): a thread loads, once, the R-1
// twiddles of each of its butterflies of every stage after the first, so
// that the stages read no twiddle table from LDS (and the block needs no LDS
// for it).  reg_tw_base(s) is where stage s's values start in the thread's
// array, reg_tw_count() its length.
template <int L, int NT, int MAXSEQ, int WF>
__host__ __device__ constexpr int reg_tw_base(int s) {
  const StagePlan P = stage_plan(L, WF);
  int n = 0;
  for (int u = 1; u < s; ++u) n += ((MAXSEQ * (L / P.R[u]) + NT - 1) / NT) * (P.R[u] - 1);
  return n;
}
template <int L, int NT, int MAXSEQ, int WF>
__host__ __device__ constexpr int reg_tw_count() {
  return reg_tw_base<L, NT, MAXSEQ, WF>(stage_plan(L, WF).n);
}

// Loads stages S .. n-1 of the register twiddles from the stage tables tab
// (global memory, the layout the LDS tables have).
template <typename T, int L, int S, int NT, int MAXSEQ, int WF>
__device__ __forceinline__ void reg_tw_load(cplx<T>* v, const cplx<T>* __restrict__ tab,
                                            int nseq) {
  constexpr StagePlan P = stage_plan(L, WF);
  if constexpr (S < P.n) {
    constexpr int R = P.R[S], NS = 1 << P.lns[S], OFF = P.off[S], LR = L / R;
    constexpr int Q = (MAXSEQ * LR + NT - 1) / NT;
    constexpr int BASE = reg_tw_base<L, NT, MAXSEQ, WF>(S);
    const int nb = nseq * LR;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int b = CGP_TID + NT * q;
      const int bb = b < nb ? b : 0;
      const int j = bb - (bb / LR) * LR;
      const int k = j & (NS - 1);
#pragma unroll
      for (int r = 1; r < R; ++r) v[BASE + q * (R - 1) + r - 1] = tab[OFF + (r - 1) * NS + k];
    }
    reg_tw_load<T, L, S + 1, NT, MAXSEQ, WF>(v, tab, nseq);
  }
}

template <typename T, int L, int S, int NT, int MAXSEQ, int WF, bool RT = false>
__device__ __forceinline__ void ct_stage(const cplx<T>* in, cplx<T>* out, int nseq,
                                         const cplx<T>* tw) {
  constexpr StagePlan P = stage_plan(L, WF);
  constexpr int R = P.R[S], LNS = P.lns[S], NS = 1 << LNS, OFF = P.off[S];
  constexpr int LR = L / R, LP = lpad(L), RS = lpad(LR);
  static_assert(LR % 8 == 0, "read offsets need L/R to be a multiple of 8");
  static_assert((NS & (NS - 1)) == 0, "write offsets need a power-of-two span");
  constexpr int Q = (MAXSEQ * LR + NT - 1) / NT;  // nseq <= MAXSEQ
  const int nb = nseq * LR;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int b = CGP_TID + NT * q;
    if (b < nb) {
      const int p = b / LR;
      const int j = b - p * LR;
      const int k = j & (NS - 1);
      const cplx<T>* src = in + p * LP + pad(j);
      cplx<T> v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = src[r * RS];
      if constexpr (NS > 1) {
        if constexpr (RT) {
          constexpr int BASE = reg_tw_base<L, NT, MAXSEQ, WF>(S);
#pragma unroll
          for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[BASE + q * (R - 1) + r - 1]);
        } else {
          const cplx<T>* t = tw + OFF + k;
#pragma unroll
          for (int r = 1; r < R; ++r) v[r] = cmul(v[r], t[(r - 1) * NS]);
        }
      }
      small_dft<T, R>(v);
      const int o = ((j >> LNS) << LNS) * R + k;
      cplx<T>* dst = out + p * LP + pad(o);
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * NS + ((r * NS) >> 3)] = v[r];
    }
  }
  __syncthreads();
}

// The same stage in place (one buffer, half the LDS of a ping-pong pair): a
// thread reads the inputs of all its butterflies, a barrier, then it writes
// their outputs (the arithmetic, and so the bits, of ct_stage).
template <typename T, int L, int S, int NT, int MAXSEQ, int WF>
__device__ __forceinline__ void ct_stage_inplace(cplx<T>* buf, int nseq, const cplx<T>* tw) {
  constexpr StagePlan P = stage_plan(L, WF);
  constexpr int R = P.R[S], LNS = P.lns[S], NS = 1 << LNS, OFF = P.off[S];
  constexpr int LR = L / R, LP = lpad(L), RS = lpad(LR);
  static_assert(LR % 8 == 0, "read offsets need L/R to be a multiple of 8");
  static_assert((NS & (NS - 1)) == 0, "write offsets need a power-of-two span");
  constexpr int Q = (MAXSEQ * LR + NT - 1) / NT;
  const int nb = nseq * LR;
  cplx<T> v[Q][R];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int b = CGP_TID + NT * q;
    if (b < nb) {
      const int p = b / LR;
      const int j = b - p * LR;
      const cplx<T>* src = buf + p * LP + pad(j);
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = src[r * RS];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int b = CGP_TID + NT * q;
    if (b < nb) {
      const int p = b / LR;
      const int j = b - p * LR;
      const int k = j & (NS - 1);
      if constexpr (NS > 1) {
        const cplx<T>* t = tw + OFF + k;
#pragma unroll
        for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], t[(r - 1) * NS]);
      }
      small_dft<T, R>(v[q]);
      const int o = ((j >> LNS) << LNS) * R + k;
      cplx<T>* dst = buf + p * LP + pad(o);
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * NS + ((r * NS) >> 3)] = v[q][r];
    }
  }
  __syncthreads();
}

template <typename T, int L, int S, int NT, int MAXSEQ, int WF>
__device__ __forceinline__ void ct_stages_inplace(cplx<T>* buf, int nseq, const cplx<T>* tw) {
  if constexpr (S < stage_plan(L, WF).n) {
    ct_stage_inplace<T, L, S, NT, MAXSEQ, WF>(buf, nseq, tw);
    ct_stages_inplace<T, L, S + 1, NT, MAXSEQ, WF>(buf, nseq, tw);
  }
}

// Compile-time transform of up to four sequences in place in buf (L = LC);
// begins and ends with a barrier.
template <typename T, int LC, int NT>
__device__ __forceinline__ cplx<T>* fft_run4_inplace(cplx<T>* buf, int nseq, const cplx<T>* tw) {
  static_assert(LC != 0, "in place: a compile-time length");
  __syncthreads();
  ct_stages_inplace<T, LC, 0, NT, 4, kWideRows>(buf, nseq, tw);
  return buf;
}

// Stages S .. SEND-1, ping-ponging between a and b; returns the buffer that
// holds the output of stage SEND-1 (a when S == SEND).
template <typename T, int L, int S, int SEND, int NT, int MAXSEQ, int WF, bool RT = false>
__device__ __forceinline__ cplx<T>* ct_stage_range(cplx<T>* a, cplx<T>* b, int nseq,
                                                   const cplx<T>* tw) {
  if constexpr (S == SEND) {
    return a;
  } else {
    ct_stage<T, L, S, NT, MAXSEQ, WF, RT>(a, b, nseq, tw);
    return ct_stage_range<T, L, S + 1, SEND, NT, MAXSEQ, WF, RT>(b, a, nseq, tw);
  }
}

template <typename T, int L, int S, int NT, int MAXSEQ, int WF>
__device__ __forceinline__ cplx<T>* ct_stages(cplx<T>* a, cplx<T>* b, int nseq,
                                              const cplx<T>* tw) {
  return ct_stage_range<T, L, S, stage_plan(L, WF).n, NT, MAXSEQ, WF>(a, b, nseq, tw);
}

// ---------------------------------------------------------------------------
// Compile-time transforms whose last stage hands its outputs to a store
// callable instead of writing LDS, e.g. straight to global memory or into
// another LDS buffer with a pointwise map: that saves the LDS pass and the
// barrier of a separate copy.  st(p, m, v, q, r) receives output m of
// sequence p; it is output r of the thread's q-th butterfly of the last
// stage, m = j + r L/R for that butterfly's index j < L/R.  The last stage
// ends without a barrier.
// ---------------------------------------------------------------------------
template <typename T, int L, int NT, int MAXSEQ, int WF, bool RT, class St>
__device__ __forceinline__ void ct_stage_last(const cplx<T>* in, int nseq, const cplx<T>* tw,
                                              St&& st) {
  constexpr StagePlan P = stage_plan(L, WF);
  constexpr int S = P.n - 1;
  constexpr int R = P.R[S], NS = 1 << P.lns[S], OFF = P.off[S];
  constexpr int LR = L / R, LP = lpad(L), RS = lpad(LR);
  static_assert(LR == NS, "the last stage spans the whole sequence");
  static_assert(LR % 8 == 0, "read offsets need L/R to be a multiple of 8");
  constexpr int Q = (MAXSEQ * LR + NT - 1) / NT;
  const int nb = nseq * LR;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int b = CGP_TID + NT * q;
    if (b < nb) {
      const int p = b / LR;
      const int j = b - p * LR;  // = j mod Ns
      const cplx<T>* src = in + p * LP + pad(j);
      cplx<T> v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = src[r * RS];
      if constexpr (RT) {
        constexpr int BASE = reg_tw_base<L, NT, MAXSEQ, WF>(S);
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[BASE + q * (R - 1) + r - 1]);
      } else {
        const cplx<T>* t = tw + OFF + j;
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], t[(r - 1) * NS]);
      }
      small_dft<T, R>(v);
#pragma unroll
      for (int r = 0; r < R; ++r) st(p, j + r * NS, v[r], q, r);
    }
  }
}

// A forward transform's last stage followed, in registers, by a pointwise
// map and the first stage of a second transform with the same plan, for
// plans whose first and last radix agree (the last stage's butterfly j
// gives outputs j + r L/R, exactly the inputs of the first stage's
// butterfly j): no pass through LDS between the two transforms.  in: the
// input of the forward's last stage; out: receives the second transform's
// first-stage output (padded layout, as ct_stage writes it); map(m, z, q, r)
// gives the second transform's input at index m from the forward output z
// at m, output r of the thread's q-th butterfly.  Register twiddles (RT) of
// the forward's last stage; the first stage has none.  Ends with a barrier.
template <int L, int WF>
__host__ __device__ constexpr bool ct_can_merge_ends() {
  if constexpr (L == 0) {
    return false;  // the runtime engine
  } else {
    constexpr StagePlan P = stage_plan(L, WF);
    return P.n >= 3 && P.R[0] == P.R[P.n - 1];
  }
}

template <typename T, int L, int NT, int WF, class Map>
__device__ __forceinline__ void ct_last_map_first(const cplx<T>* in, cplx<T>* out,
                                                  const cplx<T>* rtw, Map&& map) {
  constexpr StagePlan P = stage_plan(L, WF);
  static_assert(ct_can_merge_ends<L, WF>(), "the first and the last radix must agree");
  constexpr int S = P.n - 1;
  constexpr int R = P.R[S], LR = L / R, RS = lpad(LR);
  constexpr int Q = (LR + NT - 1) / NT;
  constexpr int BASE = reg_tw_base<L, NT, 1, WF>(S);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int j = CGP_TID + NT * q;
    if (j < LR) {
      cplx<T> v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = in[pad(j) + r * RS];
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = cmul(v[r], rtw[BASE + q * (R - 1) + r - 1]);
      small_dft<T, R>(v);
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = map(j + r * LR, v[r], q, r);
      small_dft<T, R>(v);  // the first stage (span 1: no twiddles)
      cplx<T>* dst = out + pad(j * R);
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r + (r >> 3)] = v[r];
    }
  }
  __syncthreads();
}

// Whether the last stage of ct_run_to reads buffer a (else b): the n - 1
// stages before it ping-pong from a.
template <int L, int WF>
__host__ __device__ constexpr bool ct_last_reads_a() {
  return ((stage_plan(L, WF).n - 1) & 1) == 0;
}

// Input in LDS buffer a (as fft_run, which it matches bit for bit), last
// stage to st.  RT: tw is the thread's register twiddles (reg_tw_load), else
// the LDS tables.
template <typename T, int LC, int NT, int MAXSEQ, int WF, bool RT = false, class St>
__device__ __forceinline__ void ct_run_to(St&& st, cplx<T>* a, cplx<T>* b, int nseq,
                                          const cplx<T>* tw) {
  constexpr int N = stage_plan(LC, WF).n;
  static_assert(N >= 2, "the last stage follows at least one LDS stage");
  __syncthreads();
  const cplx<T>* x = ct_stage_range<T, LC, 0, N - 1, NT, MAXSEQ, WF, RT>(a, b, nseq, tw);
  ct_stage_last<T, LC, NT, MAXSEQ, WF, RT>(x, nseq, tw, st);
}

// Forward DFT with the contract of fft_lds; LC = 0 selects the runtime
// engine (any supported length), otherwise L must equal LC and the stage
// plan is stage_plan(LC, WF) (the host builds the twiddles of the same plan).
template <typename T, int LC, int NT = kThreads, int WF = kWideRows>
__device__ __forceinline__ cplx<T>* fft_run(cplx<T>* a, cplx<T>* b, int nseq, int L, int nst,
                                            const int* words, const cplx<T>* tw) {
  if constexpr (LC == 0) {
    return fft_lds<T, NT>(a, b, nseq, L, nst, words, tw);
  } else {
    __syncthreads();
    return ct_stages<T, LC, 0, NT, 2, WF>(a, b, nseq, tw);
  }
}

// Compile-time transform of up to four sequences (L = LC), same contract.
template <typename T, int LC, int NT>
__device__ __forceinline__ cplx<T>* fft_run4(cplx<T>* a, cplx<T>* b, int nseq,
                                             const cplx<T>* tw) {
  static_assert(LC != 0, "four sequences need a compile-time length");
  __syncthreads();
  return ct_stages<T, LC, 0, NT, 4, kWideRows>(a, b, nseq, tw);
}

// Up to MAXSEQ sequences, compile-time length or (LC = 0) the runtime engine.
template <typename T, int LC, int NT, int MAXSEQ>
__device__ __forceinline__ cplx<T>* fft_runn(cplx<T>* a, cplx<T>* b, int nseq, int L, int nst,
                                             const int* words, const cplx<T>* tw) {
  if constexpr (LC == 0) {
    return fft_lds<T, NT>(a, b, nseq, L, nst, words, tw);
  } else {
    __syncthreads();
    return ct_stages<T, LC, 0, NT, MAXSEQ, kWideRows>(a, b, nseq, tw);
  }
}

// Twiddle values a thread of NT prefetches for a transform of length LC (0:
// any supported length, L <= 2048).
template <int LC, int NT, int WF = kWideRows>
__host__ __device__ constexpr int tw_per_thread() {
  return ((LC ? stage_plan(LC, WF).ntw : 2047) + NT - 1) / NT;
}

// Lengths with a compile-time transform (0: none).
__host__ __device__ constexpr int fft_special(int L) {
  return (L == 128 || L == 256 || L == 384 || L == 512 || L == 768 || L == 1024 || L == 1536 ||
          L == 2048)
             ? L
             : 0;
}

// Copy n twiddle values from global memory to LDS.
template <typename T>
__device__ __forceinline__ void load_twiddles(cplx<T>* dst, const cplx<T>* __restrict__ src,
                                              int n) {
  for (int m = CGP_TID; m < n; m += kThreads) dst[m] = src[m];
}

}  // namespace cgp
