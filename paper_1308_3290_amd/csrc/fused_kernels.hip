// Pass C + D fused (one layer): inverse x sine transform of the coarse
// spectra (Sec. 4.3), bilinear prolongation (Sec. 3.1) into LDS, and the
// Arakawa right-hand side with the TVD-RK3 stage combine (Sec. 4.1, 4.2), so
// that the prolonged psi never travels through HBM.
//
// A block owns coarse rows j0 .. j0+TJ-1 and writes omega_{s+1} on the fine
// rows C*j0 .. C*(j0+TJ)-1 (the last block also the top wall row).  The
// stencil on those rows needs psi on one more fine row above and below, i.e.
// the coarse rows j0-1 .. j0+TJ, which the block synthesises itself (at most
// four rows: two complex sequences) and keeps in LDS.  Each thread then owns
// fine columns and interpolates psi at its column and both neighbours for all
// of the block's rows in registers; the row weights are compile-time
// constants.
//
// Latency: a block is the only one on its CU, so its phases do not overlap
// with other blocks.  Every global load of the block is therefore issued at
// the start: the twiddles and spectra first (the transform waits for them
// only), then the vorticity rows, the forcing and omega_n, which arrive while
// the transform runs.  Rows are at most kFusedMaxNx + 1 nodes wide.
#include "cgp_internal.hpp"
#include "fft_lds.hpp"
#include "stencil.hpp"

namespace cgp {

// C: coarsening factor; TJ: coarse rows owned per block; LC: transform
// length with a compile-time transform, or 0.
template <typename T, int C, int TJ, int LC>
__global__ __launch_bounds__(kFusedThreads) void k_prolong_stencil(
    const MemberDesc* __restrict__ md, const int* __restrict__ grp, int ng, int nblk,
    const T* __restrict__ wt, const cplx<T>* __restrict__ twg, const T* __restrict__ ws,
    const T* __restrict__ forcing, const T* __restrict__ wn, T* __restrict__ out, double a_,
    double b_) {
  constexpr int NT = kFusedThreads;
  constexpr int NR = C * TJ + 1;  // the most fine rows a block writes (+1: top wall row)
  // twiddles per thread: (R-1) Ns summed over the stages, < L <= 1024
  constexpr int kTwPer = ((LC ? stage_plan(LC).ntw : 1023) + NT - 1) / NT;
  static_assert(kFusedMaxNx - 1 <= NT, "one spectral column and one fine column per thread");
  constexpr int kWPer = ((NR + 2) * (kFusedMaxNx + 1) + NT - 1) / NT;
  extern __shared__ __align__(16) unsigned char smem[];
  const int t = threadIdx.x;
  const int bid = xcd_contiguous(blockIdx.x, nblk);
  const MemberDesc& d = md[group_member(md, grp, ng, PASS_CD, bid)];
  const int lb = bid - d.blk0[PASS_CD];
  const int Mx = d.Mx, My = d.My, L = d.Lr, c = C;
  const int nx = d.nx, ny = d.ny, pitch = nx + 1;
  const int LP = lpad(L);
  const int ntw = d.ntw_r;

  const int j0 = lb * TJ;
  const int ilo = max(1, j0 - 1);
  const int ihi = min(My - 1, j0 + TJ);
  const int nint = ihi >= ilo ? ihi - ilo + 1 : 0;
  const int nseq = (nint + 1) / 2;
  const int last = (lb == d.nblk[PASS_CD] - 1);
  const int R0 = c * j0;
  const int R1 = last ? ny + 1 : c * (j0 + TJ);  // exclusive end of the output rows
  const int nfr = R1 - R0;                       // output rows (<= NR)
  const int nW = (nfr + 2) * pitch;              // vorticity tile: rows R0-1 .. R1

  // LDS: [ FFT buffers ] [ twiddles ] [ coarse psi rows ] [ vorticity tile ]
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* tw = buf + 4 * LP;
  T* psc = reinterpret_cast<T*>(tw + ntw);
  const int prow = Mx + 1;
  T* wtile = psc + (TJ + 2) * prow;

  // ---- issue the block's global loads.  They are unconditional (a lane
  // without an element reads element 0 of the same array and discards it), so
  // that they sit in one basic block and the transform below waits only for
  // the twiddles and spectra, not for the loads issued after them.
  T twx[kTwPer], twy[kTwPer];
#pragma unroll
  for (int q = 0; q < kTwPer; ++q) {
    const int m = t + NT * q;
    const cplx<T> z = twg[d.twr_off + (m < ntw ? m : 0)];
    twx[q] = z.x;
    twy[q] = z.y;
  }
  const T* w = wt + d.wt_off;
  T sv[4];
  {
    const int k = 1 + t;
    const size_t cbase = (size_t)(k - 1) * (My - 1) + (ilo - 1);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const bool in = k < Mx && r < nint;
      const T v = w[in ? cbase + r : 0];
      sv[r] = in ? v : T(0);
    }
  }
  const T* W = ws + d.field_off;
  const T* FF = forcing + d.field_off;
  const T* WN = wn + d.field_off;
  T* O = out + d.field_off;
  const long long g0 = (long long)(R0 - 1) * pitch;
  const long long gend = (long long)(ny + 1) * pitch;
  T wv[kWPer];
#pragma unroll
  for (int q = 0; q < kWPer; ++q) {
    const int e = t + NT * q;
    const long long g = g0 + e;
    const bool in = e < nW && g >= 0 && g < gend;
    const T v = W[in ? g : 0];
    wv[q] = in ? v : T(0);
  }
  // forcing and omega_n at the thread's column x = 1 + t, rows R0 + r
  const int x = 1 + t;
  T fv[NR], nv[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int rr = R0 + r;
    const bool in = x < nx && r < nfr && rr >= 1 && rr < ny;
    const size_t o = in ? (size_t)rr * pitch + x : 0;
    const T f = FF[o], n = WN[o];
    fv[r] = in ? f : T(0);
    nv[r] = in ? n : T(0);
  }

  // ---- twiddles and the two packed sequences (odd extension) into LDS
#pragma unroll
  for (int q = 0; q < kTwPer; ++q) {
    const int m = t + NT * q;
    if (m < ntw) tw[m] = {twx[q], twy[q]};
  }
  if (t < nseq) {
    buf[t * LP + pad(0)] = {T(0), T(0)};
    buf[t * LP + pad(Mx)] = {T(0), T(0)};
  }
  if (1 + t < Mx) {
    const int k = 1 + t;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      if (p < nseq) {
        const cplx<T> z = {sv[2 * p], sv[2 * p + 1]};
        buf[p * LP + pad(k)] = z;
        buf[p * LP + pad(2 * Mx - k)] = {-z.x, -z.y};
      }
    }
  }
  const cplx<T>* Z = fft_run<T, LC, NT>(buf, buf + 2 * LP, nseq, L, d.nst_r, d.stw_r, tw);

  // ---- coarse psi rows J = j0-1 .. j0+TJ (zero walls) into psc
  for (int i = t; i <= Mx; i += NT) {
#pragma unroll
    for (int r = 0; r < TJ + 2; ++r) {
      const int J = j0 - 1 + r;
      T v = T(0);
      if (J >= 1 && J <= My - 1 && i >= 1 && i <= Mx - 1) {
        const int idx = J - ilo;
        const cplx<T> zi = Z[(idx >> 1) * LP + pad(i)];
        v = (idx & 1) ? T(0.5) * zi.x : T(-0.5) * zi.y;
      }
      psc[r * prow + i] = v;
    }
  }
#pragma unroll
  for (int q = 0; q < kWPer; ++q) {
    const int e = t + NT * q;
    if (e < nW) wtile[e] = wv[q];
  }
  __syncthreads();

  // ---- walls: columns 0 and nx of the output rows
  if (t < nfr) O[(size_t)(R0 + t) * pitch] = T(0);
  else if (t >= 64 && t < 64 + nfr) O[(size_t)(R0 + t - 64) * pitch + nx] = T(0);

  // ---- stencil + RK3 on fine rows R0 .. R1-1 (tile row q = fine row R0-1+q)
  const T dt = T(d.dt), a = T(a_), b = T(b_);
  const T cj = T(d.cj), cb = T(d.cb);
  const T idx2 = T(d.idx2), idy2 = T(d.idy2);
  const T nu = T(d.inv_re);
  constexpr T kInvC2 = T(1) / T(C * C);
  if (x < nx) {
    // coarse columns I0 .. I0+2 (clamped to the wall column Mx) cover the
    // fine columns x-1 .. x+1 for C >= 2; for C = 1 they are those columns
    const int I0 = (x - 1) / C;
    T A[3][TJ + 2];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const int I = min(I0 + m, Mx);
#pragma unroll
      for (int r = 0; r < TJ + 2; ++r) A[m][r] = psc[r * prow + I];
    }
    // P[dx][q]: psi at fine column x-1+dx, tile row q (bilinear, Sec. 3.1;
    // times C^2, scaled below)
    T P[3][NR + 2];
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      const int xx = x - 1 + dx;
      const int rel = xx / C - I0;  // 0 or 1 (0 .. 2 when C = 1)
      const int fx = xx - (xx / C) * C;
      T cv[TJ + 2];
#pragma unroll
      for (int r = 0; r < TJ + 2; ++r) {
        T lo, hi;
        if constexpr (C == 1) {
          lo = dx == 0 ? A[0][r] : (dx == 1 ? A[1][r] : A[2][r]);
          hi = T(0);
        } else {
          lo = rel == 0 ? A[0][r] : A[1][r];
          hi = rel == 0 ? A[1][r] : A[2][r];
        }
        cv[r] = T(C - fx) * lo + T(fx) * hi;
      }
#pragma unroll
      for (int q = 0; q < NR + 2; ++q) {
        // fine row R0-1+q = C*(j0-1) + (C-1+q): coarse row j0-1+jr, weight fy
        const int u = C - 1 + q;
        const int jr = u / C, fy = u - jr * C;
        const T top = jr + 1 < TJ + 2 ? cv[jr + 1 < TJ + 2 ? jr + 1 : TJ + 1] : T(0);
        P[dx][q] = (T(C - fy) * cv[jr < TJ + 2 ? jr : TJ + 1] + T(fy) * top) * kInvC2;
      }
    }
    const bool mw = x > 1, me = x < nx - 1;
    auto wrow = [&](int q, T& w0, T& w1, T& w2) {
      const int rr = R0 - 1 + q;
      const bool in = rr >= 1 && rr <= ny - 1;
      const T* p = wtile + q * pitch + x;
      w0 = (in && mw) ? p[-1] : T(0);
      w1 = in ? p[0] : T(0);
      w2 = (in && me) ? p[1] : T(0);
    };
    T ws0, ws1, ws2, wc0, wc1, wc2;
    wrow(0, ws0, ws1, ws2);
    wrow(1, wc0, wc1, wc2);
#pragma unroll
    for (int q = 1; q <= NR; ++q) {
      if (q > nfr) break;
      T wn0, wn1, wn2;
      wrow(q + 1, wn0, wn1, wn2);
      const int rr = R0 - 1 + q;
      T v = T(0);
      if (rr != 0 && rr != ny) {
        Nbr<T> p, w;
        p.C = P[1][q]; p.E = P[2][q]; p.W = P[0][q];
        p.N = P[1][q + 1]; p.S = P[1][q - 1];
        p.NE = P[2][q + 1]; p.NW = P[0][q + 1];
        p.SE = P[2][q - 1]; p.SW = P[0][q - 1];
        w.C = wc1; w.E = wc2; w.W = wc0;
        w.N = wn1; w.S = ws1;
        w.NE = wn2; w.NW = wn0;
        w.SE = ws2; w.SW = ws0;
        const T G =
            -cj * arakawa12(p, w) - cb * beta3(p) + nu * lap5(w, idx2, idy2) + fv[q - 1];
        v = b * (w.C + dt * G);
        if (a_ != 0.0) v += a * nv[q - 1];
      }
      O[(size_t)rr * pitch + x] = v;
      ws0 = wc0; ws1 = wc1; ws2 = wc2;
      wc0 = wn0; wc1 = wn1; wc2 = wn2;
    }
  }
}

// g.L = (c << 16) | transform length with a compile-time transform (or 0).
template <typename T>
hipError_t Launch<T>::prolong_stencil(const MemberDesc* md, const Group& g, const T* wt,
                                      const cplx<T>* tw, const T* ws, const T* forcing,
                                      const T* wn, T* out, double a, double b, hipStream_t s) {
#define LAUNCH(C, TJ, LC)                                                                     \
  hipLaunchKernelGGL((k_prolong_stencil<T, C, TJ, LC>), dim3(g.nblk), dim3(kFusedThreads), g.lds, \
                     s, md, g.members, g.count, g.nblk, wt, tw, ws, forcing, wn, out, a, b)
#define BY_LEN(C, TJ)                         \
  switch (g.L & 0xffff) {                     \
    case 256: LAUNCH(C, TJ, 256); break;      \
    case 512: LAUNCH(C, TJ, 512); break;      \
    case 1024: LAUNCH(C, TJ, 1024); break;    \
    default: LAUNCH(C, TJ, 0);                \
  }
  switch (g.L >> 16) {
    case 1: BY_LEN(1, 2); break;
    case 2: BY_LEN(2, 2); break;
    case 4: BY_LEN(4, 1); break;
    default: return hipErrorInvalidValue;
  }
#undef BY_LEN
#undef LAUNCH
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::prepare_fused(size_t bytes) {
  const int b = (int)bytes;
  const void* fns[] = {
#define FNS(C, TJ)                                                          \
  reinterpret_cast<const void*>(&k_prolong_stencil<T, C, TJ, 0>),           \
      reinterpret_cast<const void*>(&k_prolong_stencil<T, C, TJ, 256>),     \
      reinterpret_cast<const void*>(&k_prolong_stencil<T, C, TJ, 512>),     \
      reinterpret_cast<const void*>(&k_prolong_stencil<T, C, TJ, 1024>)
      FNS(1, 2), FNS(2, 2), FNS(4, 1)
#undef FNS
  };
  for (const void* f : fns) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template struct Launch<float>;
template struct Launch<double>;

}  // namespace cgp
