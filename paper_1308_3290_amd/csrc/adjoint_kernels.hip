// Reverse sweep of the adjoint CGP step, one RK3 stage per launch (one layer,
// FP64, coarsening 2 or 4), fused like the forward stage kernel.  With mu = b dt lam_in:
//   lam_in  = lin + P L^-1 R src_prev  (the previous stage's source, solved:
//             its y-solved spectra are transformed back along x here and
//             prolonged in registers, Sec. 3.1 and 4.3; absent for the first
//             stage of a sweep)
//   lout    = b lam_in + J(psi_s, mu) + inv_re Lap(mu) [+ acc]
//   src     = -J(omega_s, mu) + inv_ro J(mu, y), restricted and transformed
//             along x for the next solve (pass A of the adjoint, Sec. 3.1, 4.3)
//   acc     = a lam_in (acc_mode 0) / acc += a lam_in (1) / read into lout (2)
//   gF     += mu
// The CGP solve is self-adjoint (full weighting is a multiple of the
// transpose of bilinear prolongation, the sine transforms are symmetric), so
// the forward kernels' restriction, transforms and prolongation serve here.
// A block owns TJ coarse rows and the fine rows C j0 .. C (j0+TJ)-1; the
// source is also needed on the C-1 fine rows below them (computed here).
#include "cgp_internal.hpp"
#include "fft_lds.hpp"
#include "stencil.hpp"

namespace cgp {

template <int C, int TJ, int LC, bool PREV>
__global__ __launch_bounds__(kFusedThreads) void k_adjoint_fused(
    const MemberDesc* __restrict__ md, const int* __restrict__ grp, int ng, int nblk,
    const double* __restrict__ wt2, double* __restrict__ wnext,
    const cplx<double>* __restrict__ twg, const double* __restrict__ lin,
    const double* __restrict__ ws, const double* __restrict__ psi, double* __restrict__ lout,
    double* __restrict__ acc, double* __restrict__ gF, double a, double b, int acc_mode) {
  using T = double;
  constexpr int NT = kFusedThreads;
  constexpr int NR = C * TJ + 1;      // the most own fine rows (+1: top wall row)
  constexpr int E = C - 1;            // computed rows below the block
  constexpr int NO = NR + E;          // the most computed rows
  constexpr int NP = NO + 2;          // tile rows: computed rows and one on each side
  constexpr int NRT = C * (TJ + 1) - 1;  // rows of the restriction stencils
  constexpr T kInvC2 = T(1) / T(C * C);
  static_assert(kFusedMaxNx - 1 <= NT, "one fine column per thread");
  extern __shared__ __align__(16) unsigned char smem[];
  const int t = threadIdx.x;
  const int bid = xcd_contiguous(blockIdx.x, nblk);
  const MemberDesc& d = md[group_member(md, grp, ng, PASS_CD, bid)];
  const int lb = bid - d.blk0[PASS_CD];
  // a compile-time transform length fixes the row sizes (Lr = 2 Mx, nx = C Mx)
  const int Mx = LC ? LC / 2 : d.Mx, My = d.My, L = LC ? LC : d.Lr;
  const int nx = LC ? C * (LC / 2) : d.nx, ny = d.ny, pitch = nx + 1;
  const int LP = lpad(L);
  const int ntw = d.ntw_r;
  const int j0 = lb * TJ;
  const int last = (lb == d.nblk[PASS_CD] - 1);
  const int R0 = C * j0;
  const int R1 = last ? ny + 1 : C * (j0 + TJ);
  const int nfr = R1 - R0;
  const int RB0 = R0 - 1 - E;  // fine row of tile row 0 (tile row u = fine row C (j0-1) + u)
  const int prow = Mx + 1;

  // LDS: [ transform buffers | restriction rows ] [ twiddles ] [ coarse rows ]
  const int region = (max(4 * LP * (int)sizeof(cplx<T>), NRT * pitch * (int)sizeof(T)) + 15) & ~15;
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem);
  T* rt = reinterpret_cast<T*>(smem);
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem + region);
  T* psc = reinterpret_cast<T*>(tw + ntw);

  for (int m = t; m < ntw; m += NT) tw[m] = twg[d.twr_off + m];

  // ---- previous source solved: coarse rows j0-1 .. j0+TJ (zero walls) in psc
  if constexpr (PREV) {
    const int rlo = max(1, j0 - 1);
    const int ilo = rlo - ((rlo & 1) ? 0 : 1);
    const int rhi = min(My - 1, j0 + TJ);
    const int ihi = min(My - 1, rhi + (rhi & 1));
    const int nint = ihi >= ilo ? ihi - ilo + 1 : 0;
    const int nseq = (nint + 1) / 2;
    const T* w = wt2 + d.wt_off;
    if (t < nseq) {
      buf[t * LP + pad(0)] = {T(0), T(0)};
      buf[t * LP + pad(Mx)] = {T(0), T(0)};
    }
    const int k = 1 + t;
    if (k < Mx) {
      const T* col = w + (size_t)(k - 1) * (My - 1) + (ilo - 1);
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        if (p < nseq) {
          const T v0 = 2 * p < nint ? col[2 * p] : T(0);
          const T v1 = 2 * p + 1 < nint ? col[2 * p + 1] : T(0);
          buf[p * LP + pad(k)] = {v0, v1};
          buf[p * LP + pad(2 * Mx - k)] = {-v0, -v1};
        }
      }
    }
    const cplx<T>* Z = fft_run<T, LC, NT>(buf, buf + 2 * LP, nseq, L, d.nst_r, d.stw_r, tw);
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
  }
  __syncthreads();

  // ---- walls of the own rows
  T* LO = lout + d.field_off;
  T* AC = acc + d.field_off;
  if (t < nfr) {
    LO[(size_t)(R0 + t) * pitch] = T(0);
    if (acc_mode == 0) AC[(size_t)(R0 + t) * pitch] = T(0);
  } else if (t >= 64 && t < 64 + nfr) {
    LO[(size_t)(R0 + t - 64) * pitch + nx] = T(0);
    if (acc_mode == 0) AC[(size_t)(R0 + t - 64) * pitch + nx] = T(0);
  }

  // ---- the stage's adjoint on the computed rows, one fine column per thread
  const int x = 1 + t;
  const T cj = d.cj, cb = d.cb, idx2 = d.idx2, idy2 = d.idy2, nu = d.inv_re;
  const T bdt = b * d.dt;
  const T* LI = lin + d.field_off;
  const T* WS = ws + d.field_off;
  const T* PS = psi + d.field_off;
  T* GF = gF + d.field_off;
  T src[NO];
#pragma unroll
  for (int u = 0; u < NO; ++u) src[u] = T(0);
  if (x < nx) {
    // the prolonged solve at columns x-1 .. x+1 (as the forward kernel)
    T P[3][NP];
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
#pragma unroll
      for (int u = 0; u < NP; ++u) P[dx][u] = T(0);
      if constexpr (PREV) {
        const int xx = x - 1 + dx;
        T cv[TJ + 2];
        if constexpr (C == 1) {
#pragma unroll
          for (int r = 0; r < TJ + 2; ++r) cv[r] = psc[r * prow + xx];
        } else {
          const int I = xx / C, fx = xx - I * C;
          const T a0 = T(C - fx) * kInvC2, a1 = T(fx) * kInvC2;
          const T* p0 = psc + I;
          const T* p1 = psc + min(I + 1, Mx);
#pragma unroll
          for (int r = 0; r < TJ + 2; ++r) cv[r] = a0 * p0[r * prow] + a1 * p1[r * prow];
        }
#pragma unroll
        for (int u = 0; u < NP; ++u) {
          const int jr = u / C, fy = u - jr * C;
          const T top = jr + 1 < TJ + 2 ? cv[jr + 1 < TJ + 2 ? jr + 1 : TJ + 1] : T(0);
          P[dx][u] = T(C - fy) * cv[jr < TJ + 2 ? jr : TJ + 1] + T(fy) * top;
        }
      }
    }
    // lam_in (ring and rows outside 1 .. ny-1 read as 0) times b dt
    const bool mw = x > 1, me = x < nx - 1;
    auto murow = [&](int u, T& m0, T& m1, T& m2) {
      const int rr = RB0 + u;
      const bool in = rr >= 1 && rr <= ny - 1;
      const T* p = LI + (size_t)(in ? rr : 0) * pitch + x;
      const T l0 = (in && mw) ? p[-1] + P[0][u] : T(0);
      const T l1 = in ? p[0] + P[1][u] : T(0);
      const T l2 = (in && me) ? p[1] + P[2][u] : T(0);
      m0 = bdt * l0;
      m1 = bdt * l1;
      m2 = bdt * l2;
    };
    auto wrow = [&](const T* f, int u, T& w0, T& w1, T& w2) {
      const int rr = RB0 + u;
      const bool in = rr >= 1 && rr <= ny - 1;
      const T* p = f + (size_t)(in ? rr : 0) * pitch + x;
      w0 = (in && mw) ? p[-1] : T(0);
      w1 = in ? p[0] : T(0);
      w2 = (in && me) ? p[1] : T(0);
    };
    T ms0, ms1, ms2, mc0, mc1, mc2, ws0, ws1, ws2, wc0, wc1, wc2;
    murow(0, ms0, ms1, ms2);
    murow(1, mc0, mc1, mc2);
    wrow(WS, 0, ws0, ws1, ws2);
    wrow(WS, 1, wc0, wc1, wc2);
#pragma unroll
    for (int u = 1; u < NO; ++u) {
      T mn0, mn1, mn2, wn0, wn1, wn2;
      murow(u + 1, mn0, mn1, mn2);
      wrow(WS, u + 1, wn0, wn1, wn2);
      const int rr = RB0 + u;
      const bool in = rr >= 1;  // rr <= ny - 1 holds for u < NO
      Nbr<T> mu, w;
      mu.C = mc1; mu.E = mc2; mu.W = mc0; mu.N = mn1; mu.S = ms1;
      mu.NE = mn2; mu.NW = mn0; mu.SE = ms2; mu.SW = ms0;
      w.C = wc1; w.E = wc2; w.W = wc0; w.N = wn1; w.S = ws1;
      w.NE = wn2; w.NW = wn0; w.SE = ws2; w.SW = ws0;
      const T s = -cj * arakawa12(w, mu) + cb * beta3(mu);
      src[u - 1] = in ? s : T(0);
      if (u > E) {  // own row
        const size_t o = (size_t)rr * pitch + x;
        T lo = T(0);
        if (in) {
          const Nbr<T> p = load_nbr(PS, pitch, x, rr);
          const T lc = LI[o] + P[1][u];  // lam_in at the node
          lo = b * lc + cj * arakawa12(p, mu) + nu * lap5(mu, idx2, idy2);
          if (acc_mode == 0) AC[o] = a * lc;
          else if (acc_mode == 1) AC[o] += a * lc;
          else lo += AC[o];
          GF[o] += mu.C;
        } else if (acc_mode == 0) {
          AC[o] = T(0);
        }
        LO[o] = lo;
      }
      ms0 = mc0; ms1 = mc1; ms2 = mc2; mc0 = mn0; mc1 = mn1; mc2 = mn2;
      ws0 = wc0; ws1 = wc1; ws2 = wc2; wc0 = wn0; wc1 = wn1; wc2 = wn2;
    }
    if (last) {  // the top wall row
      LO[(size_t)ny * pitch + x] = T(0);
      if (acc_mode == 0) AC[(size_t)ny * pitch + x] = T(0);
    }
  }

  // ---- the source on the block's coarse rows: restriction (rows of rt =
  // fine rows R0-E ..) and forward x transform into wnext
  __syncthreads();  // the transform buffers are free
  if (x < nx) {
#pragma unroll
    for (int k = 0; k < NRT; ++k) rt[k * pitch + x] = src[k];
  }
  if (t == 0) {
#pragma unroll
    for (int k = 0; k < NRT; ++k) {
      rt[k * pitch] = T(0);
      rt[k * pitch + nx] = T(0);
    }
  }
  __syncthreads();
  const int i = 1 + t;
  cplx<T> z = {T(0), T(0)};
  if (i < Mx) {
    T racc[NRT];
#pragma unroll
    for (int q = 0; q < NRT; ++q) {
      const T* row = rt + q * pitch + C * i;
      T s = T(0);
#pragma unroll
      for (int dx = -(C - 1); dx <= C - 1; ++dx) s += T(C - (dx < 0 ? -dx : dx)) * row[dx];
      racc[q] = s;
    }
    T v[2] = {T(0), T(0)};
#pragma unroll
    for (int r = 0; r < TJ; ++r) {
      T s = T(0);
#pragma unroll
      for (int dy = -(C - 1); dy <= C - 1; ++dy)
        s += T(C - (dy < 0 ? -dy : dy)) * racc[C * r + dy + (C - 1)];
      v[r] = s * (T(1) / T(C * C * C * C));
    }
    z = {j0 >= 1 ? v[0] : T(0), v[1]};
  }
  __syncthreads();  // rt is read
  if (i < Mx) {
    buf[pad(i)] = z;
    buf[pad(2 * Mx - i)] = {-z.x, -z.y};
  }
  if (t == 0) {
    buf[pad(0)] = {T(0), T(0)};
    buf[pad(Mx)] = {T(0), T(0)};
  }
  const cplx<T>* Z2 = fft_run<T, LC, NT>(buf, buf + LP, 1, L, d.nst_r, d.stw_r, tw);
  if (i < Mx) {
    const cplx<T> zk = Z2[pad(i)];
    T* wo = wnext + d.wt_off + (size_t)(i - 1) * (My - 1);
#pragma unroll
    for (int r = 0; r < TJ; ++r) {
      const int j = j0 + r;
      if (j >= 1 && j <= My - 1) wo[j - 1] = r == 0 ? T(-0.5) * zk.y : T(0.5) * zk.x;
    }
  }
}

// g.L = (c << 16) | transform length with a compile-time transform (or 0)
hipError_t AdjLaunch::fused(const MemberDesc* md, const Group& g, const double* wt2,
                            double* wnext, const cplx<double>* tw, const double* lin,
                            const double* ws, const double* psi, double* lout, double* acc,
                            double* gF, double a, double b, int acc_mode, hipStream_t s) {
#define LAUNCH(C, TJ, LC, PV)                                                                   \
  hipLaunchKernelGGL((k_adjoint_fused<C, TJ, LC, PV>), dim3(g.nblk), dim3(kFusedThreads), g.lds, \
                     s, md, g.members, g.count, g.nblk, wt2, wnext, tw, lin, ws, psi, lout, acc, \
                     gF, a, b, acc_mode)
#define BY_LEN(C, TJ, PV)                        \
  switch (g.L & 0xffff) {                        \
    case 128: LAUNCH(C, TJ, 128, PV); break;     \
    case 256: LAUNCH(C, TJ, 256, PV); break;     \
    case 512: LAUNCH(C, TJ, 512, PV); break;     \
    default: LAUNCH(C, TJ, 0, PV);               \
  }
#define BY_C(PV)                          \
  switch (g.L >> 16) {                    \
    case 2: BY_LEN(2, 2, PV); break;      \
    case 4: BY_LEN(4, 1, PV); break;      \
    default: return hipErrorInvalidValue; \
  }
  if (wt2) {
    BY_C(true)
  } else {
    BY_C(false)
  }
#undef BY_C
#undef BY_LEN
#undef LAUNCH
  return hipGetLastError();
}

hipError_t AdjLaunch::prepare_fused(size_t bytes) {
  const int b = (int)bytes;
  const void* fns[] = {
#define K(C, TJ, LC) reinterpret_cast<const void*>(&k_adjoint_fused<C, TJ, LC, false>), \
                     reinterpret_cast<const void*>(&k_adjoint_fused<C, TJ, LC, true>)
      K(2, 2, 0), K(2, 2, 128), K(2, 2, 256), K(2, 2, 512), K(4, 1, 0), K(4, 1, 128),
      K(4, 1, 256), K(4, 1, 512)
#undef K
  };
  for (const void* f : fns) {
    const hipError_t e = allow_dynamic_lds(f, b);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace cgp
