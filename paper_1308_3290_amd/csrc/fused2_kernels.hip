// Passes C + D (+ the next stage's pass A) fused for the two-layer model
// (Sec. 2.2, mode split of Sec. 4.3): a block owns TJ coarse rows and
//   1. transforms the y-solved barotropic and baroclinic spectra of the
//      coarse rows j0-1 .. j0+TJ back along x (one complex sequence per row:
//      the two modes as its real and imaginary parts) and recombines the
//      layers, psi_1 = psi_bt + (1 - delta) psi_bc, psi_2 = psi_bt - delta psi_bc;
//   2. interpolates psi_1, psi_2 bilinearly in registers (Sec. 3.1) and applies
//      both layers' right-hand sides with the TVD-RK3 stage combine (Sec. 4.1,
//      4.2): G_i = -J(psi_i, Q_i) - (1/Ro) J(psi_i, y) + (1/Re) Lap zeta_i
//      (+ F on layer 1, - drag zeta_2 on layer 2), zeta_i = Q_i - F_i (psi_j - psi_i);
//   3. with NEXT, restricts both new layers on its coarse rows, forms the
//      modes delta Q_1 + (1 - delta) Q_2 and Q_1 - Q_2, and transforms them
//      along x (one sequence per row), exactly as pass A does.
// Coarsening factors 1, 2 and 4 (at c = 1 the transfers are identities and a
// block owns one coarse row), transform lengths with a compile-time engine.
#include "cgp_internal.hpp"
#include "fft_lds.hpp"
#include "stencil.hpp"

namespace cgp {

template <typename T, int C, int TJ, int LC, bool NEXT, bool NTS>
__global__ __launch_bounds__(kFusedThreads) void k_prolong_stencil2(
    const MemberDesc* __restrict__ md, const int* __restrict__ grp, int ng, int nblk,
    const T* __restrict__ wt, T* __restrict__ wnext, const cplx<T>* __restrict__ twg,
    const T* __restrict__ ws, const T* __restrict__ forcing, const T* __restrict__ wn,
    T* __restrict__ out, double a_, double b_, StepCtl ctl) {
  static_assert(LC != 0, "two layers: compile-time transform length");
  constexpr int NT = kFusedThreads;
  constexpr int NR = C * TJ + 1;      // the most own fine rows (+1: top wall row)
  constexpr int E = NEXT ? C - 1 : 0;  // computed rows below the block
  constexpr int NO = NR + E;          // the most computed rows
  constexpr int NP = NO + 2;          // tile rows
  constexpr int OFF = C - 1 - E;      // tile row u is fine row C*(j0-1) + OFF + u
  constexpr int NS = TJ + 2;          // coarse rows synthesised (one sequence each)
  constexpr int MX = LC / 2;          // coarse intervals along x
  constexpr int PROW = MX + 1;
  constexpr int kTwPer = (stage_plan(LC).ntw + NT - 1) / NT;
  constexpr int kWPer = (NP * (kFusedMaxNx + 1) + NT - 1) / NT;
  constexpr T kInvC2 = T(1) / T(C * C);
  static_assert(kFusedMaxNx - 1 <= NT, "one spectral column and one fine column per thread");
  extern __shared__ __align__(16) unsigned char smem[];
  const int t = threadIdx.x;
  const int bid = xcd_contiguous(blockIdx.x, nblk);
  const MemberDesc& d = md[group_member(md, grp, ng, PASS_CD, bid)];
  const int lb = bid - d.blk0[PASS_CD];
  const int My = d.My;
  // the transform length fixes the row sizes (Lr = 2 Mx, nx = C Mx)
  const int nx = C * (LC / 2), ny = d.ny, pitch = nx + 1;
  const size_t plane = (size_t)(ny + 1) * pitch;
  constexpr int LP = lpad(LC);
  const int ntw = d.ntw_r;
  const int j0 = lb * TJ;
  const int last = (lb == d.nblk[PASS_CD] - 1);
  const int R0 = C * j0;
  const int R1 = last ? ny + 1 : C * (j0 + TJ);
  const int nfr = R1 - R0;
  const int nrow = nfr + E;
  const int RB0 = R0 - 1 - E;
  const int nW = (nrow + 2) * pitch;
  const size_t mplane = (size_t)(MX - 1) * (My - 1);

  // LDS: [ transform buffers | the two vorticity tiles | restriction rows and
  // the next transform's buffers ] [ twiddles ] [ coarse psi rows, 2 layers ]
  // [ restriction column sums ].  C = 1: the row transform runs in place
  // and the coarse psi rows and the tiles follow it in the first region,
  // [ transform buffer | psi rows, tiles | the next transform's buffers ]
  // [ twiddles ], which keeps a block within half a CU's LDS (two blocks per
  // CU; the 1024-point full grid otherwise runs one).
  constexpr bool INPLACE = C == 1;
  constexpr int kPsc = 2 * NS * PROW * (int)sizeof(T);
  const int region =
      INPLACE ? (max(NS * LP * (int)sizeof(cplx<T>), kPsc + 2 * NP * pitch * (int)sizeof(T)) +
                 15) & ~15
              : (max(2 * NS * LP * (int)sizeof(cplx<T>), 2 * NP * pitch * (int)sizeof(T)) + 15) &
                    ~15;
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem + region);
  T* psc1 = INPLACE ? reinterpret_cast<T*>(smem) : reinterpret_cast<T*>(tw + ntw);
  T* psc2 = psc1 + NS * PROW;
  T* tile1 = INPLACE ? reinterpret_cast<T*>(smem + kPsc) : reinterpret_cast<T*>(smem);
  T* tile2 = tile1 + NP * pitch;

  // ---- global loads (unconditional; see the one-layer pass): twiddles,
  // spectra and the vorticity tiles first, then (once the transform's inputs
  // are in LDS) forcing and omega_n, which arrive while the transform runs
  T twx[kTwPer], twy[kTwPer];
#pragma unroll
  for (int q = 0; q < kTwPer; ++q) {
    const int m = t + NT * q;
    const cplx<T> z = twg[d.twr_off + (m < ntw ? m : 0)];
    twx[q] = z.x;
    twy[q] = z.y;
  }
  const T* w = wt + d.wt_off;
  T sbt[NS], sbc[NS];
  {
    const int k = 1 + t;
#pragma unroll
    for (int r = 0; r < NS; ++r) {
      const int J = j0 - 1 + r;
      const bool in = k < MX && J >= 1 && J <= My - 1;
      const size_t o = in ? (size_t)(k - 1) * (My - 1) + (J - 1) : 0;
      const T vbt = w[o], vbc = w[mplane + o];
      sbt[r] = in ? vbt : T(0);
      sbc[r] = in ? vbc : T(0);
    }
  }
  const T* W = ws + d.field_off;
  const T* FF = forcing + d.field_off;
  const T* WN = wn + d.field_off;
  T* O = out + d.field_off;
  const long long g0 = (long long)RB0 * pitch;
  T wv1[kWPer], wv2[kWPer];
  {
    int er = t / pitch, ec = t - er * pitch;
    const int dr = NT / pitch, dc = NT - dr * pitch;
#pragma unroll
    for (int q = 0; q < kWPer; ++q) {
      const int e = t + NT * q;
      const int fr = RB0 + er;
      const bool in = e < nW && fr >= 1 && fr <= ny - 1 && ec >= 1 && ec <= nx - 1;
      const long long g = in ? g0 + e : 0;
      const T v1 = W[g], v2 = W[plane + g];
      wv1[q] = in ? v1 : T(0);
      wv2[q] = in ? v2 : T(0);
      er += dr;
      ec += dc;
      if (ec >= pitch) {
        ec -= pitch;
        ++er;
      }
    }
  }
  // ---- twiddles and the NS row sequences (odd extension) into LDS
#pragma unroll
  for (int q = 0; q < kTwPer; ++q) {
    const int m = t + NT * q;
    // with the psi rows after the table (C > 1) a thread past it writes slot
    // ntw, which they overwrite later: an unconditional store keeps the
    // twiddle load first instead of sunk behind the other loads and waited
    // for with them (the one-layer fused pass does the same)
    if constexpr (!INPLACE)
      tw[m < ntw ? m : ntw] = {twx[q], twy[q]};
    else if (m < ntw)
      tw[m] = {twx[q], twy[q]};
  }
  if (t < NS) {
    buf[t * LP + pad(0)] = {T(0), T(0)};
    buf[t * LP + pad(MX)] = {T(0), T(0)};
  }
  if (1 + t < MX) {
    const int k = 1 + t;
#pragma unroll
    for (int r = 0; r < NS; ++r) {
      buf[r * LP + pad(k)] = {sbt[r], sbc[r]};
      buf[r * LP + pad(2 * MX - k)] = {-sbt[r], -sbc[r]};
    }
  }
  const int x = 1 + t;
  T fv[NO], nv1[NO], nv2[NO];
#pragma unroll
  for (int u = 1; u <= NO; ++u) {
    const int rr = RB0 + u;
    const bool in = x < nx && u <= nrow && rr >= 1 && rr < ny;
    const size_t o = in ? (size_t)rr * pitch + x : 0;
    const T f = FF[o], n1 = WN[o], n2 = WN[plane + o];
    fv[u - 1] = in ? f : T(0);
    nv1[u - 1] = in ? n1 : T(0);
    nv2[u - 1] = in ? n2 : T(0);
  }

  // ---- coarse psi of both layers, rows j0-1 .. j0+TJ (zero walls)
  const T wbc1 = T(1.0 - d.delta), wbc2 = T(d.delta);
  if constexpr (INPLACE) {
    const cplx<T>* Z = fft_run4_inplace<T, LC, NT>(buf, NS, tw);
    constexpr int kPscIter = (MX + 1 + NT - 1) / NT;
    T pv1[kPscIter][NS], pv2[kPscIter][NS];
#pragma unroll
    for (int q = 0; q < kPscIter; ++q) {
      const int i = t + NT * q;
#pragma unroll
      for (int r = 0; r < NS; ++r) {
        const int J = j0 - 1 + r;
        T v1 = T(0), v2 = T(0);
        if (J >= 1 && J <= My - 1 && i >= 1 && i <= MX - 1) {
          const cplx<T> zi = Z[r * LP + pad(i)];
          const T bt = T(-0.5) * zi.y, bc = T(0.5) * zi.x;
          v1 = bt + wbc1 * bc;  // psi_1 = psi_bt + (1 - delta) psi_bc
          v2 = bt - wbc2 * bc;  // psi_2 = psi_bt - delta psi_bc
        }
        pv1[q][r] = v1;
        pv2[q][r] = v2;
      }
    }
    // the psi rows overwrite the transform's output: every thread reads its
    // values first (the tiles follow the psi rows and were never part of it)
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPscIter; ++q) {
      const int i = t + NT * q;
      if (i <= MX) {
#pragma unroll
        for (int r = 0; r < NS; ++r) {
          psc1[r * PROW + i] = pv1[q][r];
          psc2[r * PROW + i] = pv2[q][r];
        }
      }
    }
  } else {
    // the transform's last stage writes both layers' psi rows directly (no
    // LDS pass and barrier of a separate copy)
    __syncthreads();
    constexpr int NLAST = stage_plan(LC).n - 1;
    const cplx<T>* X =
        ct_stage_range<T, LC, 0, NLAST, NT, 4, kWideRows>(buf, buf + NS * LP, NS, tw);
    ct_stage_last<T, LC, NT, 4, kWideRows, false>(
        X, NS, tw, [&](int r, int i, cplx<T> zi, int, int) {
          const int J = j0 - 1 + r;
          if (J >= 1 && J <= My - 1 && i >= 1 && i <= MX - 1) {
            const T bt = T(-0.5) * zi.y, bc = T(0.5) * zi.x;
            psc1[r * PROW + i] = bt + wbc1 * bc;  // psi_1 = psi_bt + (1 - delta) psi_bc
            psc2[r * PROW + i] = bt - wbc2 * bc;  // psi_2 = psi_bt - delta psi_bc
          }
        });
    for (int i = t; i <= MX; i += NT) {
#pragma unroll
      for (int r = 0; r < NS; ++r) {
        const int J = j0 - 1 + r;
        if (J < 1 || J > My - 1 || i == 0 || i == MX) {
          psc1[r * PROW + i] = T(0);
          psc2[r * PROW + i] = T(0);
        }
      }
    }
    __syncthreads();  // the transform's output is consumed: the tiles may overwrite it
  }
#pragma unroll
  for (int q = 0; q < kWPer; ++q) {
    const int e = t + NT * q;
    if (e < nW) {
      tile1[e] = wv1[q];
      tile2[e] = wv2[q];
    }
  }
  __syncthreads();

  // ---- walls: columns 0 and nx of the own rows, both layers
  if (t < nfr) {
    O[(size_t)(R0 + t) * pitch] = T(0);
    O[plane + (size_t)(R0 + t) * pitch] = T(0);
  } else if (t >= 64 && t < 64 + nfr) {
    O[(size_t)(R0 + t - 64) * pitch + nx] = T(0);
    O[plane + (size_t)(R0 + t - 64) * pitch + nx] = T(0);
  }

  // ---- both layers' right-hand sides and RK3 on the computed rows
  const T dt = stage_dt<T>(d, ctl), a = T(a_), b = T(b_);
  const T cj = T(d.cj), cb = T(d.cb);
  const T idx2 = T(d.idx2), idy2 = T(d.idy2);
  const T nu = T(d.inv_re);
  const T F1 = T(d.f1), F2 = T(d.f2), drag = T(d.drag);
  T res1[NO], res2[NO];
#pragma unroll
  for (int u = 0; u < NO; ++u) {
    res1[u] = T(0);
    res2[u] = T(0);
  }
  if (x < nx) {
    // coarse psi of both layers at the coarse columns of x-1, x, x+1, with the
    // x weights (C - fx, fx)/C^2 applied
    T cv1[3][NS], cv2[3][NS];
    if constexpr (C == 2) {
      // x-1, x, x+1 lie on the coarse columns I, I+1, I+2 (I = (x-1)/2): the
      // first two on I and I+1, the last on I+1 and I+2, so three values per
      // row and layer serve all three; x-1 = 2I + odd has x weights
      // (2 - odd, odd)/4, x (1 - odd, 1 + odd)/4 on (I, I+1), x+1 the weights
      // of x-1 on (I+1, I+2); powers of two, so every sum is exact
      const int I = (x - 1) >> 1, odd = (x - 1) & 1;
      const int k1 = min(I + 1, MX), k2 = min(I + 2, MX);
      const T q = T(0.25);
      const T w0 = T(2 - odd) * q, w1 = T(odd) * q, v0 = T(1 - odd) * q, v1 = T(1 + odd) * q;
#pragma unroll
      for (int r = 0; r < NS; ++r) {
        const T a1 = psc1[r * PROW + I], b1 = psc1[r * PROW + k1], c1 = psc1[r * PROW + k2];
        const T a2 = psc2[r * PROW + I], b2 = psc2[r * PROW + k1], c2 = psc2[r * PROW + k2];
        cv1[0][r] = w0 * a1 + w1 * b1;
        cv1[1][r] = v0 * a1 + v1 * b1;
        cv1[2][r] = w0 * b1 + w1 * c1;
        cv2[0][r] = w0 * a2 + w1 * b2;
        cv2[1][r] = v0 * a2 + v1 * b2;
        cv2[2][r] = w0 * b2 + w1 * c2;
      }
    } else {
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int xx = x - 1 + dx;
        const int I = xx / C, fx = xx - I * C;
        const T a0 = T(C - fx) * kInvC2, a1 = T(fx) * kInvC2;
        const int i1 = min(I + 1, MX);
#pragma unroll
        for (int r = 0; r < NS; ++r) {
          cv1[dx][r] = a0 * psc1[r * PROW + I] + a1 * psc1[r * PROW + i1];
          cv2[dx][r] = a0 * psc2[r * PROW + I] + a1 * psc2[r * PROW + i1];
        }
      }
    }
    // psi at column x-1+dx, tile row u (compile-time y weights)
    auto pat = [&](const T (&cv)[3][NS], int dx, int u) -> T {
      const int m = OFF + u;
      const int jr = m / C, fy = m - jr * C;
      const T top = jr + 1 < NS ? cv[dx][jr + 1 < NS ? jr + 1 : NS - 1] : T(0);
      return T(C - fy) * cv[dx][jr < NS ? jr : NS - 1] + T(fy) * top;
    };
    const T* t1 = tile1 + x;
    const T* t2 = tile2 + x;
#pragma unroll
    for (int u = 1; u < NO; ++u) {
      const int rr = RB0 + u;
      Nbr<T> p1, p2, q1, q2;
      p1.C = pat(cv1, 1, u); p1.E = pat(cv1, 2, u); p1.W = pat(cv1, 0, u);
      p1.N = pat(cv1, 1, u + 1); p1.S = pat(cv1, 1, u - 1);
      p1.NE = pat(cv1, 2, u + 1); p1.NW = pat(cv1, 0, u + 1);
      p1.SE = pat(cv1, 2, u - 1); p1.SW = pat(cv1, 0, u - 1);
      p2.C = pat(cv2, 1, u); p2.E = pat(cv2, 2, u); p2.W = pat(cv2, 0, u);
      p2.N = pat(cv2, 1, u + 1); p2.S = pat(cv2, 1, u - 1);
      p2.NE = pat(cv2, 2, u + 1); p2.NW = pat(cv2, 0, u + 1);
      p2.SE = pat(cv2, 2, u - 1); p2.SW = pat(cv2, 0, u - 1);
      const T* r1 = t1 + u * pitch;
      const T* r2 = t2 + u * pitch;
      q1.C = r1[0]; q1.E = r1[1]; q1.W = r1[-1];
      q1.N = r1[pitch]; q1.S = r1[-pitch];
      q1.NE = r1[pitch + 1]; q1.NW = r1[pitch - 1]; q1.SE = r1[1 - pitch]; q1.SW = r1[-1 - pitch];
      q2.C = r2[0]; q2.E = r2[1]; q2.W = r2[-1];
      q2.N = r2[pitch]; q2.S = r2[-pitch];
      q2.NE = r2[pitch + 1]; q2.NW = r2[pitch - 1]; q2.SE = r2[1 - pitch]; q2.SW = r2[-1 - pitch];
      // zeta_i = Q_i - F_i (psi_j - psi_i) on the 5-point cross (zero on walls)
      Nbr<T> z1, z2;
      z1.C = q1.C - F1 * (p2.C - p1.C);
      z1.E = q1.E - F1 * (p2.E - p1.E);
      z1.W = q1.W - F1 * (p2.W - p1.W);
      z1.N = q1.N - F1 * (p2.N - p1.N);
      z1.S = q1.S - F1 * (p2.S - p1.S);
      z2.C = q2.C - F2 * (p1.C - p2.C);
      z2.E = q2.E - F2 * (p1.E - p2.E);
      z2.W = q2.W - F2 * (p1.W - p2.W);
      z2.N = q2.N - F2 * (p1.N - p2.N);
      z2.S = q2.S - F2 * (p1.S - p2.S);
      const T G1 = -cj * arakawa12(p1, q1) - cb * beta3(p1) + nu * lap5(z1, idx2, idy2) +
                   fv[u - 1];
      const T G2 = -cj * arakawa12(p2, q2) - cb * beta3(p2) + nu * lap5(z2, idx2, idy2) -
                   drag * z2.C;
      T v1 = a * nv1[u - 1] + b * (q1.C + dt * G1);  // a = 0 in stage 1
      T v2 = a * nv2[u - 1] + b * (q2.C + dt * G2);
      v1 = rr >= 1 ? v1 : T(0);
      v2 = rr >= 1 ? v2 : T(0);
      if (u > E) {
        store_field<NTS>(&O[(size_t)rr * pitch + x], v1);
        store_field<NTS>(&O[plane + (size_t)rr * pitch + x], v2);
      }
      res1[u - 1] = v1;
      res2[u - 1] = v2;
    }
    if (last) {  // the top wall row
      store_field<NTS>(&O[(size_t)ny * pitch + x], T(0));
      store_field<NTS>(&O[plane + (size_t)ny * pitch + x], T(0));
    }
  }
  // last stage of an adaptive step: the velocity maxima for the next dt
  if (wants_vmax(d, ctl)) put_vmax_coarse<T, C, TJ, NT>(d, ctl, lb, psc1, psc2, PROW, j0);
  if constexpr (NEXT) {
    // ---- pass A of the next stage on the block's coarse rows j0 .. j0+TJ-1
    // (res[k] = fine row R0-E+k): the y weights of each thread's column in
    // registers, then the x weights over the neighbouring columns' sums
    // (through LDS rows of their own), as pass A computes them
    // (restrict_rows); both layers
    const int i = 1 + t;
    cplx<T> z[TJ];
#pragma unroll
    for (int r = 0; r < TJ; ++r) z[r] = {T(0), T(0)};
    T y1[TJ], y2[TJ];
#pragma unroll
    for (int r = 0; r < TJ; ++r) {
      y1[r] = yweight<T, C>(res1 + C * r);
      y2[r] = yweight<T, C>(res2 + C * r);
    }
    T v1[TJ], v2[TJ];
    if constexpr (C == 1) {
      // coarse column i is the thread's own column: nothing to exchange
#pragma unroll
      for (int r = 0; r < TJ; ++r) {
        v1[r] = y1[r];
        v2[r] = y2[r];
      }
      __syncthreads();  // every thread is done with the tiles and psc
    } else {
      T* yc1 = psc2 + NS * PROW;
      T* yc2 = yc1 + TJ * pitch;
      if (x < nx) {
#pragma unroll
        for (int r = 0; r < TJ; ++r) {
          yc1[r * pitch + x] = y1[r];
          yc2[r * pitch + x] = y2[r];
        }
      }
      __syncthreads();  // also: every thread is done with the tiles and psc
      const int ii = i < MX ? i : 1;
#pragma unroll
      for (int r = 0; r < TJ; ++r) {
        v1[r] = xweight<T, C>(yc1 + r * pitch + C * ii) * (T(1) / T(C * C * C * C));
        v2[r] = xweight<T, C>(yc2 + r * pitch + C * ii) * (T(1) / T(C * C * C * C));
      }
    }
    if (i < MX) {
      const T wbt1 = T(d.delta), wbt2 = T(1.0 - d.delta);
#pragma unroll
      for (int r = 0; r < TJ; ++r)
        z[r] = {wbt1 * v1[r] + wbt2 * v2[r], v1[r] - v2[r]};  // (barotropic, baroclinic)
    }
    if (i < MX) {
#pragma unroll
      for (int r = 0; r < TJ; ++r) {
        buf[r * LP + pad(i)] = z[r];
        buf[r * LP + pad(2 * MX - i)] = {-z[r].x, -z[r].y};
      }
    }
    if (t < TJ) {
      buf[t * LP + pad(0)] = {T(0), T(0)};
      buf[t * LP + pad(MX)] = {T(0), T(0)};
    }
    // the last stage stores the spectra (row j0+r: sequence r) directly
    __syncthreads();
    constexpr int NLAST = stage_plan(LC).n - 1;
    const cplx<T>* X =
        ct_stage_range<T, LC, 0, NLAST, NT, 4, kWideRows>(buf, buf + TJ * LP, TJ, tw);
    ct_stage_last<T, LC, NT, 4, kWideRows, false>(
        X, TJ, tw, [&](int r, int k, cplx<T> zk, int, int) {
          const int j = j0 + r;
          if (k >= 1 && k < MX && j >= 1 && j <= My - 1) {
            T* wo = wnext + d.wt_off + (size_t)(k - 1) * (My - 1);
            wo[j - 1] = T(-0.5) * zk.y;
            wo[mplane + j - 1] = T(0.5) * zk.x;
          }
        });
  }
}

// g.L = (c << 16) | transform length (compile-time lengths only)
template <typename T>
hipError_t Launch<T>::prolong_stencil2(const MemberDesc* md, const Group& g, const T* wt,
                                       T* wnext, const cplx<T>* tw, const T* ws,
                                       const T* forcing, const T* wn, T* out, double a, double b,
                                       StepCtl ctl, bool nt_store, hipStream_t s) {
#define LAUNCH(C, TJ, LC, NX, NTS)                                                      \
  hipLaunchKernelGGL((k_prolong_stencil2<T, C, TJ, LC, NX, NTS>), dim3(g.nblk),         \
                     dim3(kFusedThreads), g.lds, s, md, g.members, g.count, g.nblk, wt, \
                     wnext, tw, ws, forcing, wn, out, a, b, ctl)
#define BY_C(NX, NTS)                                          \
  switch (g.L) {                                               \
    case (1 << 16) | 128: LAUNCH(1, 1, 128, NX, NTS); break;   \
    case (1 << 16) | 256: LAUNCH(1, 1, 256, NX, NTS); break;   \
    case (1 << 16) | 384: LAUNCH(1, 1, 384, NX, NTS); break;   \
    case (1 << 16) | 512: LAUNCH(1, 1, 512, NX, NTS); break;   \
    case (1 << 16) | 768: LAUNCH(1, 1, 768, NX, NTS); break;   \
    case (1 << 16) | 1024: LAUNCH(1, 1, 1024, NX, NTS); break; \
    case (2 << 16) | 128: LAUNCH(2, 2, 128, NX, NTS); break;   \
    case (2 << 16) | 256: LAUNCH(2, 2, 256, NX, NTS); break;   \
    case (2 << 16) | 384: LAUNCH(2, 2, 384, NX, NTS); break;   \
    case (2 << 16) | 512: LAUNCH(2, 2, 512, NX, NTS); break;   \
    case (4 << 16) | 128: LAUNCH(4, 1, 128, NX, NTS); break;   \
    case (4 << 16) | 256: LAUNCH(4, 1, 256, NX, NTS); break;   \
    default: return hipErrorInvalidValue;                      \
  }
  // the new vorticity written through the L2 only where asked for
  if (!wnext) {
    BY_C(false, false)
  } else if (nt_store) {
    BY_C(true, true)
  } else {
    BY_C(true, false)
  }
#undef BY_C
#undef LAUNCH
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::prepare_fused2(size_t bytes) {
  const int b = (int)bytes;
  const void* fns[] = {
#define K(C, TJ, LC)                                                                 \
  reinterpret_cast<const void*>(&k_prolong_stencil2<T, C, TJ, LC, false, false>),    \
      reinterpret_cast<const void*>(&k_prolong_stencil2<T, C, TJ, LC, true, false>), \
      reinterpret_cast<const void*>(&k_prolong_stencil2<T, C, TJ, LC, true, true>)
      K(1, 1, 128), K(1, 1, 256), K(1, 1, 384), K(1, 1, 512), K(1, 1, 768), K(1, 1, 1024),
      K(2, 2, 128), K(2, 2, 256), K(2, 2, 384), K(2, 2, 512), K(4, 1, 128), K(4, 1, 256)
#undef K
  };
  for (const void* f : fns) {
    const hipError_t e = allow_dynamic_lds(f, b);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template struct Launch<float>;
template struct Launch<double>;

}  // namespace cgp
