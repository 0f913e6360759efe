// Pass B of the coarse solve (Sec. 4.3) as a block-level device function,
// shared by the column-solve kernel and the persistent stage kernel of
// ensembles.
#pragma once

#include "cgp_internal.hpp"
#include "fft_lds.hpp"

namespace cgp {

// ---------------------------------------------------------------------------
// Pass B.  A block transforms one pair of coarse spectral columns (one layer:
// columns k, k+1; two layers: the barotropic and baroclinic column k) along
// y, multiplies by (2/Mx)(2/My)/lambda_kl (baroclinic: 1/(lambda_kl - F1 -
// F2)), and transforms back, from the spectra of omega (win) to those of psi
// (wout, same layout, written through the L2: store_through).  Loads are
// batched as in pass A.  The transforms use
// the column plan (stage_plan(L, kWideCols)): one sequence per 256-thread
// block has enough butterflies for radix 8 only from L = 2048 on.
// ---------------------------------------------------------------------------
// 1/x for the eigenvalues (negative, far from the overflow and subnormal
// ranges): the hardware estimate refined by two Newton steps
// r <- r + r (1 - x r), within an ulp or two of the quotient, at a third of
// the instructions of a full IEEE division.
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// One block of pass B: member d's column pair lb, NT threads (every thread
// of the block calls it; a block of more threads than the transform has
// butterflies leaves the rest idle between the barriers).  smem is the
// block's dynamic LDS, red NT/64 doubles of LDS for the step-size reduction.
// SP: the most parts of a split restriction among the group's members (0:
// none); a member with a split restriction (split_off) gets the sum of its
// nparts part spectra as the input.
template <typename T, int LC, int NT, int SP = 0>
__device__ __forceinline__ void col_solve_block(const MemberDesc& d, int lb,
                                                const T* __restrict__ win, T* __restrict__ wout,
                                                const cplx<T>* __restrict__ twg,
                                                const double* __restrict__ lam,
                                                double* __restrict__ ctl,
                                                unsigned char* smem, double* red) {
  // twiddles: with a compile-time length each thread keeps the ones of its
  // own butterflies in registers (no LDS table), else the block stages the
  // table in LDS
  constexpr int kTw = LC ? 1 : tw_per_thread<LC, NT, kWideCols>();
  constexpr int kRegTw = LC ? reg_tw_count<LC, NT, 1, kWideCols>() : 1;
  // rows per thread: My - 1 <= 1023, or My - 1 = LC/2 - 1 with a compile-time length
  constexpr int kRowIter = ((LC ? LC / 2 - 1 : 1023) + NT - 1) / NT;
  // a compile-time transform length fixes the column length (Lc = 2 My)
  const int Mx = d.Mx, My = LC ? LC / 2 : d.My, L = LC ? LC : d.Lc, nl = d.nlayers;
  const int ntw = d.ntw_c;
  const int ny1 = My - 1;
  const int LP = lpad(L);
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* buf2 = buf + LP;
  cplx<T>* tw = buf2 + LP;
  const size_t mplane = (size_t)(Mx - 1) * (My - 1);
  const double* lamx = lam + d.lam_off;
  const double* lamy = lamx + (Mx - 1);
  const double scale = 4.0 / ((double)Mx * (double)My);
  const double shift = nl == 2 ? d.f1 + d.f2 : 0.0;
  CGP_STAMP(0);  // block start

  // the pair's columns (1-based); kb may be absent (one layer, Mx - 1 odd)
  const int ka = nl == 1 ? 1 + 2 * lb : 1 + lb;
  const int kb = nl == 1 ? ka + 1 : ka;
  const bool has_b = kb <= Mx - 1;
  const size_t offa = d.wt_off + (size_t)(ka - 1) * ny1;
  const size_t offb = d.wt_off + (nl == 2 ? mplane : 0) + (size_t)((has_b ? kb : ka) - 1) * ny1;
  const T* cola = win + offa;
  const T* colb = win + offb;
  const double lxa = lamx[ka - 1];
  const double lxb = lamx[(has_b ? kb : ka) - 1] - shift;

  T twx[kTw], twy[kTw];
  cplx<T> rtw[kRegTw];
  if constexpr (LC != 0) {
    reg_tw_load<T, LC, 1, NT, 1, kWideCols>(rtw, twg + d.twc_off, 1);
  } else {
#pragma unroll
    for (int q = 0; q < kTw; ++q) {
      const int m = CGP_TID + NT * q;
      const cplx<T> z = twg[d.twc_off + (m < ntw ? m : 0)];
      twx[q] = z.x;
      twy[q] = z.y;
    }
  }
  T va[kRowIter], vb[kRowIter];
  double ly[kRowIter];
#pragma unroll
  for (int q = 0; q < kRowIter; ++q) {
    const int l = min(1 + CGP_TID + NT * q, My - 1);
    va[q] = cola[l - 1];
    const T b = colb[l - 1];
    vb[q] = has_b ? b : T(0);
    ly[q] = lamy[l - 1];
  }
  if (SP > 0 && d.split_off != 0) {
    // split restriction: the spectra of the other parts are added to those
    // of the first, in part order (the x transform is linear); every part's
    // loads are issued together (a member with fewer parts than SP reads
    // part 0 in their place and discards it)
    const int np = d.nparts;
#pragma unroll
    for (int p = 1; p < SP; ++p) {
      const size_t po = (size_t)(p < np ? p : 0) * d.split_off;
#pragma unroll
      for (int q = 0; q < kRowIter; ++q) {
        const int l = min(1 + CGP_TID + NT * q, My - 1);
        const T a = cola[po + l - 1];
        const T b = colb[po + l - 1];
        va[q] = p < np ? va[q] + a : va[q];
        vb[q] = p < np ? vb[q] + (has_b ? b : T(0)) : vb[q];
      }
    }
  }
  if constexpr (LC == 0) {
#pragma unroll
    for (int q = 0; q < kTw; ++q) {
      const int m = CGP_TID + NT * q;
      if (m < ntw) tw[m] = {twx[q], twy[q]};
    }
  }
  if (CGP_TID == 0) {
    buf[pad(0)] = {T(0), T(0)};
    buf[pad(My)] = {T(0), T(0)};
  }
#pragma unroll
  for (int q = 0; q < kRowIter; ++q) {
    const int l = 1 + CGP_TID + NT * q;
    if (l < My) {
      buf[pad(l)] = {va[q], vb[q]};
      buf[pad(2 * My - l)] = {-va[q], -vb[q]};
    }
  }
  CGP_STAMP(1);  // the columns are loaded (thread 0's share in LDS)
  if constexpr (LC != 0 && ct_can_merge_ends<LC, kWideCols>()) {
    // Compile-time transform whose first and last radix agree (1024 and 256
    // points): the forward transform's last stage, the eigenvalue divide and
    // the inverse transform's first stage run in registers, one pass through
    // LDS fewer (ct_last_map_first).  The divide takes every output m of the
    // forward transform: for m > My the packed odd sequences give
    // Z_m = -Z_(2My-m), so the same divide at wavenumber 2My - m yields the
    // odd extension of the quotients the inverse transform needs.
    constexpr StagePlan P = stage_plan(LC, kWideCols);
    constexpr int RL = P.R[P.n - 1], NSL = LC / RL;
    constexpr int QL = (NSL + NT - 1) / NT;
    double lyl[QL][RL];
#pragma unroll
    for (int q = 0; q < QL; ++q)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int m = CGP_TID + NT * q + r * NSL;
        const int k = m < My ? m : 2 * My - m;
        lyl[q][r] = lamy[min(max(k, 1), My - 1) - 1];
      }
    __syncthreads();
    cplx<T>* X = ct_stage_range<T, LC, 0, P.n - 1, NT, 1, kWideCols, true>(buf, buf2, 1, rtw);
    cplx<T>* Y = X == buf ? buf2 : buf;
    ct_last_map_first<T, LC, NT, kWideCols>(X, Y, rtw, [&](int m, cplx<T> z, int q, int r) {
      if (m == 0 || m == My) return cplx<T>{T(0), T(0)};
      return cplx<T>{T(-0.5) * z.y * T(scale * recip(lxa + lyl[q][r])),
                     T(0.5) * z.x * T(scale * recip(lxb + lyl[q][r]))};
    });
    CGP_STAMP(2);  // forward transform and divide done
    const cplx<T>* X2 = ct_stage_range<T, LC, 1, P.n - 1, NT, 1, kWideCols, true>(Y, X, 1, rtw);
    ct_stage_last<T, LC, NT, 1, kWideCols, true>(X2, 1, rtw, [&](int, int m, cplx<T> z, int, int) {
      if (m >= 1 && m < My) {
        store_through(&wout[offa + m - 1], T(-0.5) * z.y);
        if (has_b) store_through(&wout[offb + m - 1], T(0.5) * z.x);
      }
    });
  } else if constexpr (LC != 0) {
    // Compile-time transform: the last stage of the forward transform divides
    // by the eigenvalues and writes the synthesis input, and the last stage of
    // the inverse stores the result (no separate LDS passes for either).
    constexpr StagePlan P = stage_plan(LC, kWideCols);
    constexpr int RL = P.R[P.n - 1], NSL = LC / RL;
    constexpr int QL = (NSL + NT - 1) / NT;
    // lambda_y at the outputs m = j + r L/R of the thread's last-stage butterflies
    double lyl[QL][RL];
#pragma unroll
    for (int q = 0; q < QL; ++q)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int m = CGP_TID + NT * q + r * NSL;
        lyl[q][r] = lamy[min(max(m, 1), My - 1) - 1];
      }
    constexpr bool kLastA = ct_last_reads_a<LC, kWideCols>();
    cplx<T>* Y = kLastA ? buf2 : buf;
    auto divide = [&](int, int m, cplx<T> z, int q, int r) {
      if (m >= 1 && m < My) {
        const T a = T(-0.5) * z.y * T(scale * recip(lxa + lyl[q][r]));
        const T b = T(0.5) * z.x * T(scale * recip(lxb + lyl[q][r]));
        Y[pad(m)] = {a, b};
        Y[pad(2 * My - m)] = {-a, -b};
      } else if (m == 0 || m == My) {
        Y[pad(m)] = {T(0), T(0)};
      }
    };
    ct_run_to<T, LC, NT, 1, kWideCols, true>(divide, buf, buf2, 1, rtw);
    CGP_STAMP(2);  // forward transform and divide done
    auto store = [&](int, int m, cplx<T> z, int, int) {
      if (m >= 1 && m < My) {
        store_through(&wout[offa + m - 1], T(-0.5) * z.y);
        if (has_b) store_through(&wout[offb + m - 1], T(0.5) * z.x);
      }
    };
    ct_run_to<T, LC, NT, 1, kWideCols, true>(store, Y, kLastA ? buf : buf2, 1, rtw);
  } else {
    cplx<T>* Z = fft_run<T, LC, NT, kWideCols>(buf, buf2, 1, L, d.nst_c, d.stw_c, tw);
    cplx<T>* Y = (Z == buf) ? buf2 : buf;
#pragma unroll
    for (int q = 0; q < kRowIter; ++q) {
      const int l = 1 + CGP_TID + NT * q;
      if (l < My) {
        const cplx<T> z = Z[pad(l)];
        const T a = T(-0.5) * z.y * T(scale * recip(lxa + ly[q]));
        const T b = T(0.5) * z.x * T(scale * recip(lxb + ly[q]));
        Y[pad(l)] = {a, b};
        Y[pad(2 * My - l)] = {-a, -b};
      }
    }
    if (CGP_TID == 0) {
      Y[pad(0)] = {T(0), T(0)};
      Y[pad(My)] = {T(0), T(0)};
    }
    CGP_STAMP(2);  // forward transform and divide done
    const cplx<T>* R = fft_run<T, LC, NT, kWideCols>(Y, Z, 1, L, d.nst_c, d.stw_c, tw);
#pragma unroll
    for (int q = 0; q < kRowIter; ++q) {
      const int l = 1 + CGP_TID + NT * q;
      if (l < My) {
        const cplx<T> z = R[pad(l)];
        store_through(&wout[offa + l - 1], T(-0.5) * z.y);
        if (has_b) store_through(&wout[offb + l - 1], T(0.5) * z.x);
      }
    }
  }
  CGP_STAMP(3);  // inverse transform done, results stored
  // first stage of a step: the member's dt
  if (ctl != nullptr && lb == 0) update_step_dt<NT>(d, ctl, red);
}

}  // namespace cgp
