// The fused stage pass (passes C + D and the next stage's pass A, one
// layer) as a block-level device function, shared by the fused-pass kernel
// and the persistent stage kernel of ensembles.  See fused_kernels.hip for
// the block's phases.
#pragma once

#include "cgp_internal.hpp"
#include "fft_lds.hpp"
#include "stencil.hpp"

namespace cgp {

// Vorticity tile rows of a block (KW elements per thread; element e of the
// tile is tile row e / pitch, column e % pitch, tracked incrementally); the
// ring and the rows outside 1 .. ny-1 are stored as 0, so that the stencil
// reads the tile without masks.
template <typename T, int NT, int KW>
__device__ __forceinline__ void load_tile(const T* __restrict__ W, long long g0, int nW, int RB0,
                                          int pitch, int nx, int ny, T (&wv)[KW]) {
  const int t = CGP_TID;
  int er = t / pitch, ec = t - er * pitch;
  const int dr = NT / pitch, dc = NT - dr * pitch;
#pragma unroll
  for (int q = 0; q < KW; ++q) {
    const int e = t + NT * q;
    const int fr = RB0 + er;
    const bool in = e < nW && fr >= 1 && fr <= ny - 1 && ec >= 1 && ec <= nx - 1;
    const T v = W[in ? g0 + e : 0];
    wv[q] = in ? v : T(0);
    er += dr;
    ec += dc;
    if (ec >= pitch) {
      ec -= pitch;
      ++er;
    }
  }
}

// Waves per SIMD the register allocation must allow: four (two blocks per
// CU, which ensembles of many blocks need) where that fits without spills
// (FP64 blocks of four coarse rows at c = 2 need about 170 VGPRs, and their
// LDS allows one block per CU anyway).
__host__ __device__ constexpr int fused_waves_per_simd(int c, int lc, int tj = 2, int es = 8) {
  return (c <= 2 && lc != 0 && (c == 1 || tj <= 2 || es == 4)) ? 4 : 2;
}

// C: coarsening factor; TJ: coarse rows owned per block; LC: transform
// length with a compile-time transform, or 0.  NEXT: also restrict the new
// vorticity of the block's coarse rows and transform it along x (pass A of
// the next stage), which needs it on the C-1 fine rows below the block too;
// those rows are computed here as well but not stored.
// One block of the fused pass: member d's coarse rows lb*TJ .. lb*TJ+TJ-1,
// kFusedThreads threads; smem is the block's dynamic LDS.  EARLY: issue the
// vorticity tile loads with the spectra (the faster order at c = 2) rather
// than once the spectra are in LDS (fewer registers live across the
// transform).  At c >= 4 (TJ = 1) split_blocks(C) consecutive blocks share
// a coarse row, block lb owning share HB = lb mod split_blocks(C) of its
// fine rows (the caller passes HB: the prolongation weights are then
// constants).  With a compile-time transform, the inverse transform's last
// stage writes the coarse psi rows and the forward transform's last stage
// the spectra directly, without a copy through LDS.
template <typename T, int C, int TJ, int LC, bool NEXT, bool EARLY = (C == 2), bool NTS = false,
          int HB = 0>
__device__ __forceinline__ void fused_stage_block(
    const MemberDesc& d, int lb, const T* __restrict__ wt, T* __restrict__ wnext,
    const cplx<T>* __restrict__ twg, const T* __restrict__ ws, const T* __restrict__ forcing,
    const T* __restrict__ wn, T* __restrict__ out, T* __restrict__ psi_out, double a_,
    double b_, StepCtl ctl, unsigned char* smem) {
  constexpr int NT = kFusedThreads;
  constexpr int H = C >= 4 ? split_blocks(C) : 1;  // blocks per coarse row
  constexpr int CR = C / H;           // fine rows of a coarse row a block owns
  static_assert(H == 1 || TJ == 1, "shared coarse rows: one coarse row per block");
  static_assert(HB < H, "share index");
  constexpr int NR = CR * TJ + 1;     // the most own fine rows (+1: top wall row)
  // c >= 4 (one coarse row per block): the next stage's restriction is split
  // (split_yweights), so the block restricts its own fine rows only; c <= 2
  // computes the C-1 rows below the block as well, for whole restrictions
  constexpr bool SPLIT = NEXT && C >= 4;
  static_assert(!SPLIT || TJ == 1, "split restriction: one coarse row per block");
  constexpr int E = (NEXT && !SPLIT) ? C - 1 : 0;  // computed rows below the block
  constexpr int NO = NR + E;          // the most computed rows
  constexpr int NP = NO + 2;          // tile rows: computed rows and one on each side
  constexpr int OFF = C - 1 - E + HB * CR;  // tile row u is fine row C*(j0-1) + OFF + u
  constexpr int NSQ = fused_nseq(TJ);  // complex sequences of the inverse transform
  constexpr int NQ = (TJ + 1) / 2;     // complex sequences of the next stage's transform
  // twiddles per thread: (R-1) Ns summed over the stages, < L <= 1024
  constexpr int kTwPer = ((LC ? stage_plan(LC).ntw : 1023) + NT - 1) / NT;
  static_assert(kFusedMaxNx - 1 <= NT, "one spectral column and one fine column per thread");
  constexpr int kWPer = (NP * (kFusedMaxNx + 1) + NT - 1) / NT;
  const int t = CGP_TID;
  // with a compile-time transform length the row sizes are constants too
  // (Lr = 2 Mx, nx = C Mx), which turns tile and row addresses into
  // immediate offsets
  const int Mx = LC ? LC / 2 : d.Mx, My = d.My, L = LC ? LC : d.Lr;
  const int nx = LC ? C * (LC / 2) : d.nx, ny = d.ny, pitch = nx + 1;
  const int LP = lpad(L);
  const int ntw = d.ntw_r;

  // coarse rows j0-1 .. j0+TJ are synthesised in the global pairs (2m-1, 2m),
  // so that every block that synthesises a row gets the same bits for it
  const int j0 = (lb / H) * TJ;
  const int rlo = max(1, j0 - 1);
  const int ilo = rlo - ((rlo & 1) ? 0 : 1);      // odd: first row of its pair
  const int rhi = min(My - 1, j0 + TJ);
  const int ihi = min(My - 1, rhi + (rhi & 1));   // even: last row of its pair
                                                  // (My-1 odd: its partner is the wall)
  const int nint = ihi >= ilo ? ihi - ilo + 1 : 0;
  const int nseq = (nint + 1) / 2;
  const int last = (lb == d.nblk[PASS_CD] - 1);
  const int R0 = C * j0 + HB * CR;
  const int R1 = last ? ny + 1 : R0 + CR * TJ;   // exclusive end of the own rows
  const int nfr = R1 - R0;                       // own rows (<= NR)
  const int nrow = nfr + E;                      // computed rows: tile rows 1 .. nrow
  const int RB0 = R0 - 1 - E;                    // fine row of tile row 0
  const int nW = (nrow + 2) * pitch;

  // LDS: [ FFT buffers | later the vorticity tile | later the next
  // transform's buffers ] [ twiddles ] [ coarse psi rows ] [ the
  // restriction's column sums ].  Sharing the first region keeps the block
  // small enough for two blocks per CU when there are many (ensembles).
  const int region =
      (max(2 * NSQ * LP * (int)sizeof(cplx<T>), NP * pitch * (int)sizeof(T)) + 15) & ~15;
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem);
  T* wtile = reinterpret_cast<T*>(smem);
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem + region);
  T* psc = reinterpret_cast<T*>(tw + ntw);
  const int prow = Mx + 1;
  CGP_STAMP(0);  // block start

  // ---- global loads are unconditional (a lane without an element reads
  // element 0 of the same array and discards it), so that they sit in one
  // basic block.  The transform's twiddles and spectra come first.
  T twx[kTwPer], twy[kTwPer];
#pragma unroll
  for (int q = 0; q < kTwPer; ++q) {
    const int m = t + NT * q;
    const cplx<T> z = twg[d.twr_off + (m < ntw ? m : 0)];
    twx[q] = z.x;
    twy[q] = z.y;
  }
  // Spectra: row pair p of column k (rows ilo+2p, ilo+2p+1, consecutive in
  // the column) is one load; item c = (k-1) NSQ + p, so that neighbouring
  // lanes read neighbouring pairs.  A pair whose second row is the wall row
  // My is read one element lower, which keeps the load inside the column.
  const T* w = wt + d.wt_off;
  constexpr int kPairs = ((kFusedMaxNx / C - 1) * NSQ + NT - 1) / NT;
  upair<T> sp[kPairs];
#pragma unroll
  for (int q = 0; q < kPairs; ++q) {
    const int c = t + NT * q;
    const int k = 1 + c / NSQ, p = c - (k - 1) * NSQ;
    const int r0 = ilo + 2 * p;
    const bool in = k < Mx && p < nseq;
    const bool top = r0 + 1 > My - 1;
    const size_t e = (size_t)(k - 1) * (My - 1) + (r0 - 1) - (top ? 1 : 0);
    const upair<T> v = *reinterpret_cast<const upair<T>*>(w + (in ? e : 0));
    upair<T> z;
    z.x = in ? (top ? v.y : v.x) : T(0);
    z.y = in && !top ? v.y : T(0);
    sp[q] = z;
  }
  constexpr bool kEarlyTile = EARLY;
  T wv[kWPer];
  if constexpr (kEarlyTile)
    load_tile<T, NT, kWPer>(ws + d.field_off, (long long)RB0 * pitch, nW, RB0, pitch, nx, ny, wv);
  // ---- twiddles and the two packed sequences (odd extension) into LDS
#pragma unroll
  for (int q = 0; q < kTwPer; ++q) {
    const int m = t + NT * q;
    // unconditional, a thread past the table writing slot ntw (the first
    // element of psc, written only after the transform): under a condition
    // the compiler sinks the twiddle load into it, behind the spectra and
    // tile loads, and waits for all of them before the first barrier (the
    // spectra phase at 512x1024 l = 1 2.16 -> 1.84 us, 41.05 -> 40.04 us per
    // step)
    tw[m < ntw ? m : ntw] = {twx[q], twy[q]};
  }
  if (t < nseq) {
    buf[t * LP + pad(0)] = {T(0), T(0)};
    buf[t * LP + pad(Mx)] = {T(0), T(0)};
  }
#pragma unroll
  for (int q = 0; q < kPairs; ++q) {
    const int c = t + NT * q;
    const int k = 1 + c / NSQ, p = c - (k - 1) * NSQ;
    if (k < Mx && p < nseq) {
      const cplx<T> z = {sp[q].x, sp[q].y};
      buf[p * LP + pad(k)] = z;
      buf[p * LP + pad(2 * Mx - k)] = {-z.x, -z.y};
    }
  }
  const T* W = ws + d.field_off;
  const T* FF = forcing + d.field_off;
  const T* WN = wn + d.field_off;
  T* O = out + d.field_off;
  const long long g0 = (long long)RB0 * pitch;
  // ---- the stencil's inputs, issued once the transform's inputs are in
  // LDS: they arrive while the transform runs
  if constexpr (!kEarlyTile) load_tile<T, NT, kWPer>(W, g0, nW, RB0, pitch, nx, ny, wv);
  // forcing and omega_n at the thread's column x = 1 + t, computed rows
  const int x = 1 + t;
  T fv[NO], nv[NO];
#pragma unroll
  for (int u = 1; u <= NO; ++u) {
    const int rr = RB0 + u;
    const bool in = x < nx && u <= nrow && rr >= 1 && rr < ny;
    const size_t o = in ? (size_t)rr * pitch + x : 0;
    const T f = FF[o], n = WN[o];
    fv[u - 1] = in ? f : T(0);
    nv[u - 1] = in ? n : T(0);
  }

  // ---- coarse psi rows J = j0-1 .. j0+TJ (zero walls) into psc: sequence
  // p holds rows ilo+2p (imaginary part) and ilo+2p+1 (real part)
  if constexpr (LC != 0) {
    // the transform's last stage writes its outputs straight into psc (no
    // LDS pass and barrier of a separate copy)
    __syncthreads();
    CGP_STAMP(1);  // the spectra are in LDS
    constexpr int NLAST = stage_plan(LC).n - 1;
    const cplx<T>* X =
        ct_stage_range<T, LC, 0, NLAST, NT, NSQ, kWideRows>(buf, buf + NSQ * LP, nseq, tw);
    ct_stage_last<T, LC, NT, NSQ, kWideRows, false>(
        X, nseq, tw, [&](int p, int m, cplx<T> z, int, int) {
          if (m >= 1 && m < Mx) {
            const int J = ilo + 2 * p, r = J - (j0 - 1);
            if (r >= 0 && r < TJ + 2) psc[r * prow + m] = T(-0.5) * z.y;
            if (r + 1 >= 0 && r + 1 < TJ + 2 && J + 1 <= My - 1)
              psc[(r + 1) * prow + m] = T(0.5) * z.x;
          }
        });
    for (int i = t; i <= Mx; i += NT) {
#pragma unroll
      for (int r = 0; r < TJ + 2; ++r) {
        const int J = j0 - 1 + r;
        if (J < 1 || J > My - 1 || i == 0 || i == Mx) psc[r * prow + i] = T(0);
      }
    }
  } else {
    const cplx<T>* Z =
        fft_runn<T, LC, NT, NSQ>(buf, buf + NSQ * LP, nseq, L, d.nst_r, d.stw_r, tw);
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
  CGP_STAMP(2);  // inverse x transform done, coarse psi rows in LDS
  __syncthreads();  // the transform's output is consumed: the tile may overwrite it
#pragma unroll
  for (int q = 0; q < kWPer; ++q) {
    const int e = t + NT * q;
    if (e < nW) wtile[e] = wv[q];
  }
  __syncthreads();
  CGP_STAMP(3);  // vorticity tile in LDS

  // ---- walls: columns 0 and nx of the own rows (of psi_out too)
  T* PO = psi_out ? psi_out + d.field_off : nullptr;
  if (t < nfr) {
    O[(size_t)(R0 + t) * pitch] = T(0);
    if (PO) PO[(size_t)(R0 + t) * pitch] = T(0);
  } else if (t >= 64 && t < 64 + nfr) {
    O[(size_t)(R0 + t - 64) * pitch + nx] = T(0);
    if (PO) PO[(size_t)(R0 + t - 64) * pitch + nx] = T(0);
  }

  // ---- stencil + RK3 on the computed rows (tile row u = fine row RB0 + u)
  const T dt = stage_dt<T>(d, ctl), a = T(a_), b = T(b_);
  const T cj = T(d.cj), cb = T(d.cb);
  const T idx2 = T(d.idx2), idy2 = T(d.idy2);
  const T nu = T(d.inv_re);
  constexpr T kInvC2 = T(1) / T(C * C);
  T res[NO];
#pragma unroll
  for (int u = 0; u < NO; ++u) res[u] = T(0);
  if (x < nx) {
    // P[dx][u]: psi at fine column x-1+dx, tile row u (bilinear, Sec. 3.1):
    // x weights (C - fx, fx)/C^2 on the coarse columns I, I+1 (I+1 clamped
    // to the wall column Mx), then the compile-time y weights (C - fy, fy).
    // The coarse rows are prow apart; prow is a constant when L is.
    const int prow_c = LC ? LC / 2 + 1 : prow;
    T P[3][NP];
    // c = 2: fine columns x-1, x, x+1 lie on the coarse columns I, I+1, I+2
    // (I = (x-1)/2), the first two of them on I and I+1 and the last on I+1
    // and I+2, so three coarse values per row serve all three; the weights
    // are powers of two, which makes every sum exact whatever the order
    T c3[C == 2 ? 3 : 1][TJ + 2];
    T w3[C == 2 ? 6 : 1];
    if constexpr (C == 2) {
      const int I = (x - 1) >> 1, odd = (x - 1) & 1;
      const T* p0 = psc + I;
      const T* p1 = psc + min(I + 1, Mx);
      const T* p2 = psc + min(I + 2, Mx);
#pragma unroll
      for (int r = 0; r < TJ + 2; ++r) {
        c3[0][r] = p0[r * prow_c];
        c3[1][r] = p1[r * prow_c];
        c3[2][r] = p2[r * prow_c];
      }
      // x-1 = 2I + odd: column x-1 has x weights (2 - odd, odd)/4 on (I, I+1),
      // column x (x = 2I + 1 + odd) (1 - odd, 1 + odd)/4 on (I, I+1), column
      // x+1 (2 - odd, odd)/4 on (I+1, I+2)
      const T q = T(0.25);
      w3[0] = T(2 - odd) * q;
      w3[1] = T(odd) * q;
      w3[2] = T(1 - odd) * q;
      w3[3] = T(1 + odd) * q;
      w3[4] = w3[0];
      w3[5] = w3[1];
    }
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      const int xx = x - 1 + dx;  // 0 .. nx
      T cv[TJ + 2];
      if constexpr (C == 2) {
        const int k = dx == 2 ? 1 : 0;
#pragma unroll
        for (int r = 0; r < TJ + 2; ++r)
          cv[r] = w3[2 * dx] * c3[k][r] + w3[2 * dx + 1] * c3[k + 1][r];
      } else if constexpr (C == 1) {
#pragma unroll
        for (int r = 0; r < TJ + 2; ++r) cv[r] = psc[r * prow_c + xx];
      } else {
        const int I = xx / C, fx = xx - I * C;
        const T a0 = T(C - fx) * kInvC2, a1 = T(fx) * kInvC2;
        const T* p0 = psc + I;
        const T* p1 = psc + min(I + 1, Mx);
#pragma unroll
        for (int r = 0; r < TJ + 2; ++r) cv[r] = a0 * p0[r * prow_c] + a1 * p1[r * prow_c];
      }
#pragma unroll
      for (int u = 0; u < NP; ++u) {
        // fine row C*(j0-1) + m: coarse row j0-1+jr, weight fy toward jr+1
        // (rows past the last coarse row are never used; they are clamped)
        const int m = OFF + u;
        const int jr = m / C, fy = m - jr * C;
        const T top = jr + 1 < TJ + 2 ? cv[jr + 1 < TJ + 2 ? jr + 1 : TJ + 1] : T(0);
        const T on = T(C - fy) * cv[jr < TJ + 2 ? jr : TJ + 1];
        P[dx][u] = fy == 0 ? on : on + T(fy) * top;  // fy is a constant here
      }
    }
    // rows 1 .. NO-1 exist in every block (the last block's row NO is the top
    // wall); rows below 1 (first block) are computed from zeros and dropped
    const T* wt0 = wtile + x;
    T ws0 = wt0[-1], ws1 = wt0[0], ws2 = wt0[1];
    T wc0 = wt0[pitch - 1], wc1 = wt0[pitch], wc2 = wt0[pitch + 1];
#pragma unroll
    for (int u = 1; u < NO; ++u) {
      const T* wr = wt0 + (u + 1) * pitch;
      const T wn0 = wr[-1], wn1 = wr[0], wn2 = wr[1];
      const int rr = RB0 + u;
      Nbr<T> p, w;
      p.C = P[1][u]; p.E = P[2][u]; p.W = P[0][u];
      p.N = P[1][u + 1]; p.S = P[1][u - 1];
      p.NE = P[2][u + 1]; p.NW = P[0][u + 1];
      p.SE = P[2][u - 1]; p.SW = P[0][u - 1];
      w.C = wc1; w.E = wc2; w.W = wc0;
      w.N = wn1; w.S = ws1;
      w.NE = wn2; w.NW = wn0;
      w.SE = ws2; w.SW = ws0;
      const T G = -cj * arakawa12(p, w) - cb * beta3(p) + nu * lap5(w, idx2, idy2) + fv[u - 1];
      T v = a * nv[u - 1] + b * (w.C + dt * G);  // a = 0 in stage 1
      v = rr >= 1 ? v : T(0);
      if (u > E) {
        store_field<NTS>(&O[(size_t)rr * pitch + x], v);
        if (PO) PO[(size_t)rr * pitch + x] = P[1][u];  // the prolonged psi (0 on wall rows)
      }
      res[u - 1] = v;
      ws0 = wc0; ws1 = wc1; ws2 = wc2;
      wc0 = wn0; wc1 = wn1; wc2 = wn2;
    }
    if (last) {  // the top wall row
      store_field<NTS>(&O[(size_t)ny * pitch + x], T(0));
      if (PO) PO[(size_t)ny * pitch + x] = T(0);
    }
  }
  CGP_STAMP(4);  // stencil and RK3 combine done (stores issued)
  // last stage of an adaptive step: the velocity maxima for the next dt
  if (wants_vmax(d, ctl)) put_vmax_coarse<T, C, TJ, NT>(d, ctl, lb, psc, nullptr, prow, j0);
  if constexpr (NEXT) {
    // ---- pass A of the next stage on the block's coarse rows j0 .. j0+TJ-1:
    // their full-weighting stencils cover the computed rows R0-E .. R1-1
    // (res[k] = fine row R0-E+k = tile row k+1), Sec. 3.1 and 4.3
    const int i = 1 + t;
    cplx<T> z[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) z[q] = {T(0), T(0)};
    if constexpr (SPLIT) {
      // the parts of coarse rows j0 (a) and j0+1 (b) that the block's own fine
      // rows (res[k] = fine row C j0 + HB CR + k, k < CR) carry, packed as
      // pass A packs them
      // (a of the wall row 0 and b of the wall row My as 0): the y weights of
      // the thread's column in registers, then the x weights over the
      // neighbouring columns' sums (two LDS rows of their own)
      T ya, yb;
      split_yweights<T, C, CR>(res, HB * CR, ya, yb);
      T* yc = psc + (TJ + 2) * prow;
      if (x < nx) {
        yc[x] = ya;
        yc[pitch + x] = yb;
      }
      __syncthreads();  // also: every thread is done with wtile and psc
      if (i < Mx) {
        T a = xweight<T, C>(yc + C * i) * (T(1) / T(C * C * C * C));
        T b = xweight<T, C>(yc + pitch + C * i) * (T(1) / T(C * C * C * C));
        if (j0 == 0) a = T(0);
        if (j0 + 1 > My - 1) b = T(0);
        z[0] = {a, b};
      }
    } else {
      // whole restrictions: each thread holds its fine column's rows, so the
      // y weights come first, in registers, and one value per coarse row and
      // column crosses threads (through its own LDS rows, which no other
      // phase uses) for the x weights; pass A computes the same sums in the
      // same order (restrict_rows), so both give the same spectra bit for bit
      T yv[TJ];
#pragma unroll
      for (int r = 0; r < TJ; ++r) yv[r] = yweight<T, C>(res + C * r);
      T v[2 * NQ];
#pragma unroll
      for (int r = 0; r < 2 * NQ; ++r) v[r] = T(0);
      if constexpr (C == 1) {
        // coarse column i is the thread's own column: nothing to exchange
#pragma unroll
        for (int r = 0; r < TJ; ++r) v[r] = yv[r];
        __syncthreads();  // every thread is done with wtile and psc
      } else {
        T* yc = psc + (TJ + 2) * prow;
        if (x < nx) {
#pragma unroll
          for (int r = 0; r < TJ; ++r) yc[r * pitch + x] = yv[r];
        }
        __syncthreads();  // also: every thread is done with wtile and psc
        if (i < Mx) {
#pragma unroll
          for (int r = 0; r < TJ; ++r)
            v[r] = xweight<T, C>(yc + r * pitch + C * i) * (T(1) / T(C * C * C * C));
        }
      }
      // packed as pass A packs them (rows in pairs (2m, 2m+1), the wall row 0
      // as 0), so that both give the same spectra bit for bit
      if (j0 == 0) v[0] = T(0);
#pragma unroll
      for (int q = 0; q < NQ; ++q) z[q] = {v[2 * q], v[2 * q + 1]};
    }
    if (i < Mx) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        buf[q * LP + pad(i)] = z[q];
        buf[q * LP + pad(2 * Mx - i)] = {-z[q].x, -z[q].y};
      }
    }
    if (t < NQ) {
      buf[t * LP + pad(0)] = {T(0), T(0)};
      buf[t * LP + pad(Mx)] = {T(0), T(0)};
    }
    // output k of sequence q (rows j0+2q, j0+2q+1) into column k of the
    // next stage's spectra
    auto put = [&](int q, int k, cplx<T> zk) {
      if (k < 1 || k >= Mx) return;
      T* wo = wnext + d.wt_off + (size_t)(k - 1) * (My - 1);
      const T v0 = T(-0.5) * zk.y, v1 = T(0.5) * zk.x;
      if constexpr (SPLIT) {
        // the part of row j0 in part array 2 HB, that of row j0+1 in 2 HB + 1
        if (j0 >= 1) wo[2 * HB * d.split_off + j0 - 1] = v0;
        if (j0 + 1 <= My - 1) wo[(2 * HB + 1) * d.split_off + j0] = v1;
      } else {
        // rows j0+2q, j0+2q+1 are consecutive in the column: one store per pair
        const int j = j0 + 2 * q;
        if (2 * q + 1 < TJ && j >= 1 && j + 1 <= My - 1) {
          upair<T> pr;
          pr.x = v0;
          pr.y = v1;
          *reinterpret_cast<upair<T>*>(wo + j - 1) = pr;
        } else {
          if (j >= 1 && j <= My - 1) wo[j - 1] = v0;
          if (2 * q + 1 < TJ && j + 1 <= My - 1) wo[j] = v1;
        }
      }
    };
    constexpr int MQ = NQ > 2 ? 4 : 2;
    if constexpr (LC != 0) {
      // the last stage stores its outputs straight to global memory
      CGP_STAMP(5);  // restriction done
      __syncthreads();
      constexpr int NLAST = stage_plan(LC).n - 1;
      const cplx<T>* X =
          ct_stage_range<T, LC, 0, NLAST, NT, MQ, kWideRows>(buf, buf + NQ * LP, NQ, tw);
      ct_stage_last<T, LC, NT, MQ, kWideRows, false>(
          X, NQ, tw, [&](int q, int k, cplx<T> z, int, int) { put(q, k, z); });
    } else {
      const cplx<T>* Z2 =
          fft_runn<T, LC, NT, MQ>(buf, buf + NQ * LP, NQ, L, d.nst_r, d.stw_r, tw);
      if (SPLIT && i < Mx) {
        T* wo = wnext + d.wt_off + (size_t)(i - 1) * (My - 1);
        const cplx<T> zk = Z2[pad(i)];
        if (j0 >= 1) wo[2 * HB * d.split_off + j0 - 1] = T(-0.5) * zk.y;
        if (j0 + 1 <= My - 1) wo[(2 * HB + 1) * d.split_off + j0] = T(0.5) * zk.x;
      } else if (i < Mx) {
        T* wo = wnext + d.wt_off + (size_t)(i - 1) * (My - 1);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int j = j0 + 2 * q;
          const cplx<T> zk = Z2[q * LP + pad(i)];
          const T v0 = T(-0.5) * zk.y, v1 = T(0.5) * zk.x;
          if (2 * q + 1 < TJ && j >= 1 && j + 1 <= My - 1) {
            upair<T> pr;
            pr.x = v0;
            pr.y = v1;
            *reinterpret_cast<upair<T>*>(wo + j - 1) = pr;
          } else {
            if (j >= 1 && j <= My - 1) wo[j - 1] = v0;
            if (2 * q + 1 < TJ && j + 1 <= My - 1) wo[j] = v1;
          }
        }
      }
    }
  }
  CGP_STAMP(6);  // block end (the next stage's spectra stored)
}

}  // namespace cgp
