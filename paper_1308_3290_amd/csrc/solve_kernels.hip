// Coarse elliptic solve of the CGP step on gfx950:
//   pass A  full-weighting restriction (level times) fused with the forward
//           sine transform along x (Sec. 3.1, Sec. 4.3);
//   pass B  sine transform along y, eigenvalue divide, inverse transform
//           along y (Sec. 4.3); two layers: barotropic Poisson and
//           baroclinic Helmholtz divide;
//   pass C  inverse sine transform along x fused with bilinear prolongation
//           (Sec. 3.1) and, for two layers, the mode recombination.
//
// Coarse spectra live in the workspace k-major: for mode plane m,
// wt[m][k-1][j-1] (x-wavenumber k = 1..Mx-1, coarse row j = 1..My-1), so the
// y transforms of pass B read contiguous lines and passes A and C do the
// transposition through LDS.
//
// Every block has kThreads threads.  Memory phases map one thread to one
// coarse column (or spectral index) and handle all of the block's rows in
// registers, so that each thread issues its global loads together.
#include "cgp_internal.hpp"
#include "col_solve.hpp"
#include "fft_lds.hpp"
#include "stencil.hpp"

namespace cgp {

// Full weighting applied `level` times equals one tent-weighted average with
// 1-D weights (c - |d|)/c^2, |d| < c = 2^level (the l = 2 case is the
// [1 2 3 4 3 2 1]/16 stencil); it reads fine interior nodes only.
template <typename T>
__device__ __forceinline__ T restrict_generic(const T* __restrict__ f, int pitch, int c, int I,
                                              int J) {
  const T* base = f + (size_t)(c * J) * pitch + c * I;
  T acc = T(0);
  for (int dy = -(c - 1); dy <= c - 1; ++dy) {
    const T* row = base + (ptrdiff_t)dy * pitch;
    T racc = T(0);
    for (int dx = -(c - 1); dx <= c - 1; ++dx) racc += T(c - abs(dx)) * row[dx];
    acc += T(c - abs(dy)) * racc;
  }
  const T c2 = T(c) * T(c);
  return acc / (c2 * c2);
}

// ---------------------------------------------------------------------------
// Pass A.  A block restricts RB consecutive coarse rows starting at j0 (one
// layer: RB = 2, packed as the real and imaginary parts of one complex
// sequence, j0 = a_first + b a_rows, the second row absent when a_rows = 1
// and row 0 read as 0; two layers: RB = 1, its barotropic and baroclinic
// combinations) and transforms them along x.  The twiddles and every fine value of the
// block are loaded before any is used: the loads are unconditional (a lane
// without a column reads a valid neighbour), so that they are in flight
// together.
// ---------------------------------------------------------------------------
// Restriction of coarse rows j0 .. j0+RB-1 at coarse column i, separably:
// the y-weighted sums of the fine columns C i-(C-1) .. C i+(C-1) over each
// coarse row's stencil rows first, then the x weights (yweight, xweight, the
// fused kernels' order).  Rows of absent coarse rows (the wall row 0, rows
// past My-1) are clamped to the array; their values are discarded.
template <typename T, int C, int RB>
__device__ __forceinline__ void restrict_rows(const T* __restrict__ f, int pitch, int ny, int i,
                                              int j0, T* v) {
  constexpr int NF = C * (RB + 1) - 1;  // fine rows C j0-(C-1) .. C (j0+RB-1)+(C-1)
  const int fr0 = C * j0 - (C - 1);
  // the x weights accumulate column by column in xweight's order (one
  // column's rows live at a time)
  T acc[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) acc[r] = T(0);
#pragma unroll 1
  for (int e = 0; e < 2 * C - 1; ++e) {
    const T* colp = f + C * i - (C - 1) + e;
    T col[NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) col[q] = colp[(size_t)max(0, min(fr0 + q, ny)) * pitch];
    const T wx = T(C - (e < C - 1 ? C - 1 - e : e - (C - 1)));
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r] += wx * yweight<T, C>(col + C * r);
  }
#pragma unroll
  for (int r = 0; r < RB; ++r) v[r] = acc[r] * (T(1) / T(C * C * C * C));
}

// keep: which of the one-layer pair's rows are present (bit 0: j0, bit 1: j0+1)
template <typename T, int NL>
__device__ __forceinline__ void put_rows(cplx<T>* buf, int Mx, int i, const T* v, const T* u,
                                         T wbt1, T wbt2, int keep) {
  cplx<T> z;
  if constexpr (NL == 1) z = {(keep & 1) ? v[0] : T(0), (keep & 2) ? v[1] : T(0)};
  else z = {wbt1 * v[0] + wbt2 * u[0], v[0] - u[0]};  // (barotropic, baroclinic)
  buf[pad(i)] = z;
  buf[pad(2 * Mx - i)] = {-z.x, -z.y};
}

// Coarse columns i = 1 + t + kThreads q, q < kColIter, of rows j0 .. j0+RB-1.
constexpr int kColIter = 4;  // Mx - 1 <= 1023

template <typename T, int C, int NL>
__device__ __forceinline__ void restrict_block(const MemberDesc& d, const T* __restrict__ f,
                                               cplx<T>* buf, int j0, int keep) {
  constexpr int RB = NL == 1 ? 2 : 1;
  const int Mx = d.Mx, pitch = d.nx + 1, ny = d.ny;
  const size_t plane = (size_t)(ny + 1) * pitch;
  const T wbt1 = T(d.delta), wbt2 = T(1.0 - d.delta);
  if constexpr (C > 0) {
    T v[kColIter][RB], u[kColIter][RB];
#pragma unroll
    for (int q = 0; q < kColIter; ++q) {
      const int i = min(1 + (int)threadIdx.x + kThreads * q, Mx - 1);
      if (q * kThreads < Mx - 1) {
        restrict_rows<T, C, RB>(f, pitch, ny, i, j0, v[q]);
        if constexpr (NL == 2) restrict_rows<T, C, RB>(f + plane, pitch, ny, i, j0, u[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < kColIter; ++q) {
      const int i = 1 + threadIdx.x + kThreads * q;
      if (i < Mx) put_rows<T, NL>(buf, Mx, i, v[q], u[q], wbt1, wbt2, keep);
    }
  } else {
    const int c = d.c;
    for (int i = 1 + threadIdx.x; i < Mx; i += kThreads) {
      T v[RB], u[RB];
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int j = max(1, min(j0 + r, d.My - 1));
        v[r] = restrict_generic<T>(f, pitch, c, i, j);
        u[r] = NL == 2 ? restrict_generic<T>(f + plane, pitch, c, i, j) : T(0);
      }
      put_rows<T, NL>(buf, Mx, i, v, u, wbt1, wbt2, keep);
    }
  }
}

// Split restriction (one layer, c >= 4): the block of share h of coarse row
// j0 packs the parts a of row j0 and b of row j0+1 that fine rows
// C j0 + h CR .. C j0 + h CR + CR-1 carry (CR = C / split_blocks(C);
// split_yweights of each fine column, then xweight over the columns' sums,
// in the fused pass's order); a of the wall row 0 and b of the wall row My
// are 0.
template <typename T, int C>
__device__ __forceinline__ void split_block(const MemberDesc& d, const T* __restrict__ f,
                                            cplx<T>* buf, int j0, int h) {
  constexpr int CR = C / split_blocks(C);
  const int Mx = d.Mx, My = d.My, pitch = d.nx + 1;
  const int e0 = h * CR;
  T a[kColIter], b[kColIter];
#pragma unroll
  for (int q = 0; q < kColIter; ++q) {
    const int i = min(1 + (int)threadIdx.x + kThreads * q, Mx - 1);
    if (q * kThreads < Mx - 1) {
      T sa = T(0), sb = T(0);
#pragma unroll 1
      for (int e = 0; e < 2 * C - 1; ++e) {
        const T* colp = f + (size_t)(C * j0 + e0) * pitch + C * i - (C - 1) + e;
        T r[CR];
#pragma unroll
        for (int k = 0; k < CR; ++k) r[k] = colp[(size_t)k * pitch];
        T ya, yb;
        split_yweights<T, C, CR>(r, e0, ya, yb);
        const T wx = T(C - (e < C - 1 ? C - 1 - e : e - (C - 1)));
        sa += wx * ya;
        sb += wx * yb;
      }
      a[q] = sa * (T(1) / T(C * C * C * C));
      b[q] = sb * (T(1) / T(C * C * C * C));
    }
  }
#pragma unroll
  for (int q = 0; q < kColIter; ++q) {
    const int i = 1 + threadIdx.x + kThreads * q;
    if (i < Mx) {
      const cplx<T> z = {j0 >= 1 ? a[q] : T(0), j0 + 1 <= My - 1 ? b[q] : T(0)};
      buf[pad(i)] = z;
      buf[pad(2 * Mx - i)] = {-z.x, -z.y};
    }
  }
}

template <typename T, int LC, int NL>
__global__ __launch_bounds__(kThreads) void k_restrict_rowdst(
    const MemberDesc* __restrict__ md, const int* __restrict__ grp, int ng,
    const T* __restrict__ src, T* __restrict__ wt, const cplx<T>* __restrict__ twg) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int kTw = tw_per_thread<LC, kThreads>();
  const MemberDesc& d = md[group_member(md, grp, ng, PASS_A, blockIdx.x)];
  const int lb = blockIdx.x - d.blk0[PASS_A];
  const int Mx = LC ? LC / 2 : d.Mx, My = d.My, L = LC ? LC : d.Lr, ntw = d.ntw_r;
  const int LP = lpad(L);
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* tw = buf + 2 * LP;
  // split members: split_blocks(c) blocks per coarse row (share h)
  const bool split = NL == 1 && d.split_off != 0;
  const int hs = split ? d.nparts / 2 : 1;
  const int h = lb % hs;
  const int j0 = NL == 1 ? d.a_first + (lb / hs) * d.a_rows : 1 + lb;
  // rows of the pair that exist and are interior (1 .. My-1)
  const int keep = NL == 1 ? ((j0 >= 1 ? 1 : 0) | (d.a_rows == 2 && j0 + 1 <= My - 1 ? 2 : 0)) : 1;

  T twx[kTw], twy[kTw];
#pragma unroll
  for (int q = 0; q < kTw; ++q) {
    const int m = threadIdx.x + kThreads * q;
    const cplx<T> z = twg[d.twr_off + (m < ntw ? m : 0)];
    twx[q] = z.x;
    twy[q] = z.y;
  }
  if (threadIdx.x == 0) {
    buf[pad(0)] = {T(0), T(0)};
    buf[pad(Mx)] = {T(0), T(0)};
  }
  const T* f = src + d.field_off;
  if (split) {
    if (d.c == 4) split_block<T, 4>(d, f, buf, j0, h);
    else split_block<T, 8>(d, f, buf, j0, h);
  } else {
    switch (d.c) {
      case 1: restrict_block<T, 1, NL>(d, f, buf, j0, keep); break;
      case 2: restrict_block<T, 2, NL>(d, f, buf, j0, keep); break;
      case 4: restrict_block<T, 4, NL>(d, f, buf, j0, keep); break;
      case 8: restrict_block<T, 8, NL>(d, f, buf, j0, keep); break;
      default: restrict_block<T, 0, NL>(d, f, buf, j0, keep);
    }
  }
#pragma unroll
  for (int q = 0; q < kTw; ++q) {
    const int m = threadIdx.x + kThreads * q;
    if (m < ntw) tw[m] = {twx[q], twy[q]};
  }
  const cplx<T>* Z = fft_run<T, LC>(buf, buf + LP, 1, L, d.nst_r, d.stw_r, tw);

  // spectra of the block's rows, k-major (two consecutive values per k)
  T* w = wt + d.wt_off;
  const size_t mplane = (size_t)(Mx - 1) * (My - 1);
  for (int k = 1 + threadIdx.x; k < Mx; k += kThreads) {
    const cplx<T> zk = Z[pad(k)];
    const long long o = (long long)(k - 1) * (My - 1) + (j0 - 1);  // row j0 (-1 if j0 = 0)
    if constexpr (NL == 1) {
      if (split) {  // a of row j0 in part 2h; b of row j0+1 in part 2h+1
        if (j0 >= 1) w[2 * h * d.split_off + o] = T(-0.5) * zk.y;
        if (j0 + 1 <= My - 1) w[(2 * h + 1) * d.split_off + o + 1] = T(0.5) * zk.x;
      } else {
        if (keep & 1) w[o] = T(-0.5) * zk.y;
        if (keep & 2) w[o + 1] = T(0.5) * zk.x;
      }
    } else {
      w[o] = T(-0.5) * zk.y;
      w[mplane + o] = T(0.5) * zk.x;
    }
  }
}


// ---------------------------------------------------------------------------
// Pass B: one block per pair of spectral columns (col_solve.hpp).
// ---------------------------------------------------------------------------
template <typename T, int LC, int SP>
__global__ __launch_bounds__(kThreads) void k_col_solve(const MemberDesc* __restrict__ md,
                                                        const int* __restrict__ grp, int ng,
                                                        const T* __restrict__ win,
                                                        T* __restrict__ wout,
                                                        const cplx<T>* __restrict__ twg,
                                                        const double* __restrict__ lam,
                                                        double* __restrict__ ctl) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[kThreads / 64];  // step-size reduction
  const MemberDesc& d = md[group_member(md, grp, ng, PASS_B, blockIdx.x)];
  col_solve_block<T, LC, kThreads, SP>(d, blockIdx.x - d.blk0[PASS_B], win, wout, twg, lam, ctl,
                                       smem, red);
}

// ---------------------------------------------------------------------------
// Pass C.  Block owns coarse rows j0 .. j0+tj-1 and writes the fine rows
// c*j0 .. c*(j0+tj)-1 (the last block also the top wall row).  It
// synthesises coarse rows j0 .. j0+tj-1 (+1 halo row when c > 1) along x,
// keeps them in LDS with their zero walls and interpolates bilinearly
// (c = 1: the rows are written directly).
// ---------------------------------------------------------------------------
template <typename T, int LC>
__global__ __launch_bounds__(kThreads) void k_rowdst_prolong(const MemberDesc* __restrict__ md,
                                                             const int* __restrict__ grp, int ng,
                                                             const T* __restrict__ wt,
                                                             T* __restrict__ dst, int accumulate,
                                                             const cplx<T>* __restrict__ twg) {
  extern __shared__ __align__(16) unsigned char smem[];
  const MemberDesc& d = md[group_member(md, grp, ng, PASS_C, blockIdx.x)];
  const int lb = blockIdx.x - d.blk0[PASS_C];
  const int Mx = LC ? LC / 2 : d.Mx, My = d.My, L = LC ? LC : d.Lr, c = d.c, nl = d.nlayers;
  const int TJ = d.tj, P = d.pc;
  const int nx = d.nx, ny = d.ny, pitch = nx + 1;
  const size_t plane = (size_t)(ny + 1) * pitch;
  const int LP = lpad(L);
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* tw = buf + 2 * P * LP;
  T* ps = reinterpret_cast<T*>(tw + d.ntw_r);  // [nl][TJ+1][Mx+1] (c > 1 only)
  const int prow = Mx + 1;
  const size_t pplane = (size_t)(TJ + 1) * prow;

  const int j0 = lb * TJ;
  const int jend = min(My, j0 + TJ - 1 + (c > 1 ? 1 : 0));  // last coarse row needed
  const int ilo = max(1, j0);
  const int ihi = min(My - 1, jend);
  const int nint = ihi >= ilo ? ihi - ilo + 1 : 0;
  const int nseq = (nl == 1) ? (nint + 1) / 2 : nint;
  const T* w = wt + d.wt_off;
  const size_t mplane = (size_t)(Mx - 1) * (My - 1);

  load_twiddles(tw, twg + d.twr_off, d.ntw_r);
  if (threadIdx.x < nseq) {
    buf[threadIdx.x * LP + pad(0)] = {T(0), T(0)};
    buf[threadIdx.x * LP + pad(Mx)] = {T(0), T(0)};
  }
  for (int k = 1 + threadIdx.x; k < Mx; k += kThreads) {
    const T* col = w + (size_t)(k - 1) * (My - 1) + (ilo - 1);
    T v[4], u[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      v[r] = r < nint ? col[r] : T(0);
      u[r] = (nl == 2 && r < nint) ? col[mplane + r] : T(0);
    }
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      if (p < nseq) {
        const cplx<T> z = (nl == 1) ? cplx<T>{v[2 * p], v[2 * p + 1]} : cplx<T>{v[p], u[p]};
        buf[p * LP + pad(k)] = z;
        buf[p * LP + pad(2 * Mx - k)] = {-z.x, -z.y};
      }
    }
  }
  const cplx<T>* Z = fft_run<T, LC>(buf, buf + P * LP, nseq, L, d.nst_r, d.stw_r, tw);

  const T wbc1 = T(1.0 - d.delta), wbc2 = T(d.delta);
  T* out = dst + d.field_off;
  // coarse psi of row jj, column i (both layers), zero on the walls
  auto coarse = [&](int jj, int i, T& v0, T& v1) {
    v0 = T(0);
    v1 = T(0);
    if (jj >= 1 && jj <= My - 1 && i >= 1 && i <= Mx - 1) {
      const int idx = jj - ilo;
      if (nl == 1) {
        const cplx<T> zi = Z[(idx >> 1) * LP + pad(i)];
        v0 = (idx & 1) ? T(0.5) * zi.x : T(-0.5) * zi.y;
      } else {
        const cplx<T> zi = Z[idx * LP + pad(i)];
        const T bt = T(-0.5) * zi.y, bc = T(0.5) * zi.x;
        v0 = bt + wbc1 * bc;  // psi_1 = psi_bt + (1 - delta) psi_bc
        v1 = bt - wbc2 * bc;  // psi_2 = psi_bt - delta psi_bc
      }
    }
  };
  const int last = (lb == d.nblk[PASS_C] - 1);
  if (c == 1) {
    const int rend = last ? ny + 1 : j0 + TJ;
    for (int x = threadIdx.x; x <= nx; x += kThreads) {
      for (int rr = j0; rr < rend; ++rr) {
        T v0, v1;
        coarse(rr, x, v0, v1);
        const size_t o = (size_t)rr * pitch + x;
        out[o] = accumulate ? out[o] + v0 : v0;
        if (nl == 2) out[o + plane] = accumulate ? out[o + plane] + v1 : v1;
      }
    }
    return;
  }
  const int nrows = jend - j0 + 1;
  for (int i = threadIdx.x; i <= Mx; i += kThreads) {
    for (int r = 0; r < nrows; ++r) {
      T v0, v1;
      coarse(j0 + r, i, v0, v1);
      ps[(size_t)r * prow + i] = v0;
      if (nl == 2) ps[pplane + (size_t)r * prow + i] = v1;
    }
  }
  __syncthreads();

  const int rbeg = c * j0;
  const int rend = last ? ny + 1 : c * (j0 + TJ);
  const T inv_c2 = T(1) / (T(c) * T(c));
  for (int x = threadIdx.x; x <= nx; x += kThreads) {
    const int I = x / c, fx = x - I * c;
    for (int l = 0; l < nl; ++l) {
      for (int rr = rbeg; rr < rend; ++rr) {
        const int J = rr / c, fy = rr - J * c;
        const T* P0 = ps + l * pplane + (size_t)(J - j0) * prow;
        T v = T(c - fx) * P0[I];
        if (fx) v += T(fx) * P0[I + 1];
        v *= T(c - fy);
        if (fy) {
          const T* P1 = P0 + prow;
          T u = T(c - fx) * P1[I];
          if (fx) u += T(fx) * P1[I + 1];
          v += T(fy) * u;
        }
        v *= inv_c2;
        const size_t o = l * plane + (size_t)rr * pitch + x;
        out[o] = accumulate ? out[o] + v : v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Launch the instantiation for the group's transform length (g.L: a length
// with a compile-time transform, or 0 for the runtime engine).
#define CGP_BY_LENGTH(LEN, CALL)  \
  switch (LEN) {                  \
    case 128: CALL(128); break;   \
    case 256: CALL(256); break;   \
    case 384: CALL(384); break;   \
    case 512: CALL(512); break;   \
    case 768: CALL(768); break;   \
    case 1024: CALL(1024); break; \
    case 1536: CALL(1536); break; \
    case 2048: CALL(2048); break; \
    default: CALL(0);             \
  }

template <typename T>
hipError_t Launch<T>::restrict_rowdst(const MemberDesc* md, const Group& g, const T* src, T* wt,
                                      const cplx<T>* tw, hipStream_t s) {
#define CALL1(LC)                                                                               \
  hipLaunchKernelGGL((k_restrict_rowdst<T, LC, 1>), dim3(g.nblk), dim3(kThreads), g.lds, s, md, \
                     g.members, g.count, src, wt, tw)
#define CALL2(LC)                                                                               \
  hipLaunchKernelGGL((k_restrict_rowdst<T, LC, 2>), dim3(g.nblk), dim3(kThreads), g.lds, s, md, \
                     g.members, g.count, src, wt, tw)
  if (g.nlayers == 1) {
    CGP_BY_LENGTH(g.L, CALL1)
  } else {
    CGP_BY_LENGTH(g.L, CALL2)
  }
#undef CALL1
#undef CALL2
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::col_solve(const MemberDesc* md, const Group& g, const T* win, T* wout,
                                const cplx<T>* tw, const double* lam, double* ctl, int split,
                                hipStream_t s) {
#define CALL(LC, SP)                                                                       \
  hipLaunchKernelGGL((k_col_solve<T, LC, SP>), dim3(g.nblk), dim3(kThreads), g.lds, s, md, \
                     g.members, g.count, win, wout, tw, lam, ctl)
#define CALL0(LC) CALL(LC, 0)
#define CALL2(LC) CALL(LC, 2)
#define CALL4(LC) CALL(LC, 4)
  // g.split: the most parts of a split restriction among the members
  if (!split || g.split == 0) {
    CGP_BY_LENGTH(g.L, CALL0)
  } else if (g.split <= 2) {
    CGP_BY_LENGTH(g.L, CALL2)
  } else {
    CGP_BY_LENGTH(g.L, CALL4)
  }
#undef CALL0
#undef CALL2
#undef CALL4
#undef CALL
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::rowdst_prolong(const MemberDesc* md, const Group& g, const T* wt, T* dst,
                                     int accumulate, const cplx<T>* tw, hipStream_t s) {
#define CALL(LC)                                                                            \
  hipLaunchKernelGGL((k_rowdst_prolong<T, LC>), dim3(g.nblk), dim3(kThreads), g.lds, s, md, \
                     g.members, g.count, wt, dst, accumulate, tw)
  CGP_BY_LENGTH(g.L, CALL)
#undef CALL
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::prepare(size_t bytes) {
  const int b = (int)bytes;
  const void* fns[] = {
#define FNS(LC)                                                    \
  reinterpret_cast<const void*>(&k_restrict_rowdst<T, LC, 1>),     \
      reinterpret_cast<const void*>(&k_restrict_rowdst<T, LC, 2>), \
      reinterpret_cast<const void*>(&k_col_solve<T, LC, 0>),       \
      reinterpret_cast<const void*>(&k_col_solve<T, LC, 2>),       \
      reinterpret_cast<const void*>(&k_col_solve<T, LC, 4>),       \
      reinterpret_cast<const void*>(&k_rowdst_prolong<T, LC>)
      FNS(0), FNS(128), FNS(256), FNS(384), FNS(512), FNS(768), FNS(1024), FNS(1536), FNS(2048)
#undef FNS
  };
  for (const void* f : fns) {
    const hipError_t e = allow_dynamic_lds(f, b);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template struct Launch<float>;
template struct Launch<double>;

#ifdef CGP_PHASE_STAMPS
hipError_t stamps_copy_solve(unsigned long long* host, int nblocks) {
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_phase_stamps));
  if (e != hipSuccess) return e;
  return hipMemcpy(host, p, sizeof(unsigned long long) * kStampSlots * (size_t)nblocks,
                   hipMemcpyDeviceToHost);
}
#endif

}  // namespace cgp
