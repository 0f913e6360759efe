// Pass C + D fused (one layer): inverse x sine transform of the coarse
// spectra (Sec. 4.3), bilinear prolongation (Sec. 3.1) into LDS, and the
// Arakawa right-hand side with the TVD-RK3 stage combine (Sec. 4.1, 4.2), so
// that the prolonged psi never travels through HBM.
//
// A block owns coarse rows j0 .. j0+tj-1 (tj = 2) and writes omega_{s+1} on
// the fine rows c*j0 .. c*(j0+tj)-1 (the last block also the top wall row).
// The stencil on those rows needs psi on one more fine row above and below,
// i.e. the coarse rows j0-1 .. j0+tj, which the block synthesises itself (at
// most four rows: two complex sequences).  Each thread then owns one fine
// column and slides down the block's rows with a 3 x 3 vorticity window in
// registers.
#include "cgp_internal.hpp"
#include "fft_lds.hpp"
#include "stencil.hpp"

namespace cgp {

// NR: the most fine output rows a block writes (c * tj, +1 for the top wall
// row of the last block).
template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_prolong_stencil(
    const MemberDesc* __restrict__ md, const int* __restrict__ grp, int ng, int nblk,
    const T* __restrict__ wt, const cplx<T>* __restrict__ twg, const T* __restrict__ ws,
    const T* __restrict__ forcing, const T* __restrict__ wn, T* __restrict__ out, double a_,
    double b_) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int bid = xcd_contiguous(blockIdx.x, nblk);
  const MemberDesc& d = md[group_member(md, grp, ng, PASS_CD, bid)];
  const int lb = bid - d.blk0[PASS_CD];
  const int Mx = d.Mx, My = d.My, L = d.Lr, c = d.c, TJ = kFusedTj;
  const int nx = d.nx, ny = d.ny, pitch = nx + 1;
  const int LP = lpad(L);

  // LDS: [ max(FFT buffers, fine psi rows) | twiddles | coarse psi rows ]
  const int nx1 = nx + 1;
  const int head =
      (max(4 * LP * (int)sizeof(cplx<T>), (c * TJ + 3) * nx1 * (int)sizeof(T)) + 15) & ~15;
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem + head);
  T* psc = reinterpret_cast<T*>(tw + d.ntw_r);  // coarse psi rows j0-1 .. j0+TJ
  T* psf = reinterpret_cast<T*>(smem);          // fine psi rows R0-1 .. R1 (after the FFT)
  const int prow = Mx + 1;

  const int j0 = lb * TJ;
  const int ilo = max(1, j0 - 1);
  const int ihi = min(My - 1, j0 + TJ);
  const int nint = ihi >= ilo ? ihi - ilo + 1 : 0;
  const int nseq = (nint + 1) / 2;
  const T* w = wt + d.wt_off;

  // ---- coarse spectra rows ilo..ihi -> two packed sequences, odd extension
  load_twiddles(tw, twg + d.twr_off, d.ntw_r);
  if (threadIdx.x < nseq) {
    buf[threadIdx.x * LP + pad(0)] = {T(0), T(0)};
    buf[threadIdx.x * LP + pad(Mx)] = {T(0), T(0)};
  }
  for (int k = 1 + threadIdx.x; k < Mx; k += kThreads) {
    const T* col = w + (size_t)(k - 1) * (My - 1) + (ilo - 1);
    T v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = r < nint ? col[r] : T(0);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      if (p < nseq) {
        const cplx<T> z = {v[2 * p], v[2 * p + 1]};
        buf[p * LP + pad(k)] = z;
        buf[p * LP + pad(2 * Mx - k)] = {-z.x, -z.y};
      }
    }
  }
  const cplx<T>* Z = fft_lds<T>(buf, buf + 2 * LP, nseq, L, d.nst_r, d.stw_r, tw);

  // ---- coarse psi rows J = j0-1 .. j0+TJ (zero walls) into psc
  for (int i = threadIdx.x; i <= Mx; i += kThreads) {
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
  __syncthreads();

  // ---- fine psi rows R0-1 .. R1 into psf (bilinear, Sec. 3.1)
  const int last = (lb == d.nblk[PASS_CD] - 1);
  const int R0 = c * j0;
  const int R1 = last ? ny + 1 : c * (j0 + TJ);  // exclusive end of the output rows
  const int nfr = R1 - R0;                       // output rows (<= c*TJ + 1)
  const T inv_c2 = T(1) / (T(c) * T(c));
  for (int x = threadIdx.x; x <= nx; x += kThreads) {
    const int I = x / c, fx = x - I * c;
    for (int r = 0; r < nfr + 2; ++r) {
      const int rr = R0 - 1 + r;  // fine row
      T v = T(0);
      if (rr >= 0 && rr <= ny) {
        const int J = rr / c, fy = rr - J * c;
        const T* P0 = psc + (J - (j0 - 1)) * prow;
        v = T(c - fx) * P0[I];
        if (fx) v += T(fx) * P0[I + 1];
        v *= T(c - fy);
        if (fy) {
          const T* P1 = P0 + prow;
          T u = T(c - fx) * P1[I];
          if (fx) u += T(fx) * P1[I + 1];
          v += T(fy) * u;
        }
        v *= inv_c2;
      }
      psf[r * pitch + x] = v;
    }
  }
  __syncthreads();

  // ---- stencil + RK3 on fine rows R0 .. R1-1, one column per thread
  const T dt = T(d.dt), a = T(a_), b = T(b_);
  const T cj = T(1.0 / (12.0 * d.dx * d.dy));
  const T cb = T(d.inv_ro / (3.0 * d.dx));
  const T idx2 = T(1.0 / (d.dx * d.dx)), idy2 = T(1.0 / (d.dy * d.dy));
  const T nu = T(d.inv_re);
  const T* W = ws + d.field_off;
  const T* FF = forcing + d.field_off;
  const T* WN = wn + d.field_off;
  T* O = out + d.field_off;
  for (int x = threadIdx.x; x <= nx; x += kThreads) {
    if (x == 0 || x == nx) {
      for (int r = 0; r < nfr; ++r) O[(size_t)(R0 + r) * pitch + x] = T(0);
      continue;
    }
    // vorticity rows r-1, r, r+1 (fine rows R0-2+r ..) at columns x-1, x, x+1,
    // sliding down the block's rows; the ring is read as 0
    auto load = [&](int r, T& w0, T& w1, T& w2) {
      const int rr = R0 - 1 + r;
      const bool in = r < nfr + 2 && rr >= 1 && rr <= ny - 1;
      const T* row = W + (size_t)(in ? rr : 0) * pitch + x;
      w0 = (in && x > 1) ? row[-1] : T(0);
      w1 = in ? row[0] : T(0);
      w2 = (in && x < nx - 1) ? row[1] : T(0);
    };
    T s0, s1, s2, c0, c1, c2;
    load(0, s0, s1, s2);
    load(1, c0, c1, c2);
#pragma unroll
    for (int r = 1; r <= NR; ++r) {
      T n0, n1, n2;
      load(r + 1, n0, n1, n2);
      const int rr = R0 - 1 + r;
      const size_t o = (size_t)rr * pitch + x;
      if (r <= nfr) {
        if (rr == 0 || rr == ny) {
          O[o] = T(0);
        } else {
          const T* pc = psf + r * pitch + x;
          Nbr<T> p, q;
          p.C = pc[0]; p.E = pc[1]; p.W = pc[-1];
          p.N = pc[pitch]; p.S = pc[-pitch];
          p.NE = pc[pitch + 1]; p.NW = pc[pitch - 1];
          p.SE = pc[-pitch + 1]; p.SW = pc[-pitch - 1];
          q.C = c1; q.E = c2; q.W = c0;
          q.N = n1; q.S = s1;
          q.NE = n2; q.NW = n0;
          q.SE = s2; q.SW = s0;
          const T G = -cj * arakawa12(p, q) - cb * beta3(p) + nu * lap5(q, idx2, idy2) + FF[o];
          T v = b * (q.C + dt * G);
          if (a_ != 0.0) v += a * WN[o];
          O[o] = v;
        }
      }
      s0 = c0; s1 = c1; s2 = c2;
      c0 = n0; c1 = n1; c2 = n2;
    }
  }
}

// g.L carries the group's coarsening factor c (1, 2 or 4).
template <typename T>
hipError_t Launch<T>::prolong_stencil(const MemberDesc* md, const Group& g, const T* wt,
                                      const cplx<T>* tw, const T* ws, const T* forcing,
                                      const T* wn, T* out, double a, double b, hipStream_t s) {
  switch (g.L) {
    case 1:
      hipLaunchKernelGGL((k_prolong_stencil<T, kFusedTj + 1>), dim3(g.nblk), dim3(kThreads), g.lds,
                         s, md, g.members, g.count, g.nblk, wt, tw, ws, forcing, wn, out, a, b);
      break;
    case 2:
      hipLaunchKernelGGL((k_prolong_stencil<T, 2 * kFusedTj + 1>), dim3(g.nblk), dim3(kThreads),
                         g.lds, s, md, g.members, g.count, g.nblk, wt, tw, ws, forcing, wn, out,
                         a, b);
      break;
    default:
      hipLaunchKernelGGL((k_prolong_stencil<T, 4 * kFusedTj + 1>), dim3(g.nblk), dim3(kThreads),
                         g.lds, s, md, g.members, g.count, g.nblk, wt, tw, ws, forcing, wn, out,
                         a, b);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::prepare_fused(size_t bytes) {
  const int b = (int)bytes;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_prolong_stencil<T, 3>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, b);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_prolong_stencil<T, 5>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, b);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_prolong_stencil<T, 9>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, b);
  return e;
}

template struct Launch<float>;
template struct Launch<double>;

}  // namespace cgp
