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
#include "cgp_internal.hpp"
#include "fft_lds.hpp"

namespace cgp {

// Full weighting applied `level` times equals one tent-weighted average with
// 1-D weights (c - |d|)/c^2, |d| < c = 2^level (the l = 2 case is the
// [1 2 3 4 3 2 1]/16 stencil); it reads fine interior nodes only.
template <typename T, int C>
__device__ __forceinline__ T restrict_fixed(const T* __restrict__ f, int pitch, int I, int J) {
  if constexpr (C == 1) {
    return f[(size_t)J * pitch + I];
  } else {
    const T* base = f + (size_t)(C * J) * pitch + C * I;
    T acc = T(0);
#pragma unroll
    for (int dy = -(C - 1); dy <= C - 1; ++dy) {
      const T* row = base + (ptrdiff_t)dy * pitch;
      T racc = T(0);
#pragma unroll
      for (int dx = -(C - 1); dx <= C - 1; ++dx) racc += T(C - (dx < 0 ? -dx : dx)) * row[dx];
      acc += T(C - (dy < 0 ? -dy : dy)) * racc;
    }
    return acc * (T(1) / T(C * C * C * C));
  }
}

template <typename T>
__device__ __forceinline__ T restrict_any(const T* __restrict__ f, int pitch, int c, int I, int J) {
  if (c == 2) return restrict_fixed<T, 2>(f, pitch, I, J);
  if (c == 1) return restrict_fixed<T, 1>(f, pitch, I, J);
  if (c == 4) return restrict_fixed<T, 4>(f, pitch, I, J);
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
// Pass A.  Block = `pa` sequence pairs.  One layer: a pair is two consecutive
// coarse rows; two layers: a pair is the barotropic and the baroclinic
// combination of one coarse row.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_restrict_rowdst(
    const MemberDesc* __restrict__ md, int nm, const T* __restrict__ src, T* __restrict__ wt,
    const cplx<T>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int m = find_member(md, nm, PASS_A, blockIdx.x);
  const MemberDesc& d = md[m];
  const int lb = blockIdx.x - d.blk0[PASS_A];
  const int Mx = d.Mx, My = d.My, L = d.Lr, P = d.pa, c = d.c, nl = d.nlayers;
  const int pitch = d.nx + 1;
  const size_t plane = (size_t)(d.ny + 1) * pitch;
  const T* f = src + d.field_off;
  cplx<T>* bufA = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* bufB = bufA + P * L;
  const int per = (nl == 1) ? 2 : 1;  // coarse rows per pair
  const int rows_blk = per * P;
  const int j0 = 1 + lb * rows_blk;
  const T wbt1 = T(d.delta), wbt2 = T(1.0 - d.delta);

  for (int t = threadIdx.x; t < P * Mx; t += blockDim.x) {
    const int p = t / Mx;
    const int i = t - p * Mx;
    cplx<T>* z = bufA + p * L;
    if (i == 0) {
      z[0] = {T(0), T(0)};
      z[Mx] = {T(0), T(0)};
      continue;
    }
    T a = T(0), b = T(0);
    if (nl == 1) {
      const int ja = j0 + 2 * p;
      if (ja < My) a = restrict_any(f, pitch, c, i, ja);
      if (ja + 1 < My) b = restrict_any(f, pitch, c, i, ja + 1);
    } else {
      const int j = j0 + p;
      if (j < My) {
        const T q1 = restrict_any(f, pitch, c, i, j);
        const T q2 = restrict_any(f + plane, pitch, c, i, j);
        a = wbt1 * q1 + wbt2 * q2;  // barotropic right-hand side
        b = q1 - q2;                // baroclinic right-hand side
      }
    }
    z[i] = {a, b};
    z[2 * Mx - i] = {-a, -b};
  }
  const cplx<T>* Z = fft_lds(bufA, bufB, P, L, d.nst_r, d.rad_r, tw + d.twr_off);

  T* w = wt + d.wt_off;
  const size_t mplane = (size_t)(Mx - 1) * (My - 1);
  const int nvals = (Mx - 1) * rows_blk;
  for (int t = threadIdx.x; t < nvals; t += blockDim.x) {
    const int k = 1 + t / rows_blk;
    const int r = t - (k - 1) * rows_blk;
    const int j = j0 + r;
    if (j >= My) continue;
    const size_t o = (size_t)(k - 1) * (My - 1) + (j - 1);
    if (nl == 1) {
      const cplx<T> zk = Z[(r >> 1) * L + k];
      w[o] = (r & 1) ? T(0.5) * zk.x : T(-0.5) * zk.y;
    } else {
      const cplx<T> zk = Z[r * L + k];
      w[o] = T(-0.5) * zk.y;
      w[mplane + o] = T(0.5) * zk.x;
    }
  }
}

// ---------------------------------------------------------------------------
// Pass B.  Block = `pb` pairs of coarse spectral columns (one layer: columns
// k, k+1; two layers: barotropic and baroclinic column k).  Forward y
// transform, multiply by (2/Mx)(2/My)/lambda_kl, inverse y transform.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_col_solve(const MemberDesc* __restrict__ md, int nm,
                                                        T* __restrict__ wt,
                                                        const cplx<T>* __restrict__ tw,
                                                        const double* __restrict__ lam) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int m = find_member(md, nm, PASS_B, blockIdx.x);
  const MemberDesc& d = md[m];
  const int lb = blockIdx.x - d.blk0[PASS_B];
  const int Mx = d.Mx, My = d.My, L = d.Lc, P = d.pb, nl = d.nlayers;
  const int ny1 = My - 1;
  cplx<T>* bufA = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* bufB = bufA + P * L;
  T* w = wt + d.wt_off;
  const size_t mplane = (size_t)(Mx - 1) * (My - 1);
  const double* lamx = lam + d.lam_off;
  const double* lamy = lamx + (Mx - 1);
  const double scale = 4.0 / ((double)Mx * (double)My);
  const double shift = d.f1 + d.f2;  // Helmholtz shift of the baroclinic mode

  // column indices (1-based) of the two sequences of pair p; 0 = absent
  auto cols = [&](int p, int& ka, int& kb) {
    if (nl == 1) {
      ka = 1 + 2 * (lb * P + p);
      kb = ka + 1;
      if (ka > Mx - 1) ka = 0;
      if (kb > Mx - 1) kb = 0;
    } else {
      ka = 1 + lb * P + p;
      if (ka > Mx - 1) ka = 0;
      kb = ka;
    }
  };
  auto col_ptr = [&](int seq, int k) -> T* {
    // seq 0 / 1 of the pair; two layers: seq 1 is the baroclinic plane
    return w + ((nl == 2 && seq == 1) ? mplane : 0) + (size_t)(k - 1) * ny1;
  };

  for (int t = threadIdx.x; t < P * My; t += blockDim.x) {
    const int p = t / My;
    const int l = t - p * My;
    cplx<T>* z = bufA + p * L;
    if (l == 0) {
      z[0] = {T(0), T(0)};
      z[My] = {T(0), T(0)};
      continue;
    }
    int ka, kb;
    cols(p, ka, kb);
    const T a = ka ? col_ptr(0, ka)[l - 1] : T(0);
    const T b = kb ? col_ptr(1, kb)[l - 1] : T(0);
    z[l] = {a, b};
    z[2 * My - l] = {-a, -b};
  }
  cplx<T>* Z = fft_lds(bufA, bufB, P, L, d.nst_c, d.rad_c, tw + d.twc_off);
  cplx<T>* Y = (Z == bufA) ? bufB : bufA;

  for (int t = threadIdx.x; t < P * My; t += blockDim.x) {
    const int p = t / My;
    const int l = t - p * My;
    cplx<T>* y = Y + p * L;
    if (l == 0) {
      y[0] = {T(0), T(0)};
      y[My] = {T(0), T(0)};
      continue;
    }
    int ka, kb;
    cols(p, ka, kb);
    const cplx<T> zl = Z[p * L + l];
    T a = T(0), b = T(0);
    if (ka) a = T(-0.5) * zl.y * T(scale / (lamx[ka - 1] + lamy[l - 1]));
    if (kb) {
      const double lb_ = lamx[kb - 1] + lamy[l - 1] - (nl == 2 ? shift : 0.0);
      b = T(0.5) * zl.x * T(scale / lb_);
    }
    y[l] = {a, b};
    y[2 * My - l] = {-a, -b};
  }
  cplx<T>* Zs = (Z == bufA) ? bufA : bufB;  // scratch for the second transform
  const cplx<T>* R = fft_lds(Y, Zs, P, L, d.nst_c, d.rad_c, tw + d.twc_off);

  for (int t = threadIdx.x; t < P * ny1; t += blockDim.x) {
    const int p = t / ny1;
    const int l = 1 + (t - p * ny1);
    int ka, kb;
    cols(p, ka, kb);
    const cplx<T> r = R[p * L + l];
    if (ka) col_ptr(0, ka)[l - 1] = T(-0.5) * r.y;
    if (kb) col_ptr(1, kb)[l - 1] = T(0.5) * r.x;
  }
}

// ---------------------------------------------------------------------------
// Pass C.  Block owns coarse rows j0 .. j0+tj-1 and writes the fine rows
// c*j0 .. c*(j0+tj)-1 (the last block also the top wall row).  It
// synthesises coarse rows j0 .. j0+tj-1 (+1 halo row when c > 1), keeps them
// in LDS with their zero walls, and interpolates bilinearly.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_rowdst_prolong(const MemberDesc* __restrict__ md,
                                                             int nm, const T* __restrict__ wt,
                                                             T* __restrict__ dst, int accumulate,
                                                             const cplx<T>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int m = find_member(md, nm, PASS_C, blockIdx.x);
  const MemberDesc& d = md[m];
  const int lb = blockIdx.x - d.blk0[PASS_C];
  const int Mx = d.Mx, My = d.My, L = d.Lr, c = d.c, nl = d.nlayers, TJ = d.tj;
  const int nx = d.nx, ny = d.ny, pitch = nx + 1;
  const size_t plane = (size_t)(ny + 1) * pitch;
  const int PC = d.pc;
  cplx<T>* bufA = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* bufB = bufA + PC * L;
  T* ps = reinterpret_cast<T*>(bufB + PC * L);  // [nl][TJ+1][Mx+1]
  const int prow = Mx + 1;
  const size_t pplane = (size_t)(TJ + 1) * prow;

  const int j0 = lb * TJ;
  const int jend = min(My, j0 + TJ - 1 + (c > 1 ? 1 : 0));  // last coarse row needed
  const int ilo = max(1, j0);
  const int ihi = min(My - 1, jend);
  const int nint = ihi >= ilo ? ihi - ilo + 1 : 0;
  const int npairs = (nl == 1) ? (nint + 1) / 2 : nint;
  const T* w = wt + d.wt_off;
  const size_t mplane = (size_t)(Mx - 1) * (My - 1);

  for (int t = threadIdx.x; t < npairs * Mx; t += blockDim.x) {
    const int i = t / npairs;  // pair index fastest: neighbouring rows of one k
    const int p = t - i * npairs;
    cplx<T>* z = bufA + p * L;
    if (i == 0) {
      z[0] = {T(0), T(0)};
      z[Mx] = {T(0), T(0)};
      continue;
    }
    T a, b;
    const size_t kbase = (size_t)(i - 1) * (My - 1);
    if (nl == 1) {
      const int ja = ilo + 2 * p;
      a = w[kbase + ja - 1];
      b = (ja + 1 <= ihi) ? w[kbase + ja] : T(0);
    } else {
      const int j = ilo + p;
      a = w[kbase + j - 1];
      b = w[mplane + kbase + j - 1];
    }
    z[i] = {a, b};
    z[2 * Mx - i] = {-a, -b};
  }
  const cplx<T>* Z = fft_lds(bufA, bufB, npairs, L, d.nst_r, d.rad_r, tw + d.twr_off);
  // fft_lds may have left its result in bufB; ps lies beyond both buffers.

  const int nrows = jend - j0 + 1;
  const T wbc1 = T(1.0 - d.delta), wbc2 = T(d.delta);
  for (int t = threadIdx.x; t < nrows * prow; t += blockDim.x) {
    const int r = t / prow;
    const int i = t - r * prow;
    const int jj = j0 + r;
    T v0 = T(0), v1 = T(0);
    if (jj >= 1 && jj <= My - 1 && i >= 1 && i <= Mx - 1) {
      const int idx = jj - ilo;
      if (nl == 1) {
        const cplx<T> zi = Z[(idx >> 1) * L + i];
        v0 = (idx & 1) ? T(0.5) * zi.x : T(-0.5) * zi.y;
      } else {
        const cplx<T> zi = Z[idx * L + i];
        const T bt = T(-0.5) * zi.y, bc = T(0.5) * zi.x;
        v0 = bt + wbc1 * bc;  // psi_1 = psi_bt + (1 - delta) psi_bc
        v1 = bt - wbc2 * bc;  // psi_2 = psi_bt - delta psi_bc
      }
    }
    ps[(size_t)r * prow + i] = v0;
    if (nl == 2) ps[pplane + (size_t)r * prow + i] = v1;
  }
  __syncthreads();

  const int last = (lb == d.nblk[PASS_C] - 1);
  const int rbeg = c * j0;
  const int rend = last ? ny + 1 : c * (j0 + TJ);
  const T inv_c2 = T(1) / (T(c) * T(c));
  T* out = dst + d.field_off;
  const int nfr = rend - rbeg;
  for (int t = threadIdx.x; t < nfr * pitch; t += blockDim.x) {
    const int rr = rbeg + t / pitch;
    const int x = t - (rr - rbeg) * pitch;
    const int J = rr / c, fy = rr - J * c;
    const int I = x / c, fx = x - I * c;
    const int r = J - j0;
    for (int l = 0; l < nl; ++l) {
      const T* P0 = ps + l * pplane + (size_t)r * prow;
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

// ---------------------------------------------------------------------------
template <typename T>
hipError_t Launch<T>::restrict_rowdst(const MemberDesc* md, int nm, int nblk, size_t lds,
                                      const T* src, T* wt, const cplx<T>* tw, hipStream_t s) {
  hipLaunchKernelGGL(k_restrict_rowdst<T>, dim3(nblk), dim3(kThreads), lds, s, md, nm, src, wt, tw);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::col_solve(const MemberDesc* md, int nm, int nblk, size_t lds, T* wt,
                                const cplx<T>* tw, const double* lam, hipStream_t s) {
  hipLaunchKernelGGL(k_col_solve<T>, dim3(nblk), dim3(kThreads), lds, s, md, nm, wt, tw, lam);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::rowdst_prolong(const MemberDesc* md, int nm, int nblk, size_t lds,
                                     const T* wt, T* dst, int accumulate, const cplx<T>* tw,
                                     hipStream_t s) {
  hipLaunchKernelGGL(k_rowdst_prolong<T>, dim3(nblk), dim3(kThreads), lds, s, md, nm, wt, dst,
                     accumulate, tw);
  return hipGetLastError();
}

template struct Launch<float>;
template struct Launch<double>;

}  // namespace cgp
