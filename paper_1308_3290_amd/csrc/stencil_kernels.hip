// Fine-grid kernels of the CGP step on gfx950:
//   pass D     right-hand side G (Arakawa Jacobian of Sec. 4.1, beta term,
//              Laplacian eddy viscosity, forcing, two-layer coupling and
//              bottom drag) fused with the TVD-RK3 stage combine (Sec. 4.2);
//   adjoint D  the transposed right-hand side of one stage (one layer, FP64);
//   diagnostics and a non-finite check (deterministic two-stage reductions).
//
// One thread per fine node, 64 x 4 node tiles (one wavefront per tile row),
// neighbour values through the vector L1/L2.  The boundary ring of every
// output is written as zero; the ring of every vorticity-like input is read
// as zero whatever it holds.
#include "cgp_internal.hpp"
#include "stencil.hpp"

namespace cgp {

template <typename T>
__global__ __launch_bounds__(kTileX* kTileY) void k_stencil_rk3(
    const MemberDesc* __restrict__ md, int nm, const T* __restrict__ ws, const T* __restrict__ psi,
    const T* __restrict__ forcing, const T* __restrict__ wn, T* __restrict__ out, double a_,
    double b_, StepCtl ctl) {
  const int m = find_member(md, nm, PASS_D, blockIdx.x);
  const MemberDesc& d = md[m];
  const int lb = blockIdx.x - d.blk0[PASS_D];
  const int nx = d.nx, ny = d.ny, pitch = nx + 1;
  const int tiles_x = (nx + kTileX) / kTileX;
  const int by = lb / tiles_x, bx = lb - by * tiles_x;
  const int i = bx * kTileX + (threadIdx.x & (kTileX - 1));
  const int j = by * kTileY + (threadIdx.x / kTileX);
  const bool track = wants_vmax(d, ctl);  // last stage of an adaptive step
  double vmx = 0.0, vmy = 0.0;
  if (i <= nx && j <= ny) {
    const size_t plane = (size_t)(ny + 1) * pitch;
    const size_t o = d.field_off + (size_t)j * pitch + i;
    const int nl = d.nlayers;
    if (i == 0 || j == 0 || i == nx || j == ny) {
      out[o] = T(0);
      if (nl == 2) out[o + plane] = T(0);
    } else {
      const T dt = stage_dt<T>(d, ctl), a = T(a_), b = T(b_);
      const T cj = T(d.cj), cb = T(d.cb);
      const T idx2 = T(d.idx2), idy2 = T(d.idy2);
      const T nu = T(d.inv_re);
      const T* W = ws + d.field_off;
      const T* PS = psi + d.field_off;
      if (nl == 1) {
        const Nbr<T> p = load_nbr(PS, pitch, i, j);
        const Nbr<T> q = load_nbr_masked(W, pitch, nx, ny, i, j);
        const T G = -cj * arakawa12(p, q) - cb * beta3(p) + nu * lap5(q, idx2, idy2) +
                    forcing[o];
        T v = b * (q.C + dt * G);
        if (a_ != 0.0) v += a * wn[o];
        out[o] = v;
        if (track) {
          vmx = (double)fabs(p.E - p.W);
          vmy = (double)fabs(p.N - p.S);
        }
      } else {
        const T F1 = T(d.f1), F2 = T(d.f2), drag = T(d.drag);
        const Nbr<T> p1 = load_nbr(PS, pitch, i, j);
        const Nbr<T> p2 = load_nbr(PS + plane, pitch, i, j);
        const Nbr<T> q1 = load_nbr_masked(W, pitch, nx, ny, i, j);
        const Nbr<T> q2 = load_nbr_masked(W + plane, pitch, nx, ny, i, j);
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
                     forcing[o];
        const T G2 = -cj * arakawa12(p2, q2) - cb * beta3(p2) + nu * lap5(z2, idx2, idy2) -
                     drag * z2.C;
        T v1 = b * (q1.C + dt * G1);
        T v2 = b * (q2.C + dt * G2);
        if (a_ != 0.0) {
          v1 += a * wn[o];
          v2 += a * wn[o + plane];
        }
        out[o] = v1;
        out[o + plane] = v2;
        if (track) {
          vmx = (double)fmax(fabs(p1.E - p1.W), fabs(p2.E - p2.W));
          vmy = (double)fmax(fabs(p1.N - p1.S), fabs(p2.N - p2.S));
        }
      }
    }
  }
  if (track) put_vmax(d, ctl, lb, vmx, vmy, 2.0 * d.dx, 2.0 * d.dy);
}

// ---------------------------------------------------------------------------
// Adjoint of one stage's right-hand side (one layer, FP64).  mu = b dt lam_in.
//   lam_out = b lam_in + J(psi_s, mu) + inv_re Lap(mu) [+ acc]
//   psi_src = -J(omega_s, mu) + inv_ro J(mu, y)
//   acc = a lam_in (acc_mode 0) / acc += a lam_in (1) / read into lam_out (2)
//   gF += mu
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kTileX* kTileY) void k_adjoint_stencil(
    const MemberDesc* __restrict__ md, const double* __restrict__ lam_in,
    const double* __restrict__ ws, const double* __restrict__ psi, double* __restrict__ lam_out,
    double* __restrict__ psi_src, double* __restrict__ acc, double* __restrict__ gF, double a,
    double b, int acc_mode) {
  const MemberDesc& d = md[0];
  const int nx = d.nx, ny = d.ny, pitch = nx + 1;
  const int tiles_x = (nx + kTileX) / kTileX;
  const int by = blockIdx.x / tiles_x, bx = blockIdx.x - by * tiles_x;
  const int i = bx * kTileX + (threadIdx.x & (kTileX - 1));
  const int j = by * kTileY + (threadIdx.x / kTileX);
  if (i > nx || j > ny) return;
  const size_t o = (size_t)j * pitch + i;
  if (i == 0 || j == 0 || i == nx || j == ny) {
    lam_out[o] = 0.0;
    psi_src[o] = 0.0;
    if (acc_mode == 0) acc[o] = 0.0;
    return;
  }
  const double cj = d.cj, cb = d.cb;
  const double idx2 = d.idx2, idy2 = d.idy2;
  const double bdt = b * d.dt;
  Nbr<double> mu = load_nbr_masked(lam_in, pitch, nx, ny, i, j);
  const double lc = mu.C;
  mu.C *= bdt; mu.E *= bdt; mu.W *= bdt; mu.N *= bdt; mu.S *= bdt;
  mu.NE *= bdt; mu.NW *= bdt; mu.SE *= bdt; mu.SW *= bdt;
  const Nbr<double> p = load_nbr(psi, pitch, i, j);
  const Nbr<double> w = load_nbr_masked(ws, pitch, nx, ny, i, j);
  double lo = b * lc + cj * arakawa12(p, mu) + d.inv_re * lap5(mu, idx2, idy2);
  if (acc_mode == 0) acc[o] = a * lc;
  else if (acc_mode == 1) acc[o] += a * lc;
  else lo += acc[o];
  lam_out[o] = lo;
  psi_src[o] = -cj * arakawa12(w, mu) + cb * beta3(mu);
  gF[o] += mu.C;
}

// ---------------------------------------------------------------------------
// Diagnostics (eq. 26).  Per layer the x-link energy, y-link energy and
// enstrophy sums.  Block b takes the node rows b, b + nblk, ... (one row per
// block on most grids), thread t the columns t, t + 256, ...; the sums are
// reduced in a fixed order (wave butterflies, then the four waves, then the
// blocks in index order), so a call gives the same bits every time.
// ---------------------------------------------------------------------------
// Sums of v[0..5] over the block's 256 threads in a fixed order (wave
// butterflies, then the four waves in order); sum k is returned in thread k.
__device__ __forceinline__ double block_sums6(double (&v)[6], double (*red)[6]) {
#pragma unroll
  for (int k = 0; k < 6; ++k)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < 6; ++k) red[threadIdx.x >> 6][k] = v[k];
  }
  __syncthreads();
  const int k = threadIdx.x < 6 ? threadIdx.x : 0;
  return ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
}

template <typename T>
__global__ __launch_bounds__(256) void k_diag_partial(const MemberDesc* __restrict__ md,
                                                      const T* __restrict__ w,
                                                      const T* __restrict__ psi,
                                                      double* __restrict__ partial) {
  __shared__ double red[4][6];
  const MemberDesc& d = md[0];
  const int nx = d.nx, ny = d.ny, pitch = nx + 1, nl = d.nlayers;
  const size_t n = (size_t)(ny + 1) * pitch;
  const double idx = 1.0 / d.dx, idy = 1.0 / d.dy;
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // layer l: ex, ey, z at 3 l
  for (int j = blockIdx.x; j <= ny; j += gridDim.x) {
    const bool rowin = j >= 1 && j <= ny - 1;
    for (int i = threadIdx.x; i <= nx; i += 256) {
      const size_t e = (size_t)j * pitch + i;
      const bool xl = rowin && i <= nx - 1;                  // link (i, j) - (i+1, j)
      const bool yl = j <= ny - 1 && i >= 1 && i <= nx - 1;  // link (i, j) - (i, j+1)
      const bool in = rowin && i >= 1 && i <= nx - 1;
      const size_t ex1 = xl ? e + 1 : e, ey1 = yl ? e + pitch : e;
#pragma unroll
      for (int l = 0; l < 2; ++l) {
        if (l < nl) {
          const T* P = psi + l * n;
          const double pc = (double)P[e], pe = (double)P[ex1], pn = (double)P[ey1];
          const double q = (double)w[l * n + e];
          const double gx = (pe - pc) * idx, gy = (pn - pc) * idy;
          acc[3 * l] += xl ? gx * gx : 0.0;
          acc[3 * l + 1] += yl ? gy * gy : 0.0;
          acc[3 * l + 2] += in ? q * q : 0.0;
        }
      }
    }
  }
  const double v = block_sums6(acc, red);
  if (threadIdx.x < 6) partial[blockIdx.x * 6 + threadIdx.x] = v;
}

__global__ __launch_bounds__(256) void k_diag_final(const MemberDesc* __restrict__ md,
                                                    const double* __restrict__ partial, int nblk,
                                                    double* __restrict__ out) {
  __shared__ double red[4][6];
  constexpr int kPer = kDiagBlocks / 256;  // partials per thread and sum
  const MemberDesc& d = md[0];
  const double area = (double)d.nx * d.dx * (double)d.ny * d.dy;
  const double f = d.dx * d.dy / (2.0 * area);
  double v[6][kPer];  // all loads first, then the sums in a fixed order
#pragma unroll
  for (int k = 0; k < 6; ++k)
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int b = threadIdx.x + 256 * q;
      const double x = partial[(b < nblk ? b : 0) * 6 + k];
      v[k][q] = b < nblk ? x : 0.0;
    }
  double sum[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    sum[k] = 0.0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) sum[k] += v[k][q];
  }
  const double tot = block_sums6(sum, red);  // total k in thread k
  __shared__ double t6[6];
  if (threadIdx.x < 6) t6[threadIdx.x] = tot;
  __syncthreads();
  if (threadIdx.x < d.nlayers) {
    const int l = threadIdx.x;
    out[2 * l] = f * (t6[3 * l] + t6[3 * l + 1]);
    out[2 * l + 1] = f * t6[3 * l + 2];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_finite_partial(const T* __restrict__ f, long long n,
                                                        int* __restrict__ partial) {
  __shared__ int red[256];
  int bad = 0;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    const T v = f[k];
    bad |= !(v - v == T(0));  // NaN or +-inf
  }
  red[threadIdx.x] = bad;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] |= red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_finite_final(const int* __restrict__ partial, int nblk, int* __restrict__ flag) {
  if (threadIdx.x == 0) {
    int bad = 0;
    for (int b = 0; b < nblk; ++b) bad |= partial[b];
    flag[0] = bad;
  }
}

// ---------------------------------------------------------------------------
template <typename T>
hipError_t Launch<T>::stencil_rk3(const MemberDesc* md, int nm, int nblk, const T* ws,
                                  const T* psi, const T* forcing, const T* wn, T* out, double a,
                                  double b, StepCtl ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_stencil_rk3<T>, dim3(nblk), dim3(kTileX * kTileY), 0, s, md, nm, ws, psi,
                     forcing, wn, out, a, b, ctl);
  return hipGetLastError();
}

__global__ void k_time_state(const MemberDesc* __restrict__ md, int nm,
                             const double* __restrict__ ctl, double* __restrict__ out) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < nm) {
    out[2 * m] = ctl[md[m].cfl_off];
    out[2 * m + 1] = ctl[md[m].cfl_off + 1];
  }
}

hipError_t time_state(const MemberDesc* md, int nm, const double* ctl, double* out,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_time_state, dim3((nm + 255) / 256), dim3(256), 0, s, md, nm, ctl, out);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::diagnostics(const MemberDesc* md, const T* w, const T* psi, double* partial,
                                  int nblk, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_partial<T>, dim3(nblk), dim3(256), 0, s, md, w, psi, partial);
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, s, md, partial, nblk, out);
  return hipGetLastError();
}

// Running sums of a packed field (time means of the statistics workloads).
template <typename T>
__global__ __launch_bounds__(256) void k_accumulate(const MemberDesc* __restrict__ md, int nm,
                                                    const T* __restrict__ f, long long n,
                                                    double* __restrict__ sum, double weight,
                                                    const double* __restrict__ ctl) {
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    double w = weight;
    if (ctl != nullptr) {
      int lo = 0, hi = nm - 1;  // the member holding element k
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (md[mid].field_off <= k) lo = mid; else hi = mid - 1;
      }
      w *= ctl[md[lo].cfl_off];
    }
    sum[k] += w * (double)f[k];
  }
}

template <typename T>
hipError_t Launch<T>::accumulate(const MemberDesc* md, int nm, const T* f, long long n,
                                 double* sum, double weight, const double* ctl, hipStream_t s) {
  const long long want = (n + 255) / 256;
  const int nblk = (int)(want < 4096 ? (want > 0 ? want : 1) : 4096);
  hipLaunchKernelGGL(k_accumulate<T>, dim3(nblk), dim3(256), 0, s, md, nm, f, n, sum, weight,
                     ctl);
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::check_finite(const T* f, long long n, int* partial, int nblk, int* flag,
                                   hipStream_t s) {
  hipLaunchKernelGGL(k_finite_partial<T>, dim3(nblk), dim3(256), 0, s, f, n, partial);
  hipLaunchKernelGGL(k_finite_final, dim3(1), dim3(64), 0, s, partial, nblk, flag);
  return hipGetLastError();
}

hipError_t AdjLaunch::stencil(const MemberDesc* md, int nblk, const double* lam_in,
                              const double* ws, const double* psi, double* lam_out,
                              double* psi_src, double* acc, double* gF, double a, double b,
                              int acc_mode, hipStream_t s) {
  hipLaunchKernelGGL(k_adjoint_stencil, dim3(nblk), dim3(kTileX * kTileY), 0, s, md, lam_in, ws,
                     psi, lam_out, psi_src, acc, gF, a, b, acc_mode);
  return hipGetLastError();
}

template struct Launch<float>;
template struct Launch<double>;

}  // namespace cgp
