// Multigrid V-cycles for the coarse Dirichlet Poisson problem: an iterative
// black-box solver under CGP (Sec. 3 wraps any coarse solver), in place of
// the sine-transform solve of Sec. 4.3.  V(2,2) cycles with red-black
// Gauss-Seidel smoothing (red: i + j even; pre-smoothing red then black,
// post-smoothing black then red), full weighting of the residual and
// bilinear interpolation of the correction (the Sec. 3.1 operators),
// coarsening while both interval counts are even and at least 8, and the
// coarsest grid solved exactly by its dense inverse (built on the host in
// FP64).  One kernel per operation and level on the finer levels; the
// lowest levels run in one block (k_mg_tail), with the same arithmetic
// (shared helpers below) in the same order.  Node arrays with a zero ring.
#include <hip/hip_runtime.h>

#include "cgp_internal.hpp"

namespace cgp {

// f0 = R^l w at the coarse interior nodes (tent weights (c - |d|)/c^2 per
// direction, c = 2^l: l full-weighting restrictions), 0 on the ring.
template <typename T>
__global__ __launch_bounds__(256) void k_mg_restrict_field(const T* __restrict__ w, int nx,
                                                           int ny, int c, T* __restrict__ f0) {
  const int Mx = nx / c, My = ny / c;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (Mx + 1) * (My + 1)) return;
  const int J = k / (Mx + 1), I = k - J * (Mx + 1);
  T v = T(0);
  if (I >= 1 && I <= Mx - 1 && J >= 1 && J <= My - 1) {
    const int pitch = nx + 1;
    const T* base = w + (size_t)(c * J) * pitch + c * I;
    T acc = T(0);
    for (int dy = -(c - 1); dy <= c - 1; ++dy) {
      const T* row = base + (ptrdiff_t)dy * pitch;
      T racc = T(0);
      for (int dx = -(c - 1); dx <= c - 1; ++dx) racc += T(c - abs(dx)) * row[dx];
      acc += T(c - abs(dy)) * racc;
    }
    const T c2 = T(c) * T(c);
    v = acc / (c2 * c2);
  }
  f0[k] = v;
}

// Gauss-Seidel update of interior node k (row-major over the interior) if it
// has the given colour: u = (ax (uE + uW) + ay (uN + uS) - f) / (2 ax + 2 ay).
template <typename T>
__device__ __forceinline__ void mg_gs_node(T* u, const T* f, int nx, int k, T ax, T ay,
                                           T inv_d, int color) {
  const int j = 1 + k / (nx - 1), i = 1 + k % (nx - 1);
  if (((i + j) & 1) != color) return;
  const int p = nx + 1;
  const size_t o = (size_t)j * p + i;
  u[o] = (ax * (u[o + 1] + u[o - 1]) + ay * (u[o + p] + u[o - p]) - f[o]) * inv_d;
}

// Full weighting of the residual f - Lap_h u at coarse node k of the
// (nx/2 + 1) x (ny/2 + 1) array (the residual at its nine fine nodes), 0 on
// the coarse ring.
template <typename T>
__device__ __forceinline__ T mg_resid_fw(const T* u, const T* f, int nx, int ny, int k, T ax,
                                         T ay) {
  const int nxc = nx / 2, nyc = ny / 2;
  const int J = k / (nxc + 1), I = k - J * (nxc + 1);
  T v = T(0);
  if (I >= 1 && I <= nxc - 1 && J >= 1 && J <= nyc - 1) {
    const int p = nx + 1;
    T acc = T(0);
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj) {
#pragma unroll
      for (int di = -1; di <= 1; ++di) {
        const size_t o = (size_t)(2 * J + dj) * p + (2 * I + di);
        const T r = f[o] - (ax * (u[o + 1] - T(2) * u[o] + u[o - 1]) +
                            ay * (u[o + p] - T(2) * u[o] + u[o - p]));
        acc += T((di == 0 ? 2 : 1) * (dj == 0 ? 2 : 1)) * r;
      }
    }
    v = acc / T(16);
  }
  return v;
}

// Bilinear interpolation of the coarse correction uc at fine interior node k
// (row-major over the interior of the nx x ny grid); returns the node's
// offset in the fine array.
template <typename T>
__device__ __forceinline__ T mg_prolong_node(const T* uc, int nx, int k, size_t& o) {
  const int j = 1 + k / (nx - 1), i = 1 + k % (nx - 1);
  const int pc = nx / 2 + 1;
  const int I = i >> 1, J = j >> 1;
  const T* c0 = uc + (size_t)J * pc + I;
  T v;
  if (!(i & 1) && !(j & 1)) v = c0[0];
  else if (!(j & 1)) v = T(0.5) * (c0[0] + c0[1]);
  else if (!(i & 1)) v = T(0.5) * (c0[0] + c0[pc]);
  else v = T(0.25) * (c0[0] + c0[1] + c0[pc] + c0[pc + 1]);
  o = (size_t)j * (nx + 1) + i;
  return v;
}

// Row k of the coarsest grid's dense inverse times f (interior nodes
// row-major), accumulated in FP64.
template <typename T>
__device__ __forceinline__ T mg_bottom_row(const double* minv, int nb, const T* f, int nx,
                                           int k) {
  const int n1 = nx - 1, p = nx + 1;
  const double* row = minv + (size_t)k * nb;
  double s = 0.0;
  for (int m = 0; m < nb; ++m) s += row[m] * (double)f[(size_t)(1 + m / n1) * p + 1 + m % n1];
  return T(s);
}

// One half sweep of Gauss-Seidel on the interior nodes of one colour.
template <typename T>
__global__ __launch_bounds__(256) void k_mg_smooth(T* __restrict__ u, const T* __restrict__ f,
                                                   int nx, int ny, T ax, T ay, T inv_d,
                                                   int color) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (nx - 1) * (ny - 1)) return;
  mg_gs_node(u, f, nx, k, ax, ay, inv_d, color);
}

// fc = full weighting of the residual f - Lap_h u (each coarse interior node
// evaluates the residual at its nine fine nodes), 0 on the coarse ring; the
// coarse correction uc starts from zero.
template <typename T>
__global__ __launch_bounds__(256) void k_mg_residual_restrict(const T* __restrict__ u,
                                                              const T* __restrict__ f, int nx,
                                                              int ny, T ax, T ay,
                                                              T* __restrict__ fc,
                                                              T* __restrict__ uc) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (nx / 2 + 1) * (ny / 2 + 1)) return;
  fc[k] = mg_resid_fw(u, f, nx, ny, k, ax, ay);
  uc[k] = T(0);
}

// u += bilinear interpolation of the coarse correction uc at fine interior nodes.
template <typename T>
__global__ __launch_bounds__(256) void k_mg_prolong_add(const T* __restrict__ uc, int nx, int ny,
                                                        T* __restrict__ u) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (nx - 1) * (ny - 1)) return;
  size_t o;
  const T v = mg_prolong_node(uc, nx, k, o);
  u[o] += v;
}

// Coarsest grid: u = A^-1 f on the nb interior nodes (row-major), A^-1 dense
// in FP64.
template <typename T>
__global__ __launch_bounds__(256) void k_mg_bottom(const double* __restrict__ minv, int nb,
                                                   const T* __restrict__ f, int nx,
                                                   T* __restrict__ u) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nb) return;
  const int n1 = nx - 1;
  u[(size_t)(1 + k / n1) * (nx + 1) + 1 + k % n1] = mg_bottom_row(minv, nb, f, nx, k);
}

// psi = P^l uc at every fine node: bilinear from the c-spaced coarse nodes
// (equal to l bilinear prolongations), optionally added.
template <typename T>
__global__ __launch_bounds__(256) void k_mg_prolong_field(const T* __restrict__ uc, int nx,
                                                          int ny, int c, T* __restrict__ psi,
                                                          int accumulate) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (nx + 1) * (ny + 1)) return;
  const int j = k / (nx + 1), i = k - j * (nx + 1);
  const int Mx = nx / c, My = ny / c, pc = Mx + 1;
  const int I = i / c, fx = i - I * c, J = j / c, fy = j - J * c;
  const int I1 = min(I + 1, Mx), J1 = min(J + 1, My);
  const T a = T(c - fx), b = T(fx), e = T(c - fy), g = T(fy);
  const T v = (a * e * uc[(size_t)J * pc + I] + b * e * uc[(size_t)J * pc + I1] +
               a * g * uc[(size_t)J1 * pc + I] + b * g * uc[(size_t)J1 * pc + I1]) /
              (T(c) * T(c));
  psi[k] = accumulate ? psi[k] + v : v;
}

// The V-cycle from level 0 of t down to the coarsest, in one block: the
// same pre-smoothing (red, black, red, black), residual restriction, zeroed
// coarse correction, bottom solve, prolongation and post-smoothing (black,
// red, black, red) as the per-level kernels, with a barrier after each step.
template <typename T>
__global__ __launch_bounds__(kMgTailThreads) void k_mg_tail(MgTail<T> t, T* __restrict__ u0,
                                                            const T* __restrict__ f0, int zero_u,
                                                            const double* __restrict__ minv,
                                                            int nb) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* lds = reinterpret_cast<T*>(smem);
  constexpr int NT = kMgTailThreads;
  const int tid = threadIdx.x;
  auto nodes = [&](int l) { return (t.nx[l] + 1) * (t.ny[l] + 1); };
  const int n0 = nodes(0);
  for (int k = tid; k < n0; k += NT) {
    lds[t.off[0] + k] = zero_u ? T(0) : u0[k];
    lds[t.off[0] + n0 + k] = f0[k];
  }
  __syncthreads();
  auto half_sweep = [&](int l, int color) {
    T* u = lds + t.off[l];
    const T* f = u + nodes(l);
    const int ni = (t.nx[l] - 1) * (t.ny[l] - 1);
    for (int k = tid; k < ni; k += NT)
      mg_gs_node(u, f, t.nx[l], k, t.ax[l], t.ay[l], t.inv_d[l], color);
    __syncthreads();
  };
  const int top = t.nlev - 1;
  for (int l = 0; l < top; ++l) {
    for (int q = 0; q < 2; ++q) {
      half_sweep(l, 0);
      half_sweep(l, 1);
    }
    const T* u = lds + t.off[l];
    const T* f = u + nodes(l);
    T* uc = lds + t.off[l + 1];
    T* fc = uc + nodes(l + 1);
    for (int k = tid; k < nodes(l + 1); k += NT) {
      fc[k] = mg_resid_fw(u, f, t.nx[l], t.ny[l], k, t.ax[l], t.ay[l]);
      uc[k] = T(0);
    }
    __syncthreads();
  }
  {
    T* u = lds + t.off[top];
    const int n1 = t.nx[top] - 1;
    for (int k = tid; k < nb; k += NT)
      u[(size_t)(1 + k / n1) * (t.nx[top] + 1) + 1 + k % n1] =
          mg_bottom_row(minv, nb, u + nodes(top), t.nx[top], k);
    __syncthreads();
  }
  for (int l = top - 1; l >= 0; --l) {
    T* u = lds + t.off[l];
    const T* uc = lds + t.off[l + 1];
    const int ni = (t.nx[l] - 1) * (t.ny[l] - 1);
    for (int k = tid; k < ni; k += NT) {
      size_t o;
      const T v = mg_prolong_node(uc, t.nx[l], k, o);
      u[o] += v;
    }
    __syncthreads();
    for (int q = 0; q < 2; ++q) {
      half_sweep(l, 1);
      half_sweep(l, 0);
    }
  }
  for (int k = tid; k < n0; k += NT) u0[k] = lds[t.off[0] + k];
}

template <typename T>
__global__ __launch_bounds__(256) void k_mg_fill(T* __restrict__ a, long long n) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) a[k] = T(0);
}

// The step size of every member for a step's first stage (handles without
// pass B launches); one block per member.
__global__ __launch_bounds__(256) void k_step_ctl(const MemberDesc* __restrict__ md,
                                                  double* __restrict__ ctl) {
  __shared__ double red[4];
  update_step_dt<256>(md[blockIdx.x], ctl, red);
}

namespace {
inline dim3 grid_for(long long n) { return dim3((unsigned)((n + 255) / 256)); }
}  // namespace

template <typename T>
hipError_t MgLaunch<T>::restrict_field(const T* w, int nx, int ny, int c, T* f0, hipStream_t s) {
  hipLaunchKernelGGL(k_mg_restrict_field<T>, grid_for((long long)(nx / c + 1) * (ny / c + 1)),
                     dim3(256), 0, s, w, nx, ny, c, f0);
  return hipGetLastError();
}

template <typename T>
hipError_t MgLaunch<T>::smooth(T* u, const T* f, int nx, int ny, double dx, double dy, int color,
                               hipStream_t s) {
  const double ax = 1.0 / (dx * dx), ay = 1.0 / (dy * dy);
  hipLaunchKernelGGL(k_mg_smooth<T>, grid_for((long long)(nx - 1) * (ny - 1)), dim3(256), 0, s,
                     u, f, nx, ny, T(ax), T(ay), T(1.0 / (2.0 * ax + 2.0 * ay)), color);
  return hipGetLastError();
}

template <typename T>
hipError_t MgLaunch<T>::residual_restrict(const T* u, const T* f, int nx, int ny, double dx,
                                          double dy, T* fc, T* uc, hipStream_t s) {
  hipLaunchKernelGGL(k_mg_residual_restrict<T>,
                     grid_for((long long)(nx / 2 + 1) * (ny / 2 + 1)), dim3(256), 0, s, u, f, nx,
                     ny, T(1.0 / (dx * dx)), T(1.0 / (dy * dy)), fc, uc);
  return hipGetLastError();
}

template <typename T>
hipError_t MgLaunch<T>::prolong_add(const T* uc, int nx, int ny, T* u, hipStream_t s) {
  hipLaunchKernelGGL(k_mg_prolong_add<T>, grid_for((long long)(nx - 1) * (ny - 1)), dim3(256), 0,
                     s, uc, nx, ny, u);
  return hipGetLastError();
}

template <typename T>
hipError_t MgLaunch<T>::bottom(const double* minv, int nb, const T* f, int nx, T* u,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_mg_bottom<T>, grid_for(nb), dim3(256), 0, s, minv, nb, f, nx, u);
  return hipGetLastError();
}

template <typename T>
hipError_t MgLaunch<T>::prolong_field(const T* uc, int nx, int ny, int c, T* psi,
                                      int accumulate, hipStream_t s) {
  hipLaunchKernelGGL(k_mg_prolong_field<T>, grid_for((long long)(nx + 1) * (ny + 1)), dim3(256),
                     0, s, uc, nx, ny, c, psi, accumulate);
  return hipGetLastError();
}

template <typename T>
hipError_t MgLaunch<T>::tail(const MgTail<T>& t, T* u0, const T* f0, int zero_u,
                             const double* minv, int nb, hipStream_t s) {
  const int last = t.nlev - 1;
  const size_t lds = ((size_t)t.off[last] + 2 * (size_t)(t.nx[last] + 1) * (t.ny[last] + 1)) *
                     sizeof(T);
  if (t.nlev < 1 || t.nlev > kMgTailLevels || lds > kMgTailLds) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mg_tail<T>, dim3(1), dim3(kMgTailThreads), lds, s, t, u0, f0, zero_u, minv,
                     nb);
  return hipGetLastError();
}

template <typename T>
hipError_t MgLaunch<T>::fill_zero(T* a, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_mg_fill<T>, grid_for(n), dim3(256), 0, s, a, n);
  return hipGetLastError();
}

hipError_t step_ctl(const MemberDesc* md, int nm, double* ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_step_ctl, dim3(nm), dim3(256), 0, s, md, ctl);
  return hipGetLastError();
}

template struct MgLaunch<float>;
template struct MgLaunch<double>;

}  // namespace cgp
