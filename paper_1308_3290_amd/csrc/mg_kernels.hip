// Multigrid V-cycles for the coarse Dirichlet Poisson problem: an iterative
// black-box solver under CGP (Sec. 3 wraps any coarse solver), in place of
// the sine-transform solve of Sec. 4.3.  V(2,2) cycles with red-black
// Gauss-Seidel smoothing (red: i + j even; pre-smoothing red then black,
// post-smoothing black then red), full weighting of the residual and
// bilinear interpolation of the correction (the Sec. 3.1 operators),
// coarsening while both interval counts are even and at least 8, and the
// coarsest grid solved exactly by its dense inverse (built on the host in
// FP64).  One kernel per operation and level; node arrays with a zero ring.
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

// One half sweep of Gauss-Seidel on the interior nodes of one colour:
// u = (ax (uE + uW) + ay (uN + uS) - f) / (2 ax + 2 ay).
template <typename T>
__global__ __launch_bounds__(256) void k_mg_smooth(T* __restrict__ u, const T* __restrict__ f,
                                                   int nx, int ny, T ax, T ay, T inv_d,
                                                   int color) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (nx - 1) * (ny - 1)) return;
  const int j = 1 + k / (nx - 1), i = 1 + k % (nx - 1);
  if (((i + j) & 1) != color) return;
  const int p = nx + 1;
  const size_t o = (size_t)j * p + i;
  u[o] = (ax * (u[o + 1] + u[o - 1]) + ay * (u[o + p] + u[o - p]) - f[o]) * inv_d;
}

// fc = full weighting of the residual f - Lap_h u (each coarse interior node
// evaluates the residual at its nine fine nodes), 0 on the coarse ring.
template <typename T>
__global__ __launch_bounds__(256) void k_mg_residual_restrict(const T* __restrict__ u,
                                                              const T* __restrict__ f, int nx,
                                                              int ny, T ax, T ay,
                                                              T* __restrict__ fc) {
  const int nxc = nx / 2, nyc = ny / 2;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (nxc + 1) * (nyc + 1)) return;
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
  fc[k] = v;
}

// u += bilinear interpolation of the coarse correction uc at fine interior nodes.
template <typename T>
__global__ __launch_bounds__(256) void k_mg_prolong_add(const T* __restrict__ uc, int nx, int ny,
                                                        T* __restrict__ u) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (nx - 1) * (ny - 1)) return;
  const int j = 1 + k / (nx - 1), i = 1 + k % (nx - 1);
  const int pc = nx / 2 + 1;
  const int I = i >> 1, J = j >> 1;
  const T* c0 = uc + (size_t)J * pc + I;
  T v;
  if (!(i & 1) && !(j & 1)) v = c0[0];
  else if (!(j & 1)) v = T(0.5) * (c0[0] + c0[1]);
  else if (!(i & 1)) v = T(0.5) * (c0[0] + c0[pc]);
  else v = T(0.25) * (c0[0] + c0[1] + c0[pc] + c0[pc + 1]);
  u[(size_t)j * (nx + 1) + i] += v;
}

// Coarsest grid: u = A^-1 f on the nb interior nodes (row-major), A^-1 dense
// in FP64.
template <typename T>
__global__ __launch_bounds__(256) void k_mg_bottom(const double* __restrict__ minv, int nb,
                                                   const T* __restrict__ f, int nx,
                                                   T* __restrict__ u) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nb) return;
  const int n1 = nx - 1, p = nx + 1;
  const double* row = minv + (size_t)k * nb;
  double s = 0.0;
  for (int m = 0; m < nb; ++m) s += row[m] * (double)f[(size_t)(1 + m / n1) * p + 1 + m % n1];
  u[(size_t)(1 + k / n1) * p + 1 + k % n1] = T(s);
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
                                          double dy, T* fc, hipStream_t s) {
  hipLaunchKernelGGL(k_mg_residual_restrict<T>,
                     grid_for((long long)(nx / 2 + 1) * (ny / 2 + 1)), dim3(256), 0, s, u, f, nx,
                     ny, T(1.0 / (dx * dx)), T(1.0 / (dy * dy)), fc);
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
