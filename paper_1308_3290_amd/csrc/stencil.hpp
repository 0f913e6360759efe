// Fine-grid stencil helpers shared by the stencil kernels: the Arakawa
// Jacobian (Sec. 4.1), the beta term J(psi, y) and the 5-point Laplacian on
// 3x3 neighbourhoods held in registers.
#pragma once

#include "cgp_internal.hpp"

namespace cgp {

// Arakawa Jacobian J(p, q) of Sec. 4.1 times 12 dx dy: the sum of the
// brackets of J1, J2 and J3.  Arguments are the 3x3 neighbourhoods
// (E = i+1, W = i-1, N = j+1, S = j-1).
template <typename T>
struct Nbr {
  T C, E, W, N, S, NE, NW, SE, SW;
};

template <typename T>
__device__ __forceinline__ T arakawa12(const Nbr<T>& p, const Nbr<T>& q) {
  const T j1 = -(q.E - q.W) * (p.N - p.S) + (q.N - q.S) * (p.E - p.W);
  const T j2 = -q.E * (p.NE - p.SE) + q.W * (p.NW - p.SW) + q.N * (p.NE - p.NW) -
               q.S * (p.SE - p.SW);
  const T j3 = -q.NE * (p.N - p.E) + q.SW * (p.W - p.S) + q.NW * (p.N - p.W) -
               q.SE * (p.E - p.S);
  return j1 + j2 + j3;
}

// J(p, y) times 3 dx: the Jacobian with the coordinate y reduces to a centred
// x difference of p with corner averaging.
template <typename T>
__device__ __forceinline__ T beta3(const Nbr<T>& p) {
  return (p.E - p.W) + T(0.25) * ((p.NE - p.NW) + (p.SE - p.SW));
}

template <typename T>
__device__ __forceinline__ Nbr<T> load_nbr(const T* __restrict__ f, int pitch, int i, int j) {
  const T* c = f + (size_t)j * pitch + i;
  Nbr<T> n;
  n.C = c[0];
  n.E = c[1];
  n.W = c[-1];
  n.N = c[pitch];
  n.S = c[-pitch];
  n.NE = c[pitch + 1];
  n.NW = c[pitch - 1];
  n.SE = c[-pitch + 1];
  n.SW = c[-pitch - 1];
  return n;
}

// Same, with ring nodes read as zero.
template <typename T>
__device__ __forceinline__ Nbr<T> load_nbr_masked(const T* __restrict__ f, int pitch, int nx,
                                                  int ny, int i, int j) {
  Nbr<T> n = load_nbr(f, pitch, i, j);
  if (i == 1) { n.W = T(0); n.NW = T(0); n.SW = T(0); }
  if (i == nx - 1) { n.E = T(0); n.NE = T(0); n.SE = T(0); }
  if (j == 1) { n.S = T(0); n.SE = T(0); n.SW = T(0); }
  if (j == ny - 1) { n.N = T(0); n.NE = T(0); n.NW = T(0); }
  return n;
}

template <typename T>
__device__ __forceinline__ T lap5(const Nbr<T>& q, T idx2, T idy2) {
  return (q.E - T(2) * q.C + q.W) * idx2 + (q.N - T(2) * q.C + q.S) * idy2;
}

// Full weighting applied log2(C) times (Sec. 3.1) has 1-D weights
// (C - |d|)/C^2, |d| < C.  Split restriction: fine row C j + e (0 <= e < C)
// carries a share of coarse row j's restriction (y weight C - e) and of
// coarse row j+1's (y weight e), so coarse row j's restriction is the sum of
// the parts from the blocks owning fine rows C j .. C j + C-1 (the a parts)
// and C j - C+1 .. C j - 1 (the b parts of the coarse row below).  This gives
// the y-weighted sums of one fine column over the CR rows e0 .. e0+CR-1 a
// block owns (r[k] = the column's value on fine row C j + e0 + k); the x
// weights (xweight over the columns' sums) and 1/C^4 follow.  The same code
// serves pass A and the fused pass, so both give the same bits.
template <typename T, int C, int CR>
__device__ __forceinline__ void split_yweights(const T* r, int e0, T& a, T& b) {
  T sa = T(0), sb = T(0);
#pragma unroll
  for (int k = 0; k < CR; ++k) sa += T(C - (e0 + k)) * r[k];
#pragma unroll
  for (int k = 0; k < CR; ++k)
    if (e0 + k > 0) sb += T(e0 + k) * r[k];
  a = sa;
  b = sb;
}

// x-weighted sum of one fine row at coarse column i (weights C - |dx|).
template <typename T, int C>
__device__ __forceinline__ T xweight(const T* row) {
  T acc = T(0);
#pragma unroll
  for (int dx = -(C - 1); dx <= C - 1; ++dx) acc += T(C - (dx < 0 ? -dx : dx)) * row[dx];
  return acc;
}

// y-weighted sum of one fine column over the 2C-1 rows of a coarse row's
// stencil (weights C - |dy|); col[0] is the lowest of them.  A whole
// restriction (not split) takes these first and then xweight over the
// columns' sums, times 1/C^4: pass A and the fused kernels hold a column's
// rows in one thread, so only one value per coarse row crosses threads.
template <typename T, int C>
__device__ __forceinline__ T yweight(const T* col) {
  T acc = T(0);
#pragma unroll
  for (int dy = -(C - 1); dy <= C - 1; ++dy) acc += T(C - (dy < 0 ? -dy : dy)) * col[dy + C - 1];
  return acc;
}

// Remap block b of nb so that the blocks dispatched to one XCD (round robin,
// b mod 8) own a contiguous range of work items: neighbouring bands share
// their halo rows in one L2.
__device__ __forceinline__ int xcd_contiguous(int b, int nb) {
  const int per = nb >> 3, rem = nb & 7;
  const int x = b & 7, i = b >> 3;
  return x * per + min(x, rem) + i;
}

}  // namespace cgp
