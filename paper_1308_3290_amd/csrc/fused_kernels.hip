// Pass C + D fused (one layer): inverse x sine transform of the coarse
// spectra (Sec. 4.3), bilinear prolongation (Sec. 3.1) into LDS, and the
// Arakawa right-hand side with the TVD-RK3 stage combine (Sec. 4.1, 4.2), so
// that the prolonged psi never travels through HBM.  Optionally followed by
// pass A of the next stage (restriction and forward x transform of the new
// vorticity), which then needs no launch and no read of it from HBM.
//
// A block owns coarse rows j0 .. j0+TJ-1 and writes omega_{s+1} on the fine
// rows C*j0 .. C*(j0+TJ)-1 (the last block also the top wall row).  The
// stencil on those rows needs psi on one more fine row above and below, i.e.
// the coarse rows j0-1 .. j0+TJ, which the block synthesises itself (TJ + 2
// rows in at most (TJ + 3)/2 complex sequences) and keeps in LDS.  Each
// thread then owns a fine column and interpolates psi at its column and both
// neighbours for all of the block's rows in registers; the row weights are
// compile-time constants.  The step size comes from the step state (adaptive
// steps, Sec. 4.2); the last stage of a step leaves the velocity maxima of
// the block's coarse psi rows for the next step's size.
//
// Latency: a single basin has one block per CU, so a block's phases do not
// overlap with other blocks.  The twiddles and spectra are loaded first (the
// transform waits for them only); once they are in LDS the forcing and
// omega_n are issued, and they arrive while the transform runs.  The
// vorticity rows are issued with the spectra at c = 1, 2 and 4 (measured
// faster, for single basins and ensembles, once the first barrier no longer
// waits for them) and with the forcing in the split blocks of c = 8.  Rows are at most kFusedMaxNx + 1 nodes
// wide.
#include "cgp_internal.hpp"
#include "fft_lds.hpp"
#include "fused_stage.hpp"
#include "stencil.hpp"

namespace cgp {

template <typename T, int C, int TJ, int LC, bool NEXT, bool NTS>
__global__ __launch_bounds__(kFusedThreads, fused_waves_per_simd(C, LC, TJ, sizeof(T))) void
k_prolong_stencil(
    const MemberDesc* __restrict__ md, const int* __restrict__ grp, int ng, int nblk,
    const T* __restrict__ wt, T* __restrict__ wnext, const cplx<T>* __restrict__ twg,
    const T* __restrict__ ws, const T* __restrict__ forcing, const T* __restrict__ wn,
    T* __restrict__ out, T* __restrict__ psi_out, double a_, double b_, StepCtl ctl) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int bid = xcd_contiguous(blockIdx.x, nblk);
  const MemberDesc& d = md[group_member(md, grp, ng, PASS_CD, bid)];
  const int lb = bid - d.blk0[PASS_CD];
  if constexpr (C >= 4 && split_blocks(C) == 2) {
    // two blocks per coarse row: the share index selects the row weights
    if (lb & 1)
      fused_stage_block<T, C, TJ, LC, NEXT, false, NTS, 1>(d, lb, wt, wnext, twg, ws, forcing, wn,
                                                           out, psi_out, a_, b_, ctl, smem);
    else
      fused_stage_block<T, C, TJ, LC, NEXT, false, NTS, 0>(d, lb, wt, wnext, twg, ws, forcing, wn,
                                                           out, psi_out, a_, b_, ctl, smem);
  } else {
    static_assert(C < 4 || split_blocks(C) == 1, "one or two blocks per coarse row");
    fused_stage_block<T, C, TJ, LC, NEXT, true, NTS>(d, lb, wt, wnext, twg, ws, forcing, wn,
                                                        out, psi_out, a_, b_, ctl, smem);
  }
}

// g.L = (c << 16) | transform length with a compile-time transform (or 0).
template <typename T>
hipError_t Launch<T>::prolong_stencil(const MemberDesc* md, const Group& g, const T* wt,
                                      T* wnext, const cplx<T>* tw, const T* ws,
                                      const T* forcing, const T* wn, T* out, T* psi_out,
                                      double a, double b, StepCtl ctl, bool nt_store,
                                      hipStream_t s) {
#define LAUNCH(C, TJ, LC, NX, NTS)                                                      \
  hipLaunchKernelGGL((k_prolong_stencil<T, C, TJ, LC, NX, NTS>), dim3(g.nblk),          \
                     dim3(kFusedThreads), g.lds, s, md, g.members, g.count, g.nblk, wt, \
                     wnext, tw, ws, forcing, wn, out, psi_out, a, b, ctl)
// rows hold at most kFusedMaxNx intervals, so c = 1, 2, 4, 8 have transform
// lengths of at most 1024, 512, 256, 128
#define BY_LEN1(NX, NTS)                           \
  switch (g.L & 0xffff) {                          \
    case 128: LAUNCH(1, 4, 128, NX, NTS); break;   \
    case 256: LAUNCH(1, 4, 256, NX, NTS); break;   \
    case 384: LAUNCH(1, 4, 384, NX, NTS); break;   \
    case 512: LAUNCH(1, 4, 512, NX, NTS); break;   \
    case 768: LAUNCH(1, 4, 768, NX, NTS); break;   \
    case 1024: LAUNCH(1, 4, 1024, NX, NTS); break; \
    default: LAUNCH(1, 4, 0, NX, NTS);             \
  }
#define BY_LEN2T(TJ, NX, NTS)                     \
  switch (g.L & 0xffff) {                         \
    case 128: LAUNCH(2, TJ, 128, NX, NTS); break; \
    case 256: LAUNCH(2, TJ, 256, NX, NTS); break; \
    case 384: LAUNCH(2, TJ, 384, NX, NTS); break; \
    case 512: LAUNCH(2, TJ, 512, NX, NTS); break; \
    default: LAUNCH(2, TJ, 0, NX, NTS);           \
  }
// c = 2: g.rows2 coarse rows per block (cgp_config.fused_rows)
#define BY_LEN2(NX, NTS) \
  if (g.rows2 == 4) {    \
    BY_LEN2T(4, NX, NTS) \
  } else {               \
    BY_LEN2T(2, NX, NTS) \
  }
#define BY_LEN4(NX, NTS)                         \
  switch (g.L & 0xffff) {                        \
    case 128: LAUNCH(4, 1, 128, NX, NTS); break; \
    case 256: LAUNCH(4, 1, 256, NX, NTS); break; \
    default: LAUNCH(4, 1, 0, NX, NTS);           \
  }
#define BY_LEN8(NX, NTS)                         \
  switch (g.L & 0xffff) {                        \
    case 128: LAUNCH(8, 1, 128, NX, NTS); break; \
    default: LAUNCH(8, 1, 0, NX, NTS);           \
  }
#define BY_C(NX, NTS)                     \
  switch (g.L >> 16) {                    \
    case 1: BY_LEN1(NX, NTS); break;      \
    case 2: BY_LEN2(NX, NTS); break;      \
    case 4: BY_LEN4(NX, NTS); break;      \
    case 8: BY_LEN8(NX, NTS); break;      \
    default: return hipErrorInvalidValue; \
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
#undef BY_LEN1
#undef BY_LEN2
#undef BY_LEN2T
#undef BY_LEN4
#undef BY_LEN8
#undef LAUNCH
  return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::prepare_fused(size_t bytes) {
  const int b = (int)bytes;
  const void* fns[] = {
#define K(C, TJ, LC)                                                                \
  reinterpret_cast<const void*>(&k_prolong_stencil<T, C, TJ, LC, false, false>),    \
      reinterpret_cast<const void*>(&k_prolong_stencil<T, C, TJ, LC, true, false>), \
      reinterpret_cast<const void*>(&k_prolong_stencil<T, C, TJ, LC, true, true>)
      K(1, 4, 0), K(1, 4, 128), K(1, 4, 256), K(1, 4, 384), K(1, 4, 512), K(1, 4, 768),
      K(1, 4, 1024), K(2, 2, 0), K(2, 2, 128), K(2, 2, 256), K(2, 2, 384), K(2, 2, 512),
      K(2, 4, 0), K(2, 4, 128), K(2, 4, 256), K(2, 4, 384), K(2, 4, 512),
      K(4, 1, 0), K(4, 1, 128), K(4, 1, 256), K(8, 1, 0), K(8, 1, 128)
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

#ifdef CGP_PHASE_STAMPS
hipError_t stamps_copy_fused(unsigned long long* host, int nblocks) {
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_phase_stamps));
  if (e != hipSuccess) return e;
  return hipMemcpy(host, p, sizeof(unsigned long long) * kStampSlots * (size_t)nblocks,
                   hipMemcpyDeviceToHost);
}
#endif

}  // namespace cgp
