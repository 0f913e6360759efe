// Persistent stage kernel of ensembles: ONE launch per RK3 stage advances
// every member through pass B (y transforms and eigenvalue divide of the
// coarse solve, Sec. 4.3) and the fused stage pass (inverse x transform,
// prolongation, Arakawa right-hand side and RK3 combine, and the next stage's
// restriction and x transform; Sec. 3.1, 4.1, 4.2).
//
// Work is a queue of tiles in the workspace: every pass-B tile (b_tile
// column pairs of one member) precedes every fused tile (f_tile row blocks of
// one member), members in order within each kind.  A workgroup takes the
// next tile with one atomic increment of the queue head and runs it with the
// same block-level code as the per-pass kernels (col_solve.hpp,
// fused_stage.hpp), so a member gets the same bits either way.  The only
// dependency inside a stage is per member: its fused tiles read the psi
// spectra every one of its pass-B tiles writes, so finished pass-B blocks
// are added to their member's counter with a release, and a workgroup's
// first fused tile of a member begins with thread 0 waiting (acquire) until
// that counter holds the member's pass-B block count.  Deadlock-free for any grid: a workgroup reaches a fused tile
// only after every pass-B tile has been taken, and pass-B tiles never wait.
// The wait is bounded all the same (kSpinLimit polls); a tile that gives up
// sets the sticky fault flag and goes on, so the launch always drains.  The
// last workgroup to leave resets the queue head, the exit count and the
// member counters for the next launch (no memset node in captured graphs).
//
// Counters (int32, workspace): [0] queue head, [1] workgroups done, [2] fault
// flag, [3 + m] pass-B blocks of member m finished in this stage.
#define CGP_OPAQUE_TID 1  // the block-level code runs in a loop over tiles
#include "cgp_internal.hpp"
#include "col_solve.hpp"
#include "fft_lds.hpp"
#include "fused_stage.hpp"

namespace cgp {

// Polls of a fused tile's wait (each about 0.1-1 us) before it gives up: far
// beyond any real wait (a stage's pass B takes well under a millisecond).
constexpr int kSpinLimit = 1 << 20;

template <typename T>
__device__ __forceinline__ void persistent_b(const MemberDesc& d, int lb, const T* wt, T* wt2,
                                             const cplx<T>* tw, const double* lam, double* ctl,
                                             unsigned char* smem, double* red) {
  switch (d.Lc) {
    case 256: col_solve_block<T, 256, kFusedThreads>(d, lb, wt, wt2, tw, lam, ctl, smem, red); break;
    case 512: col_solve_block<T, 512, kFusedThreads>(d, lb, wt, wt2, tw, lam, ctl, smem, red); break;
    case 768: col_solve_block<T, 768, kFusedThreads>(d, lb, wt, wt2, tw, lam, ctl, smem, red); break;
    default: col_solve_block<T, 1024, kFusedThreads>(d, lb, wt, wt2, tw, lam, ctl, smem, red);
  }
}

template <typename T>
__device__ __forceinline__ void persistent_f(const MemberDesc& d, int lb, const T* wt2, T* wnext,
                                             const cplx<T>* tw, const T* ws, const T* forcing,
                                             const T* wn, T* out, double a, double b,
                                             StepCtl ctl, unsigned char* smem) {
  switch (d.Lr) {
    case 128:
      fused_stage_block<T, 2, 2, 128, true>(d, lb, wt2, wnext, tw, ws, forcing, wn, out, nullptr,
                                            a, b, ctl, smem);
      break;
    case 256:
      fused_stage_block<T, 2, 2, 256, true>(d, lb, wt2, wnext, tw, ws, forcing, wn, out, nullptr,
                                            a, b, ctl, smem);
      break;
    case 384:
      fused_stage_block<T, 2, 2, 384, true>(d, lb, wt2, wnext, tw, ws, forcing, wn, out, nullptr,
                                            a, b, ctl, smem);
      break;
    default:
      fused_stage_block<T, 2, 2, 512, true>(d, lb, wt2, wnext, tw, ws, forcing, wn, out, nullptr,
                                            a, b, ctl, smem);
  }
}

// ctl_b: the step state for pass B of a step's first stage (it sets the
// step's dt), else NULL; ctl: the fused pass's step control.
template <typename T>
__global__ __launch_bounds__(kFusedThreads, 4) void k_stage_persistent(
    const MemberDesc* __restrict__ md, const PTile* __restrict__ tiles, int ntiles,
    int* __restrict__ ctr, int nm, T* __restrict__ wt, T* __restrict__ wt2,
    const cplx<T>* __restrict__ tw, const double* __restrict__ lam, double* ctl_b,
    const T* __restrict__ ws, const T* __restrict__ forcing, const T* __restrict__ wn,
    T* __restrict__ out, double a, double b, StepCtl ctl) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_tile;
  __shared__ double red[kFusedThreads / 64];
  int* head = ctr;
  int* exited = ctr + 1;
  int* fault = ctr + 2;
  int* done_b = ctr + 3;
  // the next tile index, the same in every thread (uniform: scalar loads)
  auto next_tile = [&]() {
    if (threadIdx.x == 0) s_tile = atomicAdd(head, 1);
    __syncthreads();
    const int i = __builtin_amdgcn_readfirstlane(s_tile);
    __syncthreads();  // every thread has read s_tile before thread 0 may rewrite it
    return i;
  };
  // pass-B tiles come first in the queue: this loop ends at the first fused
  // tile (or the end), which the second loop then starts with.  Finished
  // pass-B blocks are published per member with one release (a write-back of
  // the XCD's L2) when the workgroup moves on to another member or leaves the
  // pass-B tiles, not per tile; every workgroup publishes before it can wait.
  int i = next_tile();
  int pend_m = -1, pend_n = 0;
  auto publish = [&]() {
    if (pend_n > 0 && threadIdx.x == 0)
      __hip_atomic_fetch_add(done_b + pend_m, pend_n, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    pend_n = 0;
  };
  for (; i < ntiles; i = next_tile()) {
    const PTile tl = tiles[i];
    if (tl.kind != 0) break;
    if (tl.member != pend_m) {
      publish();
      pend_m = tl.member;
    }
    const MemberDesc& d = md[tl.member];
    for (int k = 0; k < tl.count; ++k) {
      persistent_b<T>(d, tl.lb0 + k, wt, wt2, tw, lam, ctl_b, smem, red);
      __syncthreads();  // the block's stores are issued and its LDS is free
    }
    pend_n += tl.count;
  }
  publish();
  // a workgroup waits (and acquires) once per member: later tiles of the
  // member it has waited for need neither
  int ready_m = -1;
  for (; i < ntiles; i = next_tile()) {
    const PTile tl = tiles[i];
    const MemberDesc& d = md[tl.member];
    if (tl.member != ready_m) {
      if (threadIdx.x == 0) {
        const int need = d.nblk[PASS_B];
        int polls = 0;
        while (__hip_atomic_load(done_b + tl.member, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT) < need) {
          __builtin_amdgcn_s_sleep(2);
          // after a fault every wait gives up at once, so that the launch drains
          if (++polls > kSpinLimit ||
              __hip_atomic_load(fault, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            __hip_atomic_store(fault, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the member's psi spectra
      }
      __syncthreads();
      ready_m = tl.member;
    }
    for (int k = 0; k < tl.count; ++k) {
      persistent_f<T>(d, tl.lb0 + k, wt2, wt, tw, ws, forcing, wn, out, a, b, ctl, smem);
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    const int n = __hip_atomic_fetch_add(exited, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (n == (int)gridDim.x - 1) {  // every other workgroup has left: reset for the next launch
      for (int m = 0; m < nm; ++m)
        __hip_atomic_store(done_b + m, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(head, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(exited, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

template <typename T>
hipError_t PersistLaunch<T>::stage(const MemberDesc* md, const PTile* tiles, int ntiles, int* ctr,
                                   int nm, int grid, size_t lds, T* wt, T* wt2,
                                   const cplx<T>* tw, const double* lam, double* ctl_b,
                                   const T* ws, const T* forcing, const T* wn, T* out, double a,
                                   double b, StepCtl ctl, hipStream_t s) {
  hipLaunchKernelGGL((k_stage_persistent<T>), dim3(grid), dim3(kFusedThreads), lds, s, md, tiles,
                     ntiles, ctr, nm, wt, wt2, tw, lam, ctl_b, ws, forcing, wn, out, a, b, ctl);
  return hipGetLastError();
}

template <typename T>
hipError_t PersistLaunch<T>::prepare(size_t bytes) {
  return allow_dynamic_lds(reinterpret_cast<const void*>(&k_stage_persistent<T>), (int)bytes);
}

template <typename T>
hipError_t PersistLaunch<T>::blocks_per_cu(size_t lds, int* n) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      n, reinterpret_cast<const void*>(&k_stage_persistent<T>), kFusedThreads, lds);
}

template struct PersistLaunch<float>;
template struct PersistLaunch<double>;

}  // namespace cgp
