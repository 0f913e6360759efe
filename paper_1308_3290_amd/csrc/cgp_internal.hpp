// Internal declarations shared by the host runtime and the gfx950 kernels of
// the CGP time step.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Thread index within the block, as the block-level device code reads it.
// A translation unit whose kernels run that code inside a loop over work
// tiles (the persistent stage kernel) defines CGP_OPAQUE_TID before the
// first include: every use then re-reads the index through an opaque
// zero, so that the many per-thread index values derived from it are
// recomputed in each tile instead of being hoisted out of the tile loop and
// held live across it (which exceeds the register budget and spills).
#ifdef CGP_OPAQUE_TID
#define CGP_TID                                 \
  ({                                            \
    int z_;                                     \
    asm volatile("s_mov_b32 %0, 0" : "=s"(z_)); \
    (int)threadIdx.x + z_;                      \
  })
#else
#define CGP_TID ((int)threadIdx.x)
#endif

namespace cgp {

constexpr int kMaxStages = 12;   // radix stages of one complex FFT (L <= 4096)
constexpr int kThreads = 256;    // threads per block of the transform kernels
constexpr int kTileX = 64;       // stencil tile (one wavefront wide)
constexpr int kTileY = 4;

// PASS_CD: passes C and D fused (one layer).
enum Pass { PASS_A = 0, PASS_B = 1, PASS_C = 2, PASS_D = 3, PASS_CD = 4, NUM_PASSES = 5 };

// Fused C + D pass: rows of at most kFusedMaxNx intervals, coarsening
// factors 1, 2, 4 and 8 (two layers: 1, 2 and 4); a block owns
// fused_tj(c, layers) coarse rows and writes at most fused_nr(c, layers) fine
// rows.  Two layers at c = 1: one coarse row per block (the block's three
// sequences of up to 1024 points fill the LDS).
constexpr int kFusedMaxNx = 512;
constexpr int kFusedThreads = 512;  // threads per block of the fused pass
constexpr int kDiagBlocks = 2048;   // most blocks (partial sums) of the diagnostics
__host__ __device__ constexpr int fused_tj(int c, int nl = 1) {
  return c >= 4 ? 1 : (c == 2 ? 2 : (nl == 2 ? 1 : 4));
}
// One layer at c >= 4 (a coarse row per block, split restrictions): a
// block owns at most kSplitRows of the coarse row's c fine rows, so that
// c = 8 runs two blocks per coarse row (one CU each for a single basin)
// instead of one block doing eight rows' stencils.
constexpr int kSplitRows = 4;
__host__ __device__ constexpr int split_blocks(int c) { return c > kSplitRows ? c / kSplitRows : 1; }
__host__ __device__ constexpr int fused_nr(int c, int nl = 1) {
  return (nl == 1 && c >= 4 ? c / split_blocks(c) : c * fused_tj(c, nl)) + 1;
}
// complex sequences the fused one-layer pass transforms at most: the coarse
// rows j0-1 .. j0+TJ in whole pairs (2m-1, 2m)
__host__ __device__ constexpr int fused_nseq(int tj) { return (tj + 3) / 2; }

// Per-basin descriptor, uploaded once at create.  Offsets are in elements of
// the handle's scalar type T unless stated.
struct MemberDesc {
  int nx, ny;           // fine intervals
  int c;                // coarsening factor 2^level
  int Mx, My;           // coarse intervals
  int nlayers;
  int Lr, Lc;           // complex FFT lengths 2*Mx (rows) and 2*My (columns)
  int nst_r, nst_c;     // radix stage counts
  int stw_r[kMaxStages], stw_c[kMaxStages];  // stage words: radix, log2 span, table offset
  int ntw_r, ntw_c;                          // twiddle table sizes (complex values)
  int pa;               // pass A: sequences per block (1)
  int a_first, a_rows;  // pass A, one layer: block b packs coarse rows a_first + b a_rows
                        // (+1 when a_rows = 2; row 0, a wall, as 0), as the fused pass does
  int pb;               // pass B: sequences per block (1)
  int tj;               // pass C: coarse rows owned per block
  int pc;               // pass C: sequence pairs per block (derived from tj)
  int blk0[NUM_PASSES]; // first block of this member in its launch of each pass
  int nblk[NUM_PASSES]; // blocks of this member in each pass
  long long field_off;  // packed fine fields ([L][ny+1][nx+1] per member)
  long long wt_off;     // coarse spectra: L modes x (Mx-1) x (My-1), k-major
  // One layer at c >= 4 (fused steps): the restriction of a coarse row j is
  // split into the sums over the own fine rows of the blocks that cover
  // fine rows c (j-1) + 1 .. c j + c-1 (split_yweights): a block of coarse
  // row j's h-th share of its fine rows stores its part of row j at
  // wt_off + 2h split_off and its part of row j+1 at wt_off + (2h+1)
  // split_off; pass B adds the nparts parts (2 split_blocks(c)).
  // split_off = 0, nparts = 0: the spectra hold whole restrictions.
  long long split_off;
  int nparts;
  long long twr_off;    // row twiddle tables, in complex elements of T (ntw_r values)
  long long twc_off;    // column twiddle tables (ntw_c values)
  long long lam_off;    // doubles: lambda_x (Mx-1) then lambda_y (My-1)
  double dx, dy;
  double inv_re, inv_ro, f1, f2, drag, dt;
  double delta;         // barotropic weight f2/(f1+f2) (0.5 if f1 = f2 = 0)
  // stencil coefficients: 1/(12 dx dy), inv_ro/(3 dx), 1/dx^2, 1/dy^2
  double cj, cb, idx2, idy2;
  // step size (Sec. 4.2): cfl = 0 keeps dt; cfl > 0 adapts it.  The member's
  // step state sits at cfl_off in the step-state region (see StepCtl); the
  // last stage of a step leaves kVmaxSlots maxima per block of its launch
  // (npart blocks)
  double cfl, hmin;
  long long cfl_off;
  int npart;
};

// Per-wave maxima one block of a stage kernel leaves (512 threads at most).
constexpr int kVmaxSlots = 8;

// Step-size state, per member at md.cfl_off of a double region:
// [0] the dt of the current (latest) step, [1] the model time advanced so far,
// [2 .. 2 + npart kVmaxSlots) the largest |d psi/dx|, |d psi/dy| (centred
// differences, interior nodes) seen by each wave of the last stage of the
// latest step.  Pass B of a step's first stage turns these into that step's
// dt: min(dt, cfl min(dx, dy) / max) (dt itself when the max is 0); the
// stage kernels read it.
struct StepCtl {
  double* w;  // the region; NULL: fixed dt from the descriptor, no maxima
  int last;   // the launch is the last stage of a step: leave the maxima
};

// First stage of a step: member d's dt for the step (Sec. 4.2) from the
// velocity maxima the previous step's last stage left (0 before the first
// step: dt itself), and the model time.  Every thread of the block (NT
// threads) calls it; red is LDS scratch of NT / 64 doubles.
template <int NT>
__device__ __forceinline__ void update_step_dt(const MemberDesc& d, double* ctl, double* red) {
  double* st = ctl + d.cfl_off;
  double m = 0.0;
  if (d.cfl > 0) {
    const int n = d.npart * kVmaxSlots;
    for (int i = CGP_TID; i < n; i += NT) m = fmax(m, st[2 + i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((CGP_TID & 63) == 0) red[CGP_TID >> 6] = m;
    __syncthreads();
    if (CGP_TID == 0)
      for (int i = 1; i < NT / 64; ++i) m = fmax(m, red[i]);
  }
  if (CGP_TID == 0) {
    const double dt = m > 0 ? fmin(d.dt, d.cfl * d.hmin / m) : d.dt;
    st[0] = dt;
    st[1] += dt;
  }
}

// The dt a stage kernel applies.
template <typename T>
__device__ __forceinline__ T stage_dt(const MemberDesc& d, const StepCtl& c) {
  return (c.w != nullptr && d.cfl > 0) ? T(c.w[d.cfl_off]) : T(d.dt);
}

// Whether a stage launch leaves the velocity maxima for member d.
__device__ __forceinline__ bool wants_vmax(const MemberDesc& d, const StepCtl& c) {
  return c.w != nullptr && c.last && d.cfl > 0;
}

// Store the wave's largest scaled velocity max(mx / hx, my / hy) (mx, my:
// the largest differences of psi along x and y the lane saw, hx, hy the
// spacings they span) in slot (lb, wave) of member d.  Every lane of the wave
// must call it.
__device__ __forceinline__ void put_vmax(const MemberDesc& d, const StepCtl& c, int lb, double mx,
                                         double my, double hx, double hy) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mx = fmax(mx, __shfl_xor(mx, o));
    my = fmax(my, __shfl_xor(my, o));
  }
  if ((CGP_TID & 63) == 0)
    c.w[d.cfl_off + 2 + (long long)lb * kVmaxSlots + (CGP_TID >> 6)] = fmax(mx / hx, my / hy);
}

// The velocity maxima of a fused stage block, from its coarse psi rows in
// LDS (psc row r = coarse row j0-1+r, r = 0..TJ+1, columns 0..Mx, zero walls)
// instead of the prolonged fine psi: bilinear interpolation is linear in
// each coarse cell, so for C >= 2 the fine centred difference at a node
// inside a cell is that cell's slope, at a coarse node the mean of two
// slopes, and on fine rows (columns) between coarse ones a convex
// combination of the slopes of the neighbouring coarse rows (columns).  The
// largest fine centred difference is therefore the largest coarse cell slope:
// x on the interior coarse rows, y on the interior coarse columns, each
// spanning C dx (C dy).  For C = 1 the fine grid is the coarse one (centred
// differences over 2 dx, 2 dy).  Each block takes its own coarse rows j0 ..
// j0+TJ-1 (the y slopes of the cells above them); two layers pass both
// layers' rows (psc2 != NULL).  Every thread calls it.
template <typename T, int C, int TJ, int NT>
__device__ __forceinline__ void put_vmax_coarse(const MemberDesc& d, const StepCtl& ctl, int lb,
                                                const T* psc, const T* psc2, int prow, int j0) {
  const int Mx = d.Mx, My = d.My;
  double mx = 0.0, my = 0.0;
  for (int l = 0; l < (psc2 ? 2 : 1); ++l) {
    const T* P = l ? psc2 : psc;
    for (int I = CGP_TID; I < Mx; I += NT) {
#pragma unroll
      for (int r = 1; r <= TJ; ++r) {
        const int J = j0 - 1 + r;
        const T* row = P + r * prow;
        if constexpr (C == 1) {
          if (J >= 1 && J <= My - 1 && I >= 1) {
            mx = fmax(mx, (double)fabs(row[I + 1] - row[I - 1]));
            my = fmax(my, (double)fabs(row[prow + I] - row[I - prow]));
          }
        } else {
          if (J >= 1 && J <= My - 1) mx = fmax(mx, (double)fabs(row[I + 1] - row[I]));
          if (J <= My - 1 && I >= 1) my = fmax(my, (double)fabs(row[prow + I] - row[I]));
        }
      }
    }
  }
  const double k = C == 1 ? 2.0 : (double)C;
  put_vmax(d, ctl, lb, mx, my, k * d.dx, k * d.dy);
}

template <typename T>
struct cplx {
  T x, y;
};

// A store that writes through the L2 of its XCD to memory (a relaxed atomic
// store at agent scope): the kernel boundary's L2 write-back then has none
// of its lines left to write, and a reader on another XCD finds them in
// memory.  Pass B stores its solved spectra this way (512x1024 one layer:
// 0.1-1.1 us per step at l = 0-2, two layers at l = 0 135.0 -> 129.6 us).
template <typename T>
__device__ __forceinline__ void store_through(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Store of a fine-grid field element (the new vorticity); with NT written
// through the L2 (store_through), so the lines leave it as they fill instead
// of at the end of the launch.  The host asks for it when a launch has at
// most one block per CU, whose stores are then the tail of the launch (2 %
// per step for single basins with the non-temporal hint, which write-through
// stores match at one layer and beat by 1.5 us per step for two layers at
// l = 1).  With more blocks than CUs later blocks hide that tail, and
// write-through stores measured 1 % slower for the 64-basin FP64 ensemble.
// The coarse spectra, stored with a stride of one column, are slower with
// either form and use ordinary stores.  (A compile-time choice: a runtime
// branch between the two stores is merged into one ordinary store.)
template <bool NT, typename T>
__device__ __forceinline__ void store_field(T* p, T v) {
  if constexpr (NT)
    store_through(p, v);
  else
    *p = v;
}

// Two consecutive elements at an address aligned to one element, moved by one
// memory instruction (the target allows unaligned vector accesses).
template <typename T>
struct UPairOf;
template <>
struct UPairOf<double> {
  typedef double type __attribute__((ext_vector_type(2), aligned(8)));
};
template <>
struct UPairOf<float> {
  typedef float type __attribute__((ext_vector_type(2), aligned(4)));
};
template <typename T>
using upair = typename UPairOf<T>::type;

// Locate the member owning block `b` of the stencil pass (members are laid
// out in order in its grid).
__device__ inline int find_member(const MemberDesc* md, int nm, int p, int b) {
  int lo = 0, hi = nm - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (md[mid].blk0[p] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Locate the member of group `grp` (ng members, ordered by first block)
// owning block `b` of pass `p`.  A group of one member m is passed as
// ng = -(m + 1): the kernel then needs no load to find it.
__device__ __forceinline__ int group_member(const MemberDesc* md, const int* grp, int ng, int p,
                                           int b) {
  if (ng < 0) return -ng - 1;
  int lo = 0, hi = ng - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (md[grp[mid]].blk0[p] <= b) lo = mid; else hi = mid - 1;
  }
  return grp[lo];
}

// Allow kernel f up to `total` bytes of LDS per workgroup: its dynamic-LDS
// cap is set to total minus the kernel's own static LDS (the runtime rejects
// caps whose sum with the static part exceeds the workgroup's LDS).
inline hipError_t allow_dynamic_lds(const void* f, int total) {
  hipFuncAttributes a{};
  hipError_t e = hipFuncGetAttributes(&a, f);
  if (e != hipSuccess) return e;
  const int st = (int)a.sharedSizeBytes;
  return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                             total > st ? total - st : 0);
}

// One launch of a transform pass over a group of members.
struct Group {
  int L;               // transform length with a compile-time transform, or 0
                       // (fused C + D pass: (c << 16) | that length)
  int count;           // members in the group; one member m is encoded as -(m + 1)
  const int* members;  // device array of the group's member indices
  int nblk, threads;  // threads = kThreads
  size_t lds;
  int nlayers;         // layers of every member of the handle
  int split;           // the most parts of a split restriction among the members (0: none;
                       // pass B adds a member's parts)
  int rows2;           // fused pass, one layer at c = 2: coarse rows per block (2 or 4)
};

// Launch wrappers implemented in the kernel translation units.
template <typename T>
struct Launch {
  // pass A: restrict (level times) + forward x sine transform, src -> spectra
  static hipError_t restrict_rowdst(const MemberDesc* md, const Group& g, const T* src, T* wt,
                                    const cplx<T>* tw, hipStream_t s);
  // pass B: y sine transform, eigenvalue divide, y sine transform, from the
  // spectra of omega (win) to those of psi (wout)
  // With ctl != NULL (the first stage of a step) the member's first block
  // also sets the step's dt in the step state.
  // split != 0: add the B partial spectra of split members (time steps and
  // pass A); 0 where win holds whole restrictions (the adjoint's sources)
  static hipError_t col_solve(const MemberDesc* md, const Group& g, const T* win, T* wout,
                              const cplx<T>* tw, const double* lam, double* ctl, int split,
                              hipStream_t s);
  // pass C: inverse x sine transform + prolongation; accumulate != 0 adds to dst
  static hipError_t rowdst_prolong(const MemberDesc* md, const Group& g, const T* wt, T* dst,
                                   int accumulate, const cplx<T>* tw, hipStream_t s);
  // allow the transform kernels up to `bytes` of dynamic LDS per block
  static hipError_t prepare(size_t bytes);
  // passes C + D fused (one layer): x transform of the psi spectra wt,
  // prolongation into registers, stencil + RK3; with wnext != NULL also pass
  // A of the next stage on the result (spectra into wnext); with psi_out !=
  // NULL the prolonged psi is stored too
  static hipError_t prolong_stencil(const MemberDesc* md, const Group& g, const T* wt, T* wnext,
                                    const cplx<T>* tw, const T* ws, const T* forcing, const T* wn,
                                    T* out, T* psi_out, double a, double b, StepCtl ctl,
                                    bool nt_store, hipStream_t s);
  static hipError_t prepare_fused(size_t bytes);
  // the same for two layers (mode recombination and split inside; c = 1, 2, 4)
  static hipError_t prolong_stencil2(const MemberDesc* md, const Group& g, const T* wt, T* wnext,
                                     const cplx<T>* tw, const T* ws, const T* forcing,
                                     const T* wn, T* out, double a, double b, StepCtl ctl,
                                     bool nt_store, hipStream_t s);
  static hipError_t prepare_fused2(size_t bytes);
  // pass D: Arakawa right-hand side + TVD-RK3 stage combine
  static hipError_t stencil_rk3(const MemberDesc* md, int nm, int nblk, const T* ws,
                                const T* psi, const T* forcing, const T* wn, T* out, double a,
                                double b, StepCtl ctl, hipStream_t s);
  // diagnostics partial sums (2 per layer per block) + ordered final sum
  static hipError_t diagnostics(const MemberDesc* md, const T* w, const T* psi, double* partial,
                                int nblk, double* out, hipStream_t s);
  static hipError_t check_finite(const T* f, long long n, int* partial, int nblk, int* flag,
                                 hipStream_t s);
  // sum[k] += weight * w_m * f[k] (FP64) over the n packed field elements of
  // the nm members, w_m = the dt of member m's latest step (ctl != NULL) or 1
  static hipError_t accumulate(const MemberDesc* md, int nm, const T* f, long long n,
                               double* sum, double weight, const double* ctl, hipStream_t s);
};

// Persistent stage kernel of ensembles (persistent_kernels.hip): a queue of
// work tiles, pass-B tiles first.  kind 0: pass-B blocks lb0 .. lb0+count-1
// of the member; kind 1: fused-pass blocks.
struct PTile {
  int member, kind, lb0, count;
};
// Coarsening factor, row and column transform lengths the persistent kernel
// takes (compile-time transforms only, so that it stays within the
// two-blocks-per-CU register budget of the fused pass).
__host__ __device__ constexpr bool persistent_lengths(int c, int lr, int lc) {
  return c == 2 && (lr == 128 || lr == 256 || lr == 384 || lr == 512) &&
         (lc == 256 || lc == 512 || lc == 768 || lc == 1024);
}
constexpr int kPersistCounters = 3;  // head, exited, fault; then one per member

template <typename T>
struct PersistLaunch {
  // one RK3 stage of every member: pass B of the stage input's spectra wt
  // into wt2, then the fused pass from wt2 and ws into out and the next
  // spectra (wt)
  static hipError_t stage(const MemberDesc* md, const PTile* tiles, int ntiles, int* ctr, int nm,
                          int grid, size_t lds, T* wt, T* wt2, const cplx<T>* tw,
                          const double* lam, double* ctl_b, const T* ws, const T* forcing,
                          const T* wn, T* out, double a, double b, StepCtl ctl, hipStream_t s);
  static hipError_t prepare(size_t bytes);
  static hipError_t blocks_per_cu(size_t lds, int* n);
};

// Multigrid V-cycle operations on one level (an nx x ny interval node array
// with a zero ring), one launch each.
// The lowest levels of a V-cycle run in one block with every level's u and f
// in LDS (u_k at off[k], f_k right after it): at most kMgTailLevels levels
// and kMgTailLds bytes.
constexpr int kMgTailLevels = 8;
constexpr int kMgTailThreads = 1024;
constexpr size_t kMgTailLds = 64 * 1024;
template <typename T>
struct MgTail {
  int nlev = 0;
  int nx[kMgTailLevels] = {}, ny[kMgTailLevels] = {}, off[kMgTailLevels] = {};
  T ax[kMgTailLevels] = {}, ay[kMgTailLevels] = {}, inv_d[kMgTailLevels] = {};
};

template <typename T>
struct MgLaunch {
  // f0 = R^l w (coarse node array of nx/c x ny/c intervals, zero ring)
  static hipError_t restrict_field(const T* w, int nx, int ny, int c, T* f0, hipStream_t s);
  // half sweep of red-black Gauss-Seidel for Lap_h u = f on nodes i + j = color (mod 2)
  static hipError_t smooth(T* u, const T* f, int nx, int ny, double dx, double dy, int color,
                           hipStream_t s);
  // fc (nx/2 x ny/2 intervals) = full weighting of f - Lap_h u; uc = 0 (same size)
  static hipError_t residual_restrict(const T* u, const T* f, int nx, int ny, double dx,
                                      double dy, T* fc, T* uc, hipStream_t s);
  // u += bilinear interpolation of uc (nx/2 x ny/2 intervals)
  static hipError_t prolong_add(const T* uc, int nx, int ny, T* u, hipStream_t s);
  // u = minv f on the nb interior nodes of the coarsest grid
  static hipError_t bottom(const double* minv, int nb, const T* f, int nx, T* u, hipStream_t s);
  // psi (fine, nx x ny) (+)= P^l uc
  static hipError_t prolong_field(const T* uc, int nx, int ny, int c, T* psi, int accumulate,
                                  hipStream_t s);
  static hipError_t fill_zero(T* a, long long n, hipStream_t s);
  // the rest of a V-cycle from level t.nx[0] x t.ny[0] down, in one block:
  // u0, f0 that level's arrays (u0 read unless zero_u, written back)
  static hipError_t tail(const MgTail<T>& t, T* u0, const T* f0, int zero_u, const double* minv,
                         int nb, hipStream_t s);
};

// The step size of every member (the first stage of a step on handles whose
// steps launch no pass B).
hipError_t step_ctl(const MemberDesc* md, int nm, double* ctl, hipStream_t s);

// out[2m], out[2m+1] = dt of the latest step and model time of member m.
hipError_t time_state(const MemberDesc* md, int nm, const double* ctl, double* out,
                      hipStream_t s);

// Adjoint kernels (FP64 only).
struct AdjLaunch {
  // lam_out = b lam_in + J(psi_s, mu) + inv_re Lap(mu) [+ acc if add_acc];
  // psi_src = -J(omega_s, mu) + inv_ro J(mu, y); acc (+)= a lam_in; gF += mu,
  // with mu = b dt lam_in.
  static hipError_t stencil(const MemberDesc* md, int nblk, const double* lam_in,
                            const double* ws, const double* psi, double* lam_out,
                            double* psi_src, double* acc, double* gF, double a, double b,
                            int acc_mode, hipStream_t s);
  // The same stage fused with the solve of the previous stage's source (its
  // y-solved spectra wt2; NULL for the first stage of a sweep: lam_in = lin)
  // and the restriction + x transform of this stage's source (into wnext).
  // Blocks as the fused forward pass (group of pass CD).
  static hipError_t fused(const MemberDesc* md, const Group& g, const double* wt2, double* wnext,
                          const cplx<double>* tw, const double* lin, const double* ws,
                          const double* psi, double* lout, double* acc, double* gF, double a,
                          double b, int acc_mode, hipStream_t s);
  static hipError_t prepare_fused(size_t bytes);
};


// Phase stamps, compiled in only for the measurement build of the library
// (CGP_PHASE_STAMPS; libcgp_stamps.so): thread 0 of a block writes the
// device's steady clock at the phase boundaries of pass B and of the fused
// stage pass, slot s of block b (the hardware block index) at
// b * kStampSlots + s of a per-source static device array that every launch
// overwrites.  The kernels' arithmetic is unchanged; without the macro the
// stamps compile to nothing.
constexpr int kStampSlots = 8;
constexpr int kStampBlocks = 4096;
#ifdef CGP_PHASE_STAMPS
static __device__ unsigned long long g_phase_stamps[kStampBlocks * kStampSlots];
#define CGP_STAMP(slot)                                                              \
  do {                                                                               \
    if (threadIdx.x == 0 && blockIdx.x < (unsigned)::cgp::kStampBlocks)              \
      ::cgp::g_phase_stamps[blockIdx.x * ::cgp::kStampSlots + (slot)] =              \
          (unsigned long long)wall_clock64();                                        \
  } while (0)
// Copy the first nblocks blocks' stamps of pass B (solve_kernels.hip) or of
// the fused one-layer stage pass (fused_kernels.hip) to host memory.
hipError_t stamps_copy_solve(unsigned long long* host, int nblocks);
hipError_t stamps_copy_fused(unsigned long long* host, int nblocks);
#else
#define CGP_STAMP(slot) \
  do {                  \
  } while (0)
#endif

}  // namespace cgp
