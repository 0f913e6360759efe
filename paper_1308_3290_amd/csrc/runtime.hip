// Host runtime and C ABI of the CGP time step (see include/cgp.h).
//
// A handle describes one or more basins ("members").  Everything it needs on
// the device lives in the caller's workspace, laid out as
//   [member descriptors][twiddle tables][eigenvalue tables][coarse spectra]
//   [psi][stage 1][stage 2][reduction partials]
// with 256-byte aligned regions.  Fine fields of all members are packed back
// to back in member order.  Every pass of a stage is ONE launch over all
// members; the block -> member map is a prefix sum stored in the descriptors.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <utility>
#include <vector>

#include "cgp.h"
#include "cgp_internal.hpp"
#include "fft_lds.hpp"

using namespace cgp;

namespace {

thread_local std::string g_err;

cgp_status fail(cgp_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

cgp_status hip_fail(hipError_t e, const char* what) {
  return fail(CGP_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                      \
  do {                                           \
    hipError_t e_ = (expr);                      \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

constexpr size_t kAlign = 256;
constexpr int kFiniteBlocks = 256;
constexpr size_t kMaxLds = 160 * 1024;  // LDS per workgroup on gfx950

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool pow2_or_3pow2(int n) {
  if (n <= 0) return false;
  while (n % 2 == 0) n /= 2;
  return n == 1 || n == 3;
}

// Stage words of the runtime transform (see stage_plan); returns the stage
// count and the twiddle table size in *ntw.
int plan_stages(int L, int wide_from, int* words, int* ntw) {
  const StagePlan p = stage_plan(L, wide_from);
  for (int s = 0; s < p.n; ++s) words[s] = stage_word(p.R[s], p.lns[s], p.off[s]);
  *ntw = p.ntw;
  return p.n;
}

cgp_status validate(const cgp_config* c) {
  if (!c) return fail(CGP_ERR_INVALID, "config is NULL");
  if (c->reserved != 0) return fail(CGP_ERR_INVALID, "reserved field must be 0");
  if (c->nlayers != 1 && c->nlayers != 2)
    return fail(CGP_ERR_INVALID, "nlayers must be 1 or 2 (got %d)", c->nlayers);
  if (c->dtype != CGP_F32 && c->dtype != CGP_F64)
    return fail(CGP_ERR_INVALID, "dtype must be CGP_F32 or CGP_F64 (got %d)", c->dtype);
  if (c->level < 0 || c->level > 6) return fail(CGP_ERR_INVALID, "level must be in 0..6");
  if (c->nx < 4 || c->ny < 4) return fail(CGP_ERR_INVALID, "nx, ny must be >= 4");
  const int f = 1 << c->level;
  if (c->nx % f || c->ny % f)
    return fail(CGP_ERR_INVALID, "nx=%d, ny=%d not divisible by 2^level=%d", c->nx, c->ny, f);
  const int Mx = c->nx / f, My = c->ny / f;
  if (Mx < 4 || My < 4)
    return fail(CGP_ERR_UNSUPPORTED, "coarse grid %dx%d below 4x4", Mx, My);
  if (!pow2_or_3pow2(Mx) || !pow2_or_3pow2(My))
    return fail(CGP_ERR_UNSUPPORTED, "coarse sizes %dx%d must be 2^k or 3*2^k", Mx, My);
  if (Mx > 1024 || My > 1024)
    return fail(CGP_ERR_UNSUPPORTED, "coarse size above 1024");
  if (c->nlayers == 2 && f > 1 && Mx > 512)
    return fail(CGP_ERR_UNSUPPORTED, "two-layer coarse rows above 512 with coarsening");
  const double vals[] = {c->lx, c->ly, c->y0, c->inv_re, c->inv_ro, c->f1, c->f2, c->drag, c->dt,
                         c->cfl};
  for (double v : vals)
    if (!std::isfinite(v)) return fail(CGP_ERR_INVALID, "non-finite coefficient");
  if (!(c->lx > 0) || !(c->ly > 0)) return fail(CGP_ERR_INVALID, "lx, ly must be > 0");
  if (c->inv_re < 0 || c->f1 < 0 || c->f2 < 0 || c->drag < 0)
    return fail(CGP_ERR_INVALID, "inv_re, f1, f2, drag must be >= 0");
  if (c->cfl < 0) return fail(CGP_ERR_INVALID, "cfl must be >= 0 (0: fixed dt)");
  if (c->solver != 0 && c->solver != 1)
    return fail(CGP_ERR_INVALID, "solver must be 0 (sine transform) or 1 (multigrid)");
  if (c->mg_cycles < 0 || c->mg_cycles > 1000)
    return fail(CGP_ERR_INVALID, "mg_cycles must be in 0..1000");
  if (c->fused_rows != 0 && c->fused_rows != 2 && c->fused_rows != 4)
    return fail(CGP_ERR_INVALID, "fused_rows must be 0, 2 or 4 (got %d)", c->fused_rows);
  return CGP_OK;
}

struct Layout {
  // wt: spectra of omega (pass A out, pass B in); wt2: spectra of psi (pass B
  // out, pass C / fused pass in)
  size_t desc = 0, order = 0, tw = 0, lam = 0, ctl = 0, mgm = 0, ptile = 0, pctr = 0, wt = 0,
         wt2 = 0, psi = 0, st1 = 0, st2 = 0, diag = 0, fin = 0, mg = 0, total = 0;
  long long field_elems = 0;
};

// One launch of a transform pass on the host side.
struct HostGroup {
  int L = 0;                 // launch key: compile-time transform length or 0
                             // (fused pass: (c << 16) | length)
  std::vector<int> members;  // member indices in member order
  int nblk = 0;
  size_t lds = 0;
  int order_off = 0;         // offset of the member list in the order region (ints)
};

// One level of the multigrid solver: an nx x ny interval grid (spacings dx,
// dy) with its correction u and right-hand side f (element offsets in the
// multigrid region).
struct MgLevel {
  int nx = 0, ny = 0;
  double dx = 0, dy = 0;
  long long u = 0, f = 0;
};

struct Plan {
  std::vector<MemberDesc> md;
  int solver = 0;                    // 0: sine transform, 1: multigrid
  int mg_cycles = 0;
  std::vector<MgLevel> mg;           // finest (the coarse CGP grid) first
  int mg_nb = 0;                     // unknowns of the coarsest grid
  int mg_tail = 0;                   // first level of the one-block tail (mg.size(): none)
  Layout lay;
  std::vector<HostGroup> groups[4];  // passes A, B, C and the fused C + D pass
  int nblk_d = 0;                    // pass D: one launch over every member
  int dtype = CGP_F64, nlayers = 1;
  bool fused = false;                // time steps use the fused C + D pass
  // member chains of the fused step: (pass B group, fused group) pairs with
  // the same members; the chains of a step are independent, so a captured
  // step runs them on separate streams (ensembles of several sizes)
  std::vector<std::pair<int, int>> chains;
  // persistent stage kernel (one launch per RK3 stage over every member):
  // available when every member takes it (persistent_lengths), its launch
  // setting, the LDS a workgroup needs and the most tiles the queue can hold
  bool persist_ok = false;
  cgp_launch launch{0, 1, 1, 0};
  int rows2 = 2;                     // coarse rows per fused block at c = 2 (one layer)
  size_t persist_lds = 0;
  int persist_max_tiles = 0;
};

// Group the members of one transform pass by length and size each launch.
// `len` gives a member's transform length, `fill` sets its per-block share
// for the group's block size and returns (blocks, LDS bytes).
template <typename LenF, typename FillF>
void build_groups(std::vector<MemberDesc>& md, int pass, LenF len, FillF fill,
                  std::vector<HostGroup>& groups) {
  std::map<int, int> by_len;
  for (int m = 0; m < (int)md.size(); ++m) {
    const int key = len(md[m]);
    auto it = by_len.find(key);
    if (it == by_len.end()) {
      it = by_len.emplace(key, (int)groups.size()).first;
      HostGroup g;
      g.L = key;
      groups.push_back(g);
    }
    groups[it->second].members.push_back(m);
  }
  for (HostGroup& g : groups) {
    for (int m : g.members) {
      auto r = fill(md[m], g);
      md[m].blk0[pass] = g.nblk;
      md[m].nblk[pass] = r.first;
      g.nblk += r.first;
      g.lds = std::max(g.lds, r.second);
    }
  }
}

cgp_status make_plan(const cgp_config* cfgs, int count, Plan* plan) {
  if (!cfgs || count < 1) return fail(CGP_ERR_INVALID, "need at least one member");
  const int dtype = cfgs[0].dtype, nl = cfgs[0].nlayers;
  const size_t es = dtype == CGP_F64 ? 8 : 4;
  const size_t cs = 2 * es;
  plan->dtype = dtype;
  plan->nlayers = nl;
  plan->md.assign(count, MemberDesc{});
  long long fld = 0, wt = 0, tw = 0, lam = 0;
  for (int m = 0; m < count; ++m) {
    const cgp_config& c = cfgs[m];
    cgp_status st = validate(&c);
    if (st != CGP_OK) return st;
    if (c.dtype != dtype || c.nlayers != nl)
      return fail(CGP_ERR_INVALID, "all members must share dtype and nlayers");
    if (c.solver != cfgs[0].solver)
      return fail(CGP_ERR_INVALID, "all members must share the coarse solver");
    if (c.fused_rows != cfgs[0].fused_rows)
      return fail(CGP_ERR_INVALID, "all members must share fused_rows");
    MemberDesc& d = plan->md[m];
    d.nx = c.nx;
    d.ny = c.ny;
    d.c = 1 << c.level;
    d.Mx = c.nx / d.c;
    d.My = c.ny / d.c;
    d.nlayers = nl;
    d.Lr = 2 * d.Mx;
    d.Lc = 2 * d.My;
    d.nst_r = plan_stages(d.Lr, kWideRows, d.stw_r, &d.ntw_r);
    d.nst_c = plan_stages(d.Lc, kWideCols, d.stw_c, &d.ntw_c);
    d.field_off = fld;
    fld += (long long)nl * (c.ny + 1) * (c.nx + 1);
    d.wt_off = wt;
    wt += (long long)nl * (d.Mx - 1) * (d.My - 1);
    d.twr_off = tw;
    tw += d.ntw_r;
    d.twc_off = tw;
    tw += d.ntw_c;
    d.lam_off = lam;
    lam += (d.Mx - 1) + (d.My - 1);
    d.dx = c.lx / c.nx;
    d.dy = c.ly / c.ny;
    d.inv_re = c.inv_re;
    d.inv_ro = c.inv_ro;
    d.f1 = nl == 2 ? c.f1 : 0.0;
    d.f2 = nl == 2 ? c.f2 : 0.0;
    d.drag = nl == 2 ? c.drag : 0.0;
    d.dt = c.dt;
    d.cfl = c.cfl;
    d.hmin = std::min(c.lx / c.nx, c.ly / c.ny);
    d.delta = (d.f1 + d.f2 > 0) ? d.f2 / (d.f1 + d.f2) : 0.5;
    d.cj = 1.0 / (12.0 * d.dx * d.dy);
    d.cb = d.inv_ro / (3.0 * d.dx);
    d.idx2 = 1.0 / (d.dx * d.dx);
    d.idy2 = 1.0 / (d.dy * d.dy);
    d.blk0[PASS_D] = plan->nblk_d;
    d.nblk[PASS_D] = ((d.nx + kTileX) / kTileX) * ((d.ny + kTileY) / kTileY);
    plan->nblk_d += d.nblk[PASS_D];
  }
  // A block transforms at most two sequences and at most 2048 complex values.
  auto pairs = [](int L) { return L <= 512 ? 2 : 1; };
  // fused C + D pass (rows of at most kFusedMaxNx intervals, c <= 8; two
  // layers: c <= 4 and a compile-time transform length).  Its last block
  // owns exactly tj(c) coarse rows (fused_tj, or cgp_config.fused_rows at
  // c = 2, one layer), so the coarse row count must be a multiple of that
  // (only My = 6 at c = 1, one layer, and My = 6 at c = 2 with 4 rows, are
  // not).
  plan->rows2 = nl == 1 && cfgs[0].fused_rows == 4 ? 4 : 2;
  auto tj_of = [&](const MemberDesc& d) {
    return nl == 1 && d.c == 2 ? plan->rows2 : fused_tj(d.c, nl);
  };
  // multigrid (one layer, single basin): levels from the coarse CGP grid
  // down to the coarsest (an odd interval count or one below 8)
  plan->solver = cfgs[0].solver;
  if (plan->solver == 1) {
    if (count != 1 || nl != 1)
      return fail(CGP_ERR_UNSUPPORTED, "the multigrid solver takes one layer, single basin");
    const MemberDesc& d = plan->md[0];
    plan->mg_cycles = cfgs[0].mg_cycles > 0 ? cfgs[0].mg_cycles : 12;
    int gx = d.Mx, gy = d.My;
    double hx = d.dx * d.c, hy = d.dy * d.c;
    long long off = 0;
    for (;;) {
      MgLevel lv;
      lv.nx = gx; lv.ny = gy; lv.dx = hx; lv.dy = hy;
      lv.u = off; off += (long long)(gx + 1) * (gy + 1);
      lv.f = off; off += (long long)(gx + 1) * (gy + 1);
      plan->mg.push_back(lv);
      if (gx % 2 || gy % 2 || gx < 8 || gy < 8) break;
      gx /= 2; gy /= 2; hx *= 2; hy *= 2;
    }
    plan->mg_nb = (gx - 1) * (gy - 1);
    if (plan->mg_nb > 1024)
      return fail(CGP_ERR_UNSUPPORTED, "multigrid coarsest grid %dx%d too large", gx, gy);
    // the lowest levels whose u and f fit kMgTailLds run in one block
    const int nlv = (int)plan->mg.size();
    size_t tail_bytes = 0;
    plan->mg_tail = nlv;
    for (int k = nlv - 1; k >= 0 && nlv - k <= kMgTailLevels; --k) {
      tail_bytes += 2 * (size_t)(plan->mg[k].nx + 1) * (plan->mg[k].ny + 1) * es;
      if (tail_bytes > kMgTailLds) break;
      plan->mg_tail = k;
    }
  }
  bool fusable = plan->solver == 0;
  for (const MemberDesc& d : plan->md) {
    fusable = fusable && d.nx <= kFusedMaxNx && d.c <= (nl == 1 ? 8 : 4) &&
              d.My % tj_of(d) == 0;
    if (nl == 2) fusable = fusable && fft_special(d.Lr) != 0;
  }
  // one layer at c >= 4 with the fused pass: split restrictions (part p of
  // every member's spectra at p times the size of all members' spectra, in
  // the same region)
  int max_parts = 1;
  for (MemberDesc& d : plan->md) {
    d.split_off = (fusable && nl == 1 && d.c >= 4) ? wt : 0;
    d.nparts = d.split_off ? 2 * split_blocks(d.c) : 0;
    max_parts = std::max(max_parts, d.nparts);
  }
  // pass A: one complex sequence per block: coarse rows packed as the fused
  // pass packs them when it computes the next stage's spectra (so that both
  // give the same bits), else a pair of rows; two layers: one row's modes;
  // split members: split_blocks(c) blocks per coarse row j0 = 0 .. My-1
  build_groups(plan->md, PASS_A, [](const MemberDesc& d) { return fft_special(d.Lr); },
               [&](MemberDesc& d, HostGroup&) {
                 d.pa = 1;
                 d.a_rows = nl == 1 ? (fusable && fused_tj(d.c) == 1 ? 1 : 2) : 1;
                 d.a_first = (nl == 1 && fusable && (d.a_rows == 2 || d.split_off)) ? 0 : 1;
                 const int nrows = d.My - d.a_first;
                 const size_t lds = ((size_t)2 * lpad(d.Lr) + d.ntw_r) * cs;
                 const int shares = d.split_off ? d.nparts / 2 : 1;
                 return std::make_pair((nrows + d.a_rows - 1) / d.a_rows * shares, lds);
               },
               plan->groups[0]);
  // pass B: one complex sequence per block: a pair of spectral columns (one
  // layer) or one column's two modes
  build_groups(plan->md, PASS_B, [](const MemberDesc& d) { return fft_special(d.Lc); },
               [&](MemberDesc& d, HostGroup&) {
                 d.pb = 1;
                 const int cols = nl == 1 ? 2 : 1;
                 // two transform buffers; the twiddle table only for the
                 // runtime engine (compile-time lengths keep them in registers)
                 const size_t lds =
                     ((size_t)2 * lpad(d.Lc) + (fft_special(d.Lc) ? 0 : d.ntw_c)) * cs;
                 return std::make_pair((d.Mx - 1 + cols - 1) / cols, lds);
               },
               plan->groups[1]);
  // pass C: tj owned coarse rows (+1 halo row when c > 1) per block
  build_groups(plan->md, PASS_C, [](const MemberDesc& d) { return fft_special(d.Lr); },
               [&](MemberDesc& d, HostGroup&) {
                 const int halo = d.c > 1 ? 1 : 0;
                 d.pc = nl == 1 ? pairs(d.Lr) : (d.Lr <= 1024 ? 2 : 1);
                 d.tj = (nl == 1 ? 2 * d.pc : d.pc) - halo;
                 const size_t lds = ((size_t)2 * d.pc * lpad(d.Lr) + d.ntw_r) * cs +
                                    (halo ? (size_t)nl * (d.tj + 1) * (d.Mx + 1) * es : 0);
                 const int nb = halo ? (d.My + d.tj - 1) / d.tj : (d.My + 1 + d.tj - 1) / d.tj;
                 return std::make_pair(nb, lds);
               },
               plan->groups[2]);
  for (int p = 0; p < 3; ++p)
    for (const HostGroup& g : plan->groups[p])
      if (g.lds > kMaxLds)
        return fail(CGP_ERR_UNSUPPORTED, "a transform pass needs more than 160 KiB LDS per block");
  // fused C + D: a block owns fused_tj(c) coarse rows (one layer at c >= 4:
  // a share of one coarse row's fine rows, split_blocks(c) blocks per row)
  // and synthesises the two neighbouring ones (at most two packed
  // sequences); one launch per coarsening factor and transform length.
  if (fusable) {
    build_groups(plan->md, PASS_CD,
                 [](const MemberDesc& d) { return (d.c << 16) | fft_special(d.Lr); },
                 [&](MemberDesc& d, HostGroup&) {
                   // vorticity tile(s): own rows, c - 1 rows below them for
                   // the next stage's restriction, one more on each side
                   // (shares LDS with the transform buffers: two sequences
                   // per block for one layer, tj + 2 for two)
                   const int tj = tj_of(d);
                   const int nr = d.c <= 2 ? d.c * tj + 1 : fused_nr(d.c, nl);
                   const size_t tile = (size_t)nl * (nr + 2 + d.c - 1) * (d.nx + 1) * es;
                   const size_t psc = (size_t)nl * (tj + 2) * (d.Mx + 1) * es;
                   // rows of the restriction's column sums at c > 1: tj per
                   // layer (whole restrictions), or two (the a and b parts of
                   // a split one, one layer at c >= 4)
                   const int ysums = d.c == 1 ? 0 : nl == 2 ? 2 * tj : d.c >= 4 ? 2 : tj;
                   size_t lds;
                   if (nl == 2 && d.c == 1) {
                     // in-place row transform; psi rows and tiles in its region
                     const size_t fft = (size_t)(tj + 2) * lpad(d.Lr) * cs;
                     lds = ((std::max(fft, psc + tile) + 15) & ~(size_t)15) +
                           (size_t)d.ntw_r * cs;
                   } else {
                     const size_t fft =
                         (size_t)2 * (nl == 1 ? fused_nseq(tj) : tj + 2) * lpad(d.Lr) * cs;
                     const size_t region = (std::max(fft, tile) + 15) & ~(size_t)15;
                     lds = region + (size_t)d.ntw_r * cs + psc + (size_t)ysums * (d.nx + 1) * es;
                   }
                   const int shares = nl == 1 && d.c >= 4 ? split_blocks(d.c) : 1;
                   return std::make_pair((d.My + tj - 1) / tj * shares, lds);
                 },
                 plan->groups[3]);
    plan->fused = true;
    for (const HostGroup& g : plan->groups[3]) plan->fused = plan->fused && g.lds <= kMaxLds;
    if (!plan->fused) plan->groups[3].clear();
  }
  Layout& L = plan->lay;
  size_t off = 0;
  L.desc = off; off = align_up(off + sizeof(MemberDesc) * count);
  L.order = off; off = align_up(off + sizeof(int) * 4 * count);
  int o = 0;
  for (int p = 0; p < 4; ++p)
    for (HostGroup& g : plan->groups[p]) {
      g.order_off = o;
      o += (int)g.members.size();
    }
  L.tw = off; off = align_up(off + (size_t)tw * 2 * es);
  L.lam = off; off = align_up(off + (size_t)lam * sizeof(double));
  // step-size state: per member [dt, time, kVmaxSlots maxima per block of
  // the stage launch]
  long long ctl = 0;
  for (MemberDesc& d : plan->md) {
    d.npart = plan->fused ? d.nblk[PASS_CD] : d.nblk[PASS_D];
    d.cfl_off = ctl;
    ctl += 2 + (long long)d.npart * kVmaxSlots;
  }
  L.ctl = off; off = align_up(off + (size_t)ctl * sizeof(double));
  L.mgm = off; off = align_up(off + (size_t)plan->mg_nb * plan->mg_nb * sizeof(double));
  // persistent stage kernel: the tile queue (at most one tile per block of
  // passes B and CD) and its counters, zero at create
  plan->persist_ok = plan->fused && nl == 1 && plan->rows2 == 2;
  plan->persist_max_tiles = 0;
  for (const MemberDesc& d : plan->md) {
    plan->persist_ok = plan->persist_ok && persistent_lengths(d.c, d.Lr, d.Lc);
    plan->persist_max_tiles += d.nblk[PASS_B] + d.nblk[PASS_CD];
  }
  if (plan->persist_ok) {
    for (const MemberDesc& d : plan->md) {
      const size_t b_lds = (size_t)2 * lpad(d.Lc) * cs;  // compile-time column transform
      size_t f_lds = 0;
      for (const HostGroup& g : plan->groups[3])
        for (int m : g.members)
          if (&plan->md[m] == &d) f_lds = g.lds;
      plan->persist_lds = std::max(plan->persist_lds, std::max(b_lds, f_lds));
    }
  }
  L.ptile = off;
  off = align_up(off + (plan->persist_ok ? sizeof(PTile) * plan->persist_max_tiles : 0));
  L.pctr = off;
  off = align_up(off + (plan->persist_ok ? sizeof(int) * (kPersistCounters + count) : 0));
  L.wt = off; off = align_up(off + (size_t)wt * max_parts * es);
  L.wt2 = off; off = align_up(off + (size_t)wt * es);
  L.field_elems = fld;
  L.psi = off; off = align_up(off + (size_t)fld * es);
  L.st1 = off; off = align_up(off + (size_t)fld * es);
  L.st2 = off; off = align_up(off + (size_t)fld * es);
  L.diag = off; off = align_up(off + (size_t)kDiagBlocks * 2 * 3 * sizeof(double));
  L.fin = off; off = align_up(off + (size_t)(kFiniteBlocks + 1) * sizeof(int));
  long long mg_elems = 0;
  for (const MgLevel& lv : plan->mg) mg_elems += 2LL * (lv.nx + 1) * (lv.ny + 1);
  L.mg = off; off = align_up(off + (size_t)mg_elems * es);
  L.total = off;
  if (plan->fused && plan->groups[1].size() == plan->groups[3].size() &&
      plan->groups[3].size() > 1) {
    for (size_t i = 0; i < plan->groups[3].size(); ++i)
      for (size_t j = 0; j < plan->groups[1].size(); ++j)
        if (plan->groups[1][j].members == plan->groups[3][i].members)
          plan->chains.emplace_back((int)j, (int)i);
    if (plan->chains.size() != plan->groups[3].size()) plan->chains.clear();
  }
  return CGP_OK;
}

}  // namespace

struct cgp_handle {
  Plan plan;
  char* ws = nullptr;
  std::vector<char> host_tables;  // kept alive until destroy (async upload source)
  // graph cache: (omega, forcing, rotation phase of the fused step, running
  // sum of cgp_step_mean or NULL) -> executable graph of one step
  std::map<std::tuple<const void*, const void*, int, const void*>, hipGraphExec_t> graphs;
  // side streams and events of chained graph captures (made on first use)
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> events;
  // recorded on the caller's stream after the last graph replay a call
  // enqueued (made on first use); dropping the graphs waits for it
  hipEvent_t graph_done = nullptr;
  // persistent stage kernel: tiles in the queue and the launch grid
  int persist_ntiles = 0, persist_grid = 0;
  int ncu = 0;  // compute units of the handle's device
  int nm() const { return (int)plan.md.size(); }
  template <typename T> T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  const MemberDesc* d_md() const { return at<MemberDesc>(plan.lay.desc); }
  Group group(int pass, int i) const {
    const HostGroup& g = plan.groups[pass][i];
    const int count = g.members.size() == 1 ? -(g.members[0] + 1) : (int)g.members.size();
    int split = 0;
    for (int m : g.members) split = std::max(split, plan.md[m].nparts);
    return Group{g.L,     count,        at<int>(plan.lay.order) + g.order_off,
                 g.nblk,  kThreads,     g.lds,
                 plan.nlayers, split,   plan.rows2};
  }
  int ngroups(int pass) const { return (int)plan.groups[pass].size(); }
};

namespace {

const double kRkA[3] = {0.0, 0.75, 1.0 / 3.0};
const double kRkB[3] = {1.0, 0.25, 2.0 / 3.0};

// One pass of the coarse solve (0: A, 1: B, 2: C) over every member.
// ctl (pass B of a step's first stage): the step state, whose dt is set.
// only >= 0: that group of the pass alone.
// split (pass B): add the b spectra of split members (0 after the adjoint's
// fused stage, whose sources are whole restrictions).
template <typename T>
hipError_t enqueue_pass(cgp_handle* h, int pass, const T* src, T* dst, int accumulate,
                        hipStream_t s, double* ctl = nullptr, int only = -1, int split = 1) {
  const Plan& p = h->plan;
  const cplx<T>* tw = h->at<cplx<T>>(p.lay.tw);
  T* wt = h->at<T>(p.lay.wt);
  T* wt2 = h->at<T>(p.lay.wt2);
  for (int i = 0; i < h->ngroups(pass); ++i) {
    if (only >= 0 && i != only) continue;
    const Group g = h->group(pass, i);
    hipError_t e;
    if (pass == 0)
      e = Launch<T>::restrict_rowdst(h->d_md(), g, src, wt, tw, s);
    else if (pass == 1)
      e = Launch<T>::col_solve(h->d_md(), g, wt, wt2, tw, h->at<double>(p.lay.lam), ctl, split,
                               s);
    else
      e = Launch<T>::rowdst_prolong(h->d_md(), g, wt2, dst, accumulate, tw, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// One multigrid V(2,2) cycle from level k (the correction u_k of the
// right-hand side f_k; coarser levels' u zeroed before use).
template <typename T>
hipError_t mg_vcycle(cgp_handle* h, int k, hipStream_t s) {
  const Plan& p = h->plan;
  T* base = h->at<T>(p.lay.mg);
  const MgLevel& lv = p.mg[k];
  T* u = base + lv.u;
  T* f = base + lv.f;
  if (k == p.mg_tail) {  // this level and the coarser ones in one block
    MgTail<T> t;
    t.nlev = (int)p.mg.size() - k;
    int off = 0;
    for (int l = 0; l < t.nlev; ++l) {
      const MgLevel& m = p.mg[k + l];
      const double ax = 1.0 / (m.dx * m.dx), ay = 1.0 / (m.dy * m.dy);
      t.nx[l] = m.nx;
      t.ny[l] = m.ny;
      t.off[l] = off;
      t.ax[l] = T(ax);
      t.ay[l] = T(ay);
      t.inv_d[l] = T(1.0 / (2.0 * ax + 2.0 * ay));
      off += 2 * (m.nx + 1) * (m.ny + 1);
    }
    // below the top level the correction starts from zero
    return MgLaunch<T>::tail(t, u, f, k > 0 ? 1 : 0, h->at<double>(p.lay.mgm), p.mg_nb, s);
  }
  if (k + 1 == (int)p.mg.size())
    return MgLaunch<T>::bottom(h->at<double>(p.lay.mgm), p.mg_nb, f, lv.nx, u, s);
  hipError_t e = hipSuccess;
  for (int q = 0; q < 2 && e == hipSuccess; ++q) {  // pre-smoothing: red, black
    e = MgLaunch<T>::smooth(u, f, lv.nx, lv.ny, lv.dx, lv.dy, 0, s);
    if (e == hipSuccess) e = MgLaunch<T>::smooth(u, f, lv.nx, lv.ny, lv.dx, lv.dy, 1, s);
  }
  const MgLevel& cl = p.mg[k + 1];
  if (e == hipSuccess)
    e = MgLaunch<T>::residual_restrict(u, f, lv.nx, lv.ny, lv.dx, lv.dy, base + cl.f,
                                       base + cl.u, s);
  if (e == hipSuccess) e = mg_vcycle<T>(h, k + 1, s);
  if (e == hipSuccess) e = MgLaunch<T>::prolong_add(base + cl.u, lv.nx, lv.ny, u, s);
  for (int q = 0; q < 2 && e == hipSuccess; ++q) {  // post-smoothing: black, red
    e = MgLaunch<T>::smooth(u, f, lv.nx, lv.ny, lv.dx, lv.dy, 1, s);
    if (e == hipSuccess) e = MgLaunch<T>::smooth(u, f, lv.nx, lv.ny, lv.dx, lv.dy, 0, s);
  }
  return e;
}

// psi (+)= P^l A_c^-1 R^l omega with the multigrid coarse solve (single basin).
template <typename T>
hipError_t enqueue_solve_mg(cgp_handle* h, const T* src, T* dst, int accumulate, hipStream_t s,
                            double* ctl) {
  const Plan& p = h->plan;
  const MemberDesc& d = p.md[0];
  T* base = h->at<T>(p.lay.mg);
  const MgLevel& l0 = p.mg[0];
  hipError_t e = MgLaunch<T>::restrict_field(src + d.field_off, d.nx, d.ny, d.c, base + l0.f, s);
  if (e == hipSuccess)
    e = MgLaunch<T>::fill_zero(base + l0.u, (long long)(l0.nx + 1) * (l0.ny + 1), s);
  for (int cyc = 0; cyc < p.mg_cycles && e == hipSuccess; ++cyc) e = mg_vcycle<T>(h, 0, s);
  if (e == hipSuccess)
    e = MgLaunch<T>::prolong_field(base + l0.u, d.nx, d.ny, d.c, dst + d.field_off, accumulate,
                                   s);
  if (e == hipSuccess && ctl) e = step_ctl(h->d_md(), h->nm(), ctl, s);
  return e;
}

template <typename T>
hipError_t enqueue_solve(cgp_handle* h, const T* src, T* dst, int accumulate, hipStream_t s,
                         double* ctl = nullptr) {
  if (h->plan.solver == 1) return enqueue_solve_mg<T>(h, src, dst, accumulate, s, ctl);
  hipError_t e = enqueue_pass<T>(h, 0, src, nullptr, 0, s);
  if (e == hipSuccess) e = enqueue_pass<T>(h, 1, nullptr, nullptr, 0, s, ctl);
  if (e == hipSuccess) e = enqueue_pass<T>(h, 2, nullptr, dst, accumulate, s);
  return e;
}

// Fused pass C + D over every member: out = a wn + b (ws + dt G(ws, psi(ws)));
// with `next`, also pass A on out (its spectra into wt for the next stage);
// psi_out (optional) receives psi(ws).
template <typename T>
hipError_t enqueue_fused(cgp_handle* h, const T* ws, const T* forcing, const T* wn, T* out,
                         double a, double b, bool next, hipStream_t s, T* psi_out = nullptr,
                         StepCtl ctl = StepCtl{nullptr, 0}, int only = -1) {
  const Plan& p = h->plan;
  for (int i = 0; i < h->ngroups(3); ++i) {
    if (only >= 0 && i != only) continue;
    T* wnext = next ? h->at<T>(p.lay.wt) : nullptr;
    const Group g = h->group(3, i);
    // at most one block per CU: the new vorticity written through the L2
    const bool nt = g.nblk <= h->ncu;
    hipError_t e =
        p.nlayers == 1
            ? Launch<T>::prolong_stencil(h->d_md(), g, h->at<T>(p.lay.wt2), wnext,
                                         h->at<cplx<T>>(p.lay.tw), ws, forcing, wn, out, psi_out,
                                         a, b, ctl, nt, s)
            : Launch<T>::prolong_stencil2(h->d_md(), g, h->at<T>(p.lay.wt2), wnext,
                                          h->at<cplx<T>>(p.lay.tw), ws, forcing, wn, out, a, b,
                                          ctl, nt, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// One CGPRK3 step (unfused passes): w1 -> stage 1 buffer, w2 -> stage 2
// buffer, w_{n+1} -> omega.  psi0..psi2, when given, receive the stage stream
// functions.
template <typename T>
hipError_t enqueue_step(cgp_handle* h, T* omega, const T* forcing, hipStream_t s,
                        T* st1 = nullptr, T* st2 = nullptr, T* psi0 = nullptr,
                        T* psi1 = nullptr, T* psi2 = nullptr) {
  const Plan& p = h->plan;
  const bool tape = st1 != nullptr;  // the adjoint's recomputation: fixed dt
  T* b1 = st1 ? st1 : h->at<T>(p.lay.st1);
  T* b2 = st2 ? st2 : h->at<T>(p.lay.st2);
  T* pd = h->at<T>(p.lay.psi);
  T* psis[3] = {psi0 ? psi0 : pd, psi1 ? psi1 : pd, psi2 ? psi2 : pd};
  const T* src[3] = {omega, b1, b2};
  T* dst[3] = {b1, b2, omega};
  double* ctl = tape ? nullptr : h->at<double>(p.lay.ctl);
  for (int st = 0; st < 3; ++st) {
    hipError_t e = enqueue_solve<T>(h, src[st], psis[st], 0, s, st == 0 ? ctl : nullptr);
    if (e != hipSuccess) return e;
    e = Launch<T>::stencil_rk3(h->d_md(), h->nm(), p.nblk_d, src[st], psis[st], forcing,
                               omega, dst[st], kRkA[st], kRkB[st], StepCtl{ctl, st == 2}, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// One CGPRK3 step with the fused pass.  Each stage is pass B and the fused
// pass, which also leaves the spectra of its result for the next stage (the
// spectra of the state must be in place on entry).  The fused pass reads the
// vorticity of the stage input on rows of neighbouring blocks, so no stage
// may overwrite a field it reads: the state rotates through bufs[0..2]
// (omega and the two stage buffers) with period 3.  The state is in bufs[pos]
// on entry and in bufs[(pos+1) % 3] on exit.
template <typename T>
hipError_t enqueue_step_fused(cgp_handle* h, T* omega, const T* forcing, int pos,
                              hipStream_t s, int chain = -1) {
  const Plan& p = h->plan;
  T* bufs[3] = {omega, h->at<T>(p.lay.st1), h->at<T>(p.lay.st2)};
  T* S = bufs[pos];
  T* X = bufs[(pos + 1) % 3];
  T* Y = bufs[(pos + 2) % 3];
  const T* src[3] = {S, X, Y};
  T* dst[3] = {X, Y, X};
  double* ctl = h->at<double>(p.lay.ctl);
  const int gb = chain >= 0 ? p.chains[chain].first : -1;
  const int gf = chain >= 0 ? p.chains[chain].second : -1;
  for (int st = 0; st < 3; ++st) {
    hipError_t e = enqueue_pass<T>(h, 1, nullptr, nullptr, 0, s, st == 0 ? ctl : nullptr, gb);
    if (e == hipSuccess)
      e = enqueue_fused<T>(h, src[st], forcing, S, dst[st], kRkA[st], kRkB[st], true, s,
                           nullptr, StepCtl{ctl, st == 2}, gf);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// One CGPRK3 step as three launches of the persistent stage kernel, with the
// state rotation of enqueue_step_fused (the spectra of the state must be in
// place on entry).
template <typename T>
hipError_t enqueue_step_persistent(cgp_handle* h, T* omega, const T* forcing, int pos,
                                   hipStream_t s) {
  const Plan& p = h->plan;
  T* bufs[3] = {omega, h->at<T>(p.lay.st1), h->at<T>(p.lay.st2)};
  T* S = bufs[pos];
  T* X = bufs[(pos + 1) % 3];
  T* Y = bufs[(pos + 2) % 3];
  const T* src[3] = {S, X, Y};
  T* dst[3] = {X, Y, X};
  double* ctl = h->at<double>(p.lay.ctl);
  for (int st = 0; st < 3; ++st) {
    hipError_t e = PersistLaunch<T>::stage(
        h->d_md(), h->at<PTile>(p.lay.ptile), h->persist_ntiles, h->at<int>(p.lay.pctr), h->nm(),
        h->persist_grid, p.persist_lds, h->at<T>(p.lay.wt), h->at<T>(p.lay.wt2),
        h->at<cplx<T>>(p.lay.tw), h->at<double>(p.lay.lam), st == 0 ? ctl : nullptr, src[st],
        forcing, S, dst[st], kRkA[st], kRkB[st], StepCtl{ctl, st == 2}, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// A fused step in the handle's launch mode.
template <typename T>
hipError_t enqueue_step_mode(cgp_handle* h, T* omega, const T* forcing, int pos, hipStream_t s) {
  return h->plan.launch.mode == 1 ? enqueue_step_persistent<T>(h, omega, forcing, pos, s)
                                  : enqueue_step_fused<T>(h, omega, forcing, pos, s);
}

// One fused step into explicit buffers (the adjoint's tape): stage inputs
// w[0..2] (w[0] holds omega_n, and the spectra of w[0] must be in place),
// stream functions psi[0..2], result wnext (distinct from all of them).
template <typename T>
hipError_t enqueue_step_tape(cgp_handle* h, T* const w[3], T* const psi[3], T* wnext,
                             const T* forcing, hipStream_t s) {
  T* dst[3] = {w[1], w[2], wnext};
  for (int st = 0; st < 3; ++st) {
    hipError_t e = enqueue_pass<T>(h, 1, nullptr, nullptr, 0, s);
    if (e == hipSuccess)
      e = enqueue_fused<T>(h, w[st], forcing, w[0], dst[st], kRkA[st], kRkB[st], true, s,
                           psi[st]);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// reps back-to-back launches of pass p (3 = stencil, 4 = fused C + D, 5 =
// fused C + D + next pass A, in their stage-2 form)
template <typename T>
hipError_t enqueue_pass_reps(cgp_handle* h, int p, const T* omega, const T* forcing, int reps,
                             hipStream_t s) {
  const Plan& pl = h->plan;
  T* b1 = h->at<T>(pl.lay.st1);
  T* b2 = h->at<T>(pl.lay.st2);
  T* pd = h->at<T>(pl.lay.psi);
  for (int r = 0; r < reps; ++r) {
    hipError_t e;
    if (p < 3) e = enqueue_pass<T>(h, p, omega, pd, 0, s);
    else if (p == 3)
      e = Launch<T>::stencil_rk3(h->d_md(), h->nm(), pl.nblk_d, b1, pd, forcing, omega, b2,
                                 kRkA[1], kRkB[1], StepCtl{nullptr, 0}, s);
    else e = enqueue_fused<T>(h, b1, forcing, omega, b2, kRkA[1], kRkB[1], p == 5, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The work queue of the persistent stage kernel for launch setting l: every
// member's pass-B tiles (l.b_tile column pairs each), then every member's
// fused tiles (l.f_tile row blocks each), members in order.
std::vector<PTile> persist_tiles(const Plan& p, const cgp_launch& l) {
  std::vector<PTile> t;
  for (int kind = 0; kind < 2; ++kind)
    for (int m = 0; m < (int)p.md.size(); ++m) {
      const int n = p.md[m].nblk[kind == 0 ? PASS_B : PASS_CD];
      const int per = kind == 0 ? l.b_tile : l.f_tile;
      for (int lb = 0; lb < n; lb += per) t.push_back(PTile{m, kind, lb, std::min(per, n - lb)});
    }
  return t;
}

// Launch grid of the persistent kernel: wg_per_cu (or as many workgroups as
// can be resident) per compute unit, at most one per tile.
template <typename T>
cgp_status persist_grid(cgp_handle* h, int ntiles, int* grid) {
  int dev = 0, ncu = 0, per = h->plan.launch.wg_per_cu;
  HIP_TRY(hipGetDevice(&dev), "device");
  HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
  if (per <= 0) HIP_TRY(PersistLaunch<T>::blocks_per_cu(h->plan.persist_lds, &per), "occupancy");
  *grid = std::max(1, std::min(ntiles, std::max(1, per) * ncu));
  return CGP_OK;
}

// The dynamic-LDS cap is an attribute of the kernel function, shared by every
// handle of the process: it is raised once to the whole 160 KiB a workgroup
// may use (it only bounds what a launch may request), never lowered, so that
// a handle created later with smaller blocks cannot cap the launches of one
// created earlier.  Done once per scalar type, under the lock of a static.
template <typename T>
hipError_t allow_full_lds() {
  static const hipError_t once = [] {
    hipError_t e = Launch<T>::prepare(kMaxLds);
    if (e == hipSuccess) e = Launch<T>::prepare_fused(kMaxLds);
    if (e == hipSuccess) e = Launch<T>::prepare_fused2(kMaxLds);
    if (e == hipSuccess && sizeof(T) == 8) e = AdjLaunch::prepare_fused(kMaxLds);
    if (e == hipSuccess) e = PersistLaunch<T>::prepare(kMaxLds);
    return e;
  }();
  return once;
}

template <typename T>
cgp_status create_tables(cgp_handle* h, hipStream_t s) {
  const Plan& p = h->plan;
  const Layout& L = p.lay;
  // host image of [desc][order][tw][lam][step state]
  h->host_tables.assign(L.wt, 0);
  std::memcpy(h->host_tables.data() + L.desc, p.md.data(), sizeof(MemberDesc) * p.md.size());
  int* order = reinterpret_cast<int*>(h->host_tables.data() + L.order);
  for (int pass = 0; pass < 4; ++pass)
    for (const HostGroup& g : p.groups[pass])
      for (size_t i = 0; i < g.members.size(); ++i) order[g.order_off + i] = g.members[i];
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(h->host_tables.data() + L.tw);
  double* lam = reinterpret_cast<double*>(h->host_tables.data() + L.lam);
  const double pi = 3.14159265358979323846264338327950288;
  for (const MemberDesc& d : p.md) {
    for (int pass = 0; pass < 2; ++pass) {
      const int Ln = pass == 0 ? d.Lr : d.Lc;
      const int nst = pass == 0 ? d.nst_r : d.nst_c;
      const int* words = pass == 0 ? d.stw_r : d.stw_c;
      cplx<T>* t = tw + (pass == 0 ? d.twr_off : d.twc_off);
      for (int st = 0; st < nst; ++st) {
        const int R = words[st] & 15, ns = 1 << ((words[st] >> 4) & 31), off = words[st] >> 9;
        const int step = Ln / (ns * R);
        for (int r = 1; r < R; ++r)
          for (int k = 0; k < ns; ++k) {
            // w_L^m, m = r k L/(Ns R), reduced mod L for an exact argument
            const long long m = ((long long)r * k * step) % Ln;
            const double ang = 2.0 * pi * (double)m / (double)Ln;
            t[off + (r - 1) * ns + k].x = (T)std::cos(ang);
            t[off + (r - 1) * ns + k].y = (T)(-std::sin(ang));
          }
      }
    }
    // lambda_k = (2cos(pi k/M) - 2)/h^2 = -4 sin^2(pi k/(2M))/h^2 on the coarse grid
    const double hx = d.dx * d.c, hy = d.dy * d.c;
    double* lx = lam + d.lam_off;
    double* ly = lx + (d.Mx - 1);
    for (int k = 1; k < d.Mx; ++k) {
      const double sn = std::sin(pi * k / (2.0 * d.Mx));
      lx[k - 1] = -4.0 * sn * sn / (hx * hx);
    }
    for (int l = 1; l < d.My; ++l) {
      const double sn = std::sin(pi * l / (2.0 * d.My));
      ly[l - 1] = -4.0 * sn * sn / (hy * hy);
    }
  }
  // the persistent kernel's work queue (its counters stay 0)
  if (p.persist_ok) {
    const std::vector<PTile> t = persist_tiles(p, p.launch);
    std::memcpy(h->host_tables.data() + L.ptile, t.data(), t.size() * sizeof(PTile));
    h->persist_ntiles = (int)t.size();
    cgp_status st = persist_grid<T>(h, h->persist_ntiles, &h->persist_grid);
    if (st != CGP_OK) return st;
  }
  // step state: dt of the latest step = the configured dt, time 0, maxima 0
  double* ctl = reinterpret_cast<double*>(h->host_tables.data() + L.ctl);
  for (const MemberDesc& d : p.md) ctl[d.cfl_off] = d.dt;
  // multigrid: inverse of the coarsest grid's 5-point matrix (Gauss-Jordan
  // with partial pivoting, FP64; the matrix is symmetric negative definite)
  if (p.solver == 1) {
    const MgLevel& b = p.mg.back();
    const int n = p.mg_nb, n1 = b.nx - 1;
    const double ax = 1.0 / (b.dx * b.dx), ay = 1.0 / (b.dy * b.dy);
    std::vector<double> A((size_t)n * n, 0.0), X((size_t)n * n, 0.0);
    for (int k = 0; k < n; ++k) {
      const int i = k % n1, j = k / n1;
      A[(size_t)k * n + k] = -2.0 * ax - 2.0 * ay;
      if (i > 0) A[(size_t)k * n + k - 1] = ax;
      if (i < n1 - 1) A[(size_t)k * n + k + 1] = ax;
      if (j > 0) A[(size_t)k * n + k - n1] = ay;
      if (j < b.ny - 2) A[(size_t)k * n + k + n1] = ay;
      X[(size_t)k * n + k] = 1.0;
    }
    for (int col = 0; col < n; ++col) {
      int piv = col;
      for (int r = col + 1; r < n; ++r)
        if (std::fabs(A[(size_t)r * n + col]) > std::fabs(A[(size_t)piv * n + col])) piv = r;
      if (piv != col)
        for (int q = 0; q < n; ++q) {
          std::swap(A[(size_t)piv * n + q], A[(size_t)col * n + q]);
          std::swap(X[(size_t)piv * n + q], X[(size_t)col * n + q]);
        }
      const double inv = 1.0 / A[(size_t)col * n + col];
      for (int q = 0; q < n; ++q) {
        A[(size_t)col * n + q] *= inv;
        X[(size_t)col * n + q] *= inv;
      }
      for (int r = 0; r < n; ++r) {
        if (r == col) continue;
        const double fct = A[(size_t)r * n + col];
        if (fct == 0.0) continue;
        for (int q = 0; q < n; ++q) {
          A[(size_t)r * n + q] -= fct * A[(size_t)col * n + q];
          X[(size_t)r * n + q] -= fct * X[(size_t)col * n + q];
        }
      }
    }
    std::memcpy(h->host_tables.data() + L.mgm, X.data(), X.size() * sizeof(double));
  }
  HIP_TRY(allow_full_lds<T>(), "LDS attribute");
  HIP_TRY(hipMemcpyAsync(h->ws, h->host_tables.data(), L.wt, hipMemcpyHostToDevice, s),
          "table upload");
  // ring of the internal psi / stage buffers: produced fields always write
  // their ring, so no clearing is needed; the spectra are fully overwritten.
  return CGP_OK;
}

cgp_status check_handle(cgp_handle* h) {
  if (!h) return fail(CGP_ERR_INVALID, "handle is NULL");
  return CGP_OK;
}

cgp_status create_common(const cgp_config* cfgs, int count, void* ws, size_t bytes, void* stream,
                         cgp_handle** out) {
  if (!out) return fail(CGP_ERR_INVALID, "out is NULL");
  *out = nullptr;
  Plan plan;
  cgp_status st = make_plan(cfgs, count, &plan);
  if (st != CGP_OK) return st;
  if (!ws) return fail(CGP_ERR_INVALID, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % kAlign)
    return fail(CGP_ERR_INVALID, "workspace must be 256-byte aligned");
  if (bytes < plan.lay.total)
    return fail(CGP_ERR_INVALID, "workspace too small: %zu < %zu", bytes, plan.lay.total);
  int dev = 0, ncu = 0;
  hipError_t de = hipGetDevice(&dev);
  if (de == hipSuccess)
    de = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (de != hipSuccess) return hip_fail(de, "CU count");
  cgp_handle* h = new cgp_handle;
  h->plan = std::move(plan);
  h->ws = static_cast<char*>(ws);
  h->ncu = ncu;
  hipStream_t s = static_cast<hipStream_t>(stream);
  st = h->plan.dtype == CGP_F64 ? create_tables<double>(h, s) : create_tables<float>(h, s);
  if (st != CGP_OK) {
    delete h;
    return st;
  }
  // the host image must outlive the copy
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    delete h;
    return hip_fail(e, "table upload sync");
  }
  *out = h;
  return CGP_OK;
}

// sum += dt * (state after a step), over the handle's field layout.
template <typename T>
hipError_t enqueue_mean(cgp_handle* h, const T* state, double* sum, hipStream_t s) {
  return Launch<T>::accumulate(h->d_md(), h->nm(), state, h->plan.lay.field_elems, sum, 1.0,
                               h->at<double>(h->plan.lay.ctl), s);
}

// The state buffer of a fused step that started at rotation phase pos.
template <typename T>
T* fused_state_after(cgp_handle* h, T* w, int pos) {
  const int q = (pos + 1) % 3;
  return q == 0 ? w : h->at<T>(q == 1 ? h->plan.lay.st1 : h->plan.lay.st2);
}

// Graph of one step for (omega, forcing, pos, sum), captured on first use;
// pos = 3 (fused handles): the three steps of a full rotation, pos 0 -> 0;
// sum != NULL: each step followed by its time-weighted accumulation.
template <typename T>
cgp_status step_graph(cgp_handle* h, T* w, const T* F, int pos, double* sum, hipStream_t s,
                      hipGraphExec_t* out) {
  auto key = std::make_tuple(static_cast<const void*>(w), static_cast<const void*>(F), pos,
                             static_cast<const void*>(sum));
  auto it = h->graphs.find(key);
  if (it != h->graphs.end()) {
    *out = it->second;
    return CGP_OK;
  }
  const size_t nch = h->plan.chains.size();
  if (h->plan.fused && nch > 1 && !sum && h->plan.launch.mode == 0 && h->side.size() + 1 < nch) {
    // side streams (default priority) and fork / join events, made once
    while (h->side.size() + 1 < nch) {
      hipStream_t st = nullptr;
      HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "side stream");
      h->side.push_back(st);
    }
    while (h->events.size() < nch) {
      hipEvent_t ev = nullptr;
      HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event");
      h->events.push_back(ev);
    }
  }
  hipGraph_t g = nullptr;
  HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
  hipError_t e = hipSuccess;
  const int q0 = pos == 3 ? 0 : pos, q1 = pos == 3 ? 3 : pos + 1;
  if (!h->plan.fused) {
    e = enqueue_step<T>(h, w, F, s);
    if (e == hipSuccess && sum) e = enqueue_mean<T>(h, w, sum, s);
  } else if (nch > 1 && !sum && h->plan.launch.mode == 0) {
    // independent member chains forked onto side streams and joined back
    const int nc = (int)nch;
    hipEvent_t* ev = h->events.data();
    e = hipEventRecord(ev[0], s);
    for (int k = 0; k < nc && e == hipSuccess; ++k) {
      hipStream_t sk = k == 0 ? s : h->side[k - 1];
      if (k > 0) e = hipStreamWaitEvent(sk, ev[0], 0);
      for (int q = q0; q < q1 && e == hipSuccess; ++q) e = enqueue_step_fused<T>(h, w, F, q, sk, k);
      if (k > 0 && e == hipSuccess) e = hipEventRecord(ev[k], sk);
    }
    for (int k = 1; k < nc && e == hipSuccess; ++k) e = hipStreamWaitEvent(s, ev[k], 0);
  } else {
    for (int q = q0; q < q1 && e == hipSuccess; ++q) {
      e = enqueue_step_mode<T>(h, w, F, q, s);
      if (e == hipSuccess && sum) e = enqueue_mean<T>(h, fused_state_after<T>(h, w, q), sum, s);
    }
  }
  hipError_t e2 = hipStreamEndCapture(s, &g);
  if (e != hipSuccess) return hip_fail(e, "capture step");
  if (e2 != hipSuccess) return hip_fail(e2, "end capture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hip_fail(e, "graph instantiate");
  h->graphs[key] = exec;
  *out = exec;
  return CGP_OK;
}

template <typename T>
cgp_status step_impl(cgp_handle* h, void* omega, const void* forcing, void* psi_out, int nsteps,
                     int use_graph, hipStream_t s, double* sum = nullptr) {
  T* w = static_cast<T*>(omega);
  const T* F = static_cast<const T*>(forcing);
  const bool graph = use_graph && s != nullptr;
  bool replayed = false;
  if (!h->plan.fused) {
    for (int n = 0; n < nsteps; ++n) {
      if (graph) {
        hipGraphExec_t exec = nullptr;
        cgp_status st = step_graph<T>(h, w, F, 0, sum, s, &exec);
        if (st != CGP_OK) return st;
        HIP_TRY(hipGraphLaunch(exec, s), "graph launch");
        replayed = true;
      } else {
        HIP_TRY(enqueue_step<T>(h, w, F, s), "step launch");
        if (sum) HIP_TRY(enqueue_mean<T>(h, w, sum, s), "accumulate launch");
      }
    }
  } else if (nsteps > 0) {
    // spectra of omega, then steps rotating the state through omega and the
    // stage buffers; the result is copied back to omega unless it is there
    HIP_TRY(enqueue_pass<T>(h, 0, w, nullptr, 0, s), "pass A launch");
    int pos = 0;
    for (int n = 0; n < nsteps;) {
      if (graph) {
        // whole rotations as one graph, the rest step by step
        const int q = (pos == 0 && nsteps - n >= 3) ? 3 : pos;
        hipGraphExec_t exec = nullptr;
        cgp_status st = step_graph<T>(h, w, F, q, sum, s, &exec);
        if (st != CGP_OK) return st;
        HIP_TRY(hipGraphLaunch(exec, s), "graph launch");
        replayed = true;
        const int done = q == 3 ? 3 : 1;
        n += done;
        pos = (pos + done) % 3;
      } else {
        HIP_TRY(enqueue_step_mode<T>(h, w, F, pos, s), "step launch");
        if (sum) HIP_TRY(enqueue_mean<T>(h, fused_state_after<T>(h, w, pos), sum, s),
                         "accumulate launch");
        ++n;
        pos = (pos + 1) % 3;
      }
    }
    if (pos != 0) {
      const T* from = h->at<T>(pos == 1 ? h->plan.lay.st1 : h->plan.lay.st2);
      HIP_TRY(hipMemcpyAsync(w, from, (size_t)h->plan.lay.field_elems * sizeof(T),
                             hipMemcpyDeviceToDevice, s),
              "state copy");
    }
  }
  if (replayed) {
    if (!h->graph_done)
      HIP_TRY(hipEventCreateWithFlags(&h->graph_done, hipEventDisableTiming), "graph event");
    HIP_TRY(hipEventRecord(h->graph_done, s), "graph event record");
  }
  if (psi_out) HIP_TRY(enqueue_solve<T>(h, w, static_cast<T*>(psi_out), 0, s), "psi launch");
  return CGP_OK;
}

// Destroy the handle's graph executables once their last replay has finished
// (a caller may drop them right after enqueueing a replay on its stream).
void drop_graphs(cgp_handle* h) {
  if (!h->graphs.empty() && h->graph_done) (void)hipEventSynchronize(h->graph_done);
  for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
  h->graphs.clear();
}

// ---------------------------------------------------------------------------
// Static device scratch of cgp_step_noalloc: the workspace of one call, for
// callers that cannot allocate device memory.  Each GPU the library runs on
// holds its own copy of the array until the process ends.  In host code the
// array's name is only a host-side stand-in: its device address on the
// current device comes from hipGetSymbolAddress, taken once per device at the
// first call on that device and kept in g_scratch_ptr; only that pointer is
// handed to kernels and copies.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)48 << 20;  // the 512 x 1024 workloads, FP64, 1-2 layers

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // device address of `scratch`, per device id

cgp_status scratch_address(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "current device");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "address of the static scratch");
    if (!p || reinterpret_cast<uintptr_t>(p) % kAlign)
      return fail(CGP_ERR_DEVICE, "static scratch has no 256-byte aligned device address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CGP_OK;
}

template <typename T>
cgp_status step_noalloc_impl(const cgp_config* cfg, void* omega, const void* forcing,
                             void* psi_out, int nsteps, hipStream_t s) {
  cgp_handle h;
  cgp_status st = make_plan(cfg, 1, &h.plan);
  if (st != CGP_OK) return st;
  if (h.plan.lay.total > kScratchBytes)
    return fail(CGP_ERR_INVALID,
                "cgp_step_noalloc: this configuration needs %zu bytes of workspace, above the "
                "%zu bytes of the static scratch (use cgp_create with a caller workspace)",
                h.plan.lay.total, kScratchBytes);
  void* ws = nullptr;
  st = scratch_address(&ws);
  if (st != CGP_OK) return st;
  h.ws = static_cast<char*>(ws);
  // the tables and the step state of a fresh handle, every call (the array
  // keeps whatever the last call on this GPU left)
  st = create_tables<T>(&h, s);
  if (st != CGP_OK) return st;
  HIP_TRY(hipStreamSynchronize(s), "table upload sync");  // the host image dies with h
  // direct launches only: no graph, stream or event is created
  return step_impl<T>(&h, omega, forcing, psi_out, nsteps, 0, s);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* cgp_last_error(void) { return g_err.c_str(); }

const char* cgp_version(void) { return "cgp-mi355x 0.1 (gfx950)"; }

cgp_status cgp_workspace_size(const cgp_config* cfg, size_t* bytes) {
  return cgp_ensemble_workspace_size(cfg, 1, bytes);
}

cgp_status cgp_ensemble_workspace_size(const cgp_config* members, int32_t count, size_t* bytes) {
  if (!bytes) return fail(CGP_ERR_INVALID, "bytes is NULL");
  Plan plan;
  cgp_status st = make_plan(members, count, &plan);
  if (st != CGP_OK) return st;
  *bytes = plan.lay.total;
  return CGP_OK;
}

cgp_status cgp_ensemble_offsets(const cgp_config* members, int32_t count, int64_t* offsets,
                                int64_t* total) {
  Plan plan;
  cgp_status st = make_plan(members, count, &plan);
  if (st != CGP_OK) return st;
  if (offsets)
    for (int m = 0; m < count; ++m) offsets[m] = plan.md[m].field_off;
  if (total) *total = plan.lay.field_elems;
  return CGP_OK;
}

cgp_status cgp_create(const cgp_config* cfg, void* ws, size_t bytes, void* stream,
                      cgp_handle** out) {
  return create_common(cfg, 1, ws, bytes, stream, out);
}

cgp_status cgp_ensemble_create(const cgp_config* members, int32_t count, void* ws, size_t bytes,
                               void* stream, cgp_handle** out) {
  return create_common(members, count, ws, bytes, stream, out);
}

cgp_status cgp_destroy(cgp_handle* h) {
  if (!h) return CGP_OK;
  drop_graphs(h);
  if (h->graph_done) (void)hipEventDestroy(h->graph_done);
  for (hipStream_t st : h->side) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : h->events) (void)hipEventDestroy(ev);
  delete h;
  return CGP_OK;
}

cgp_status cgp_ensemble_step(cgp_handle* h, void* omega, const void* forcing, int32_t nsteps,
                             int32_t use_graph, void* stream) {
  if (check_handle(h) != CGP_OK) return CGP_ERR_INVALID;
  if (!omega || !forcing) return fail(CGP_ERR_INVALID, "omega or forcing is NULL");
  if (nsteps < 0) return fail(CGP_ERR_INVALID, "nsteps < 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return h->plan.dtype == CGP_F64
             ? step_impl<double>(h, omega, forcing, nullptr, nsteps, use_graph, s)
             : step_impl<float>(h, omega, forcing, nullptr, nsteps, use_graph, s);
}

cgp_status cgp_step(cgp_handle* h, void* omega, const void* forcing, void* psi_out,
                    int32_t nsteps, void* stream) {
  if (check_handle(h) != CGP_OK) return CGP_ERR_INVALID;
  if (h->nm() != 1) return fail(CGP_ERR_INVALID, "cgp_step needs a single-basin handle");
  if (!omega || !forcing) return fail(CGP_ERR_INVALID, "omega or forcing is NULL");
  if (nsteps < 0) return fail(CGP_ERR_INVALID, "nsteps < 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return h->plan.dtype == CGP_F64
             ? step_impl<double>(h, omega, forcing, psi_out, nsteps, 0, s)
             : step_impl<float>(h, omega, forcing, psi_out, nsteps, 0, s);
}

cgp_status cgp_step_noalloc(const cgp_config* cfg, void* omega, const void* forcing,
                            void* psi_out, int32_t nsteps, void* stream) {
  if (!cfg) return fail(CGP_ERR_INVALID, "config is NULL");
  if (!omega || !forcing) return fail(CGP_ERR_INVALID, "omega or forcing is NULL");
  if (nsteps < 0) return fail(CGP_ERR_INVALID, "nsteps < 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return cfg->dtype == CGP_F64
             ? step_noalloc_impl<double>(cfg, omega, forcing, psi_out, nsteps, s)
             : step_noalloc_impl<float>(cfg, omega, forcing, psi_out, nsteps, s);
}

cgp_status cgp_step_mean(cgp_handle* h, void* omega, const void* forcing, int32_t nsteps,
                         double* sum, int32_t use_graph, void* stream) {
  if (check_handle(h) != CGP_OK) return CGP_ERR_INVALID;
  if (!omega || !forcing || !sum) return fail(CGP_ERR_INVALID, "omega, forcing or sum is NULL");
  if (nsteps < 0) return fail(CGP_ERR_INVALID, "nsteps < 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return h->plan.dtype == CGP_F64
             ? step_impl<double>(h, omega, forcing, nullptr, nsteps, use_graph, s, sum)
             : step_impl<float>(h, omega, forcing, nullptr, nsteps, use_graph, s, sum);
}

cgp_status cgp_solve(cgp_handle* h, const void* omega, void* psi, void* stream) {
  if (check_handle(h) != CGP_OK) return CGP_ERR_INVALID;
  if (!omega || !psi) return fail(CGP_ERR_INVALID, "omega or psi is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = h->plan.dtype == CGP_F64
                     ? enqueue_solve<double>(h, static_cast<const double*>(omega),
                                             static_cast<double*>(psi), 0, s)
                     : enqueue_solve<float>(h, static_cast<const float*>(omega),
                                            static_cast<float*>(psi), 0, s);
  if (e != hipSuccess) return hip_fail(e, "solve launch");
  return CGP_OK;
}

cgp_status cgp_diagnostics(cgp_handle* h, const void* omega, const void* psi, double* out,
                           void* stream) {
  if (check_handle(h) != CGP_OK) return CGP_ERR_INVALID;
  if (h->nm() != 1) return fail(CGP_ERR_INVALID, "diagnostics need a single-basin handle");
  if (!omega || !psi || !out) return fail(CGP_ERR_INVALID, "NULL pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* part = h->at<double>(h->plan.lay.diag);
  // one node row per block where that fits in kDiagBlocks blocks
  const int nblk = std::min(kDiagBlocks, h->plan.md[0].ny + 1);
  hipError_t e = h->plan.dtype == CGP_F64
                     ? Launch<double>::diagnostics(h->d_md(), static_cast<const double*>(omega),
                                                   static_cast<const double*>(psi), part, nblk,
                                                   out, s)
                     : Launch<float>::diagnostics(h->d_md(), static_cast<const float*>(omega),
                                                  static_cast<const float*>(psi), part, nblk,
                                                  out, s);
  if (e != hipSuccess) return hip_fail(e, "diagnostics launch");
  return CGP_OK;
}

cgp_status cgp_check_finite(cgp_handle* h, const void* field, int64_t count, int32_t* flag,
                            void* stream) {
  if (check_handle(h) != CGP_OK) return CGP_ERR_INVALID;
  if (!field || !flag || count < 0) return fail(CGP_ERR_INVALID, "bad argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int* part = h->at<int>(h->plan.lay.fin);
  hipError_t e = h->plan.dtype == CGP_F64
                     ? Launch<double>::check_finite(static_cast<const double*>(field), count,
                                                    part, kFiniteBlocks, flag, s)
                     : Launch<float>::check_finite(static_cast<const float*>(field), count, part,
                                                   kFiniteBlocks, flag, s);
  if (e != hipSuccess) return hip_fail(e, "finite-check launch");
  return CGP_OK;
}

cgp_status cgp_assert_finite(cgp_handle* h, const void* field, int64_t count, void* stream) {
  if (check_handle(h) != CGP_OK) return CGP_ERR_INVALID;
  if (!field || count < 0) return fail(CGP_ERR_INVALID, "bad argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int* part = h->at<int>(h->plan.lay.fin);
  int* flag = part + kFiniteBlocks;  // the workspace's own flag word
  hipError_t e = h->plan.dtype == CGP_F64
                     ? Launch<double>::check_finite(static_cast<const double*>(field), count,
                                                    part, kFiniteBlocks, flag, s)
                     : Launch<float>::check_finite(static_cast<const float*>(field), count, part,
                                                   kFiniteBlocks, flag, s);
  if (e != hipSuccess) return hip_fail(e, "finite-check launch");
  int host = 0;
  HIP_TRY(hipMemcpyAsync(&host, flag, sizeof(int), hipMemcpyDeviceToHost, s), "flag read");
  HIP_TRY(hipStreamSynchronize(s), "flag sync");
  if (host) return fail(CGP_ERR_NONFINITE, "the field holds a NaN or an infinity");
  return CGP_OK;
}

cgp_status cgp_accumulate(cgp_handle* h, const void* field, double* sum, double weight,
                          int32_t times_dt, void* stream) {
  if (check_handle(h) != CGP_OK) return CGP_ERR_INVALID;
  if (!field || !sum) return fail(CGP_ERR_INVALID, "bad argument");
  if (!std::isfinite(weight)) return fail(CGP_ERR_INVALID, "non-finite weight");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const double* ctl = times_dt ? h->at<double>(h->plan.lay.ctl) : nullptr;
  const long long n = h->plan.lay.field_elems;
  hipError_t e = h->plan.dtype == CGP_F64
                     ? Launch<double>::accumulate(h->d_md(), h->nm(),
                                                  static_cast<const double*>(field), n, sum,
                                                  weight, ctl, s)
                     : Launch<float>::accumulate(h->d_md(), h->nm(),
                                                 static_cast<const float*>(field), n, sum, weight,
                                                 ctl, s);
  if (e != hipSuccess) return hip_fail(e, "accumulate launch");
  return CGP_OK;
}

cgp_status cgp_time_passes(cgp_handle* h, const void* omega, const void* forcing, int32_t reps,
                           double* ms, void* stream) {
  if (check_handle(h) != CGP_OK) return CGP_ERR_INVALID;
  if (!omega || !forcing || !ms || reps < 1) return fail(CGP_ERR_INVALID, "bad argument");
  if (h->plan.solver != 0)
    return fail(CGP_ERR_UNSUPPORTED, "pass timing needs the sine-transform solver");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(CGP_ERR_DEVICE, "event create");
  cgp_status st = CGP_OK;
  for (int p = 0; p < 6 && st == CGP_OK; ++p) {
    if (p >= 4 && !h->plan.fused) {
      ms[p] = 0.0;
      continue;
    }
    hipError_t e = hipEventRecord(e0, s);
    if (e == hipSuccess)
      e = h->plan.dtype == CGP_F64
              ? enqueue_pass_reps<double>(h, p, static_cast<const double*>(omega),
                                          static_cast<const double*>(forcing), reps, s)
              : enqueue_pass_reps<float>(h, p, static_cast<const float*>(omega),
                                         static_cast<const float*>(forcing), reps, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e != hipSuccess) st = hip_fail(e, "timed passes");
    else ms[p] = (double)t / reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

cgp_status cgp_set_launch(cgp_handle* h, const cgp_launch* l, void* stream) {
  if (check_handle(h) != CGP_OK) return CGP_ERR_INVALID;
  if (!l) return fail(CGP_ERR_INVALID, "launch is NULL");
  if (l->mode != 0 && l->mode != 1) return fail(CGP_ERR_INVALID, "mode must be 0 or 1");
  if (l->b_tile < 1 || l->f_tile < 1) return fail(CGP_ERR_INVALID, "tiles must be >= 1");
  if (l->wg_per_cu < 0 || l->wg_per_cu > 16) return fail(CGP_ERR_INVALID, "wg_per_cu in 0..16");
  Plan& p = h->plan;
  if (l->mode == 1 && !p.persist_ok)
    return fail(CGP_ERR_UNSUPPORTED,
                "the persistent stage kernel takes one layer at coarsening factor 2 with row "
                "transforms of 128-512 and column transforms of 256-1024 points");
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the graphs of the old launch go first: their last replay may still read
  // the work queue that the upload below rewrites
  drop_graphs(h);
  p.launch = *l;
  if (p.persist_ok) {
    // the queue of the new tiles (same counters: they are zero between launches)
    const std::vector<PTile> t = persist_tiles(p, p.launch);
    char* img = h->host_tables.data() + p.lay.ptile;
    std::memcpy(img, t.data(), t.size() * sizeof(PTile));
    h->persist_ntiles = (int)t.size();
    HIP_TRY(hipMemcpyAsync(h->ws + p.lay.ptile, img, t.size() * sizeof(PTile),
                           hipMemcpyHostToDevice, s),
            "tile upload");
    HIP_TRY(hipStreamSynchronize(s), "tile upload sync");
    const cgp_status st = p.dtype == CGP_F64
                              ? persist_grid<double>(h, h->persist_ntiles, &h->persist_grid)
                              : persist_grid<float>(h, h->persist_ntiles, &h->persist_grid);
    if (st != CGP_OK) return st;
  }
  return CGP_OK;
}

cgp_status cgp_get_launch(cgp_handle* h, cgp_launch* l, int32_t* available) {
  if (check_handle(h) != CGP_OK) return CGP_ERR_INVALID;
  if (!l) return fail(CGP_ERR_INVALID, "launch is NULL");
  *l = h->plan.launch;
  if (available) *available = h->plan.persist_ok ? 1 : 0;
  return CGP_OK;
}

cgp_status cgp_persistent_fault(cgp_handle* h, int32_t* flag, void* stream) {
  if (check_handle(h) != CGP_OK) return CGP_ERR_INVALID;
  if (!flag) return fail(CGP_ERR_INVALID, "flag is NULL");
  *flag = 0;
  if (!h->plan.persist_ok) return CGP_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipMemcpyAsync(flag, h->ws + h->plan.lay.pctr + 2 * sizeof(int), sizeof(int),
                         hipMemcpyDeviceToHost, s),
          "fault flag read");
  HIP_TRY(hipStreamSynchronize(s), "fault flag sync");
  return CGP_OK;
}

cgp_status cgp_time_step_passes(cgp_handle* h, void* omega, const void* forcing, int32_t nsteps,
                                double* ms, void* stream) {
  if (check_handle(h) != CGP_OK) return CGP_ERR_INVALID;
  if (!omega || !forcing || !ms || nsteps < 1 || nsteps > 4096)
    return fail(CGP_ERR_INVALID, "bad argument (nsteps in 1..4096)");
  if (!h->plan.fused)
    return fail(CGP_ERR_UNSUPPORTED, "in-step pass timing needs the fused stage pass");
  hipStream_t s = static_cast<hipStream_t>(stream);
  // events: one before and one after each of the 6 launches per step, plus
  // one at each end of the whole run
  const int nev = 12 * nsteps + 2;
  std::vector<hipEvent_t> ev(nev, nullptr);
  cgp_status st = CGP_OK;
  // timing-only events: no system-scope fence (cache writeback and
  // invalidation) when they are recorded, which would slow the launches
  // between them
  for (int i = 0; i < nev && st == CGP_OK; ++i)
    if (hipEventCreateWithFlags(&ev[i], hipEventDisableSystemFence) != hipSuccess)
      st = fail(CGP_ERR_DEVICE, "event create");
  hipError_t e = hipSuccess;
  if (st == CGP_OK) {
    auto run = [&](auto tag) -> hipError_t {
      using T = decltype(tag);
      T* w = static_cast<T*>(omega);
      const T* F = static_cast<const T*>(forcing);
      const Plan& p = h->plan;
      T* bufs[3] = {w, h->at<T>(p.lay.st1), h->at<T>(p.lay.st2)};
      double* ctl = h->at<double>(p.lay.ctl);
      hipError_t r = enqueue_pass<T>(h, 0, w, nullptr, 0, s);
      if (r == hipSuccess) r = hipEventRecord(ev[0], s);
      int k = 1;
      for (int n = 0; n < nsteps && r == hipSuccess; ++n) {
        // the launches of enqueue_step_fused at rotation phase n mod 3
        const int pos = n % 3;
        T* S = bufs[pos];
        T* X = bufs[(pos + 1) % 3];
        T* Y = bufs[(pos + 2) % 3];
        const T* src[3] = {S, X, Y};
        T* dst[3] = {X, Y, X};
        for (int stg = 0; stg < 3 && r == hipSuccess; ++stg) {
          r = hipEventRecord(ev[k++], s);
          if (r == hipSuccess)
            r = enqueue_pass<T>(h, 1, nullptr, nullptr, 0, s, stg == 0 ? ctl : nullptr);
          if (r == hipSuccess) r = hipEventRecord(ev[k++], s);
          if (r == hipSuccess) r = hipEventRecord(ev[k++], s);
          if (r == hipSuccess)
            r = enqueue_fused<T>(h, src[stg], F, S, dst[stg], kRkA[stg], kRkB[stg], true, s,
                                 nullptr, StepCtl{ctl, stg == 2});
          if (r == hipSuccess) r = hipEventRecord(ev[k++], s);
        }
      }
      if (r == hipSuccess) r = hipEventRecord(ev[k], s);
      if (r == hipSuccess && nsteps % 3 != 0)
        r = hipMemcpyAsync(w, bufs[nsteps % 3], (size_t)p.lay.field_elems * sizeof(T),
                           hipMemcpyDeviceToDevice, s);
      return r;
    };
    e = h->plan.dtype == CGP_F64 ? run(double{}) : run(float{});
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    double sum[2] = {0.0, 0.0};
    for (int n = 0; n < nsteps && e == hipSuccess; ++n)
      for (int stg = 0; stg < 3 && e == hipSuccess; ++stg)
        for (int q = 0; q < 2 && e == hipSuccess; ++q) {
          const int a = 1 + 12 * n + 4 * stg + 2 * q;
          float t = 0.f;
          e = hipEventElapsedTime(&t, ev[a], ev[a + 1]);
          sum[q] += t;
        }
    float tot = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&tot, ev[0], ev[nev - 1]);
    if (e != hipSuccess) {
      st = hip_fail(e, "in-step pass timing");
    } else {
      ms[0] = sum[0] / (3.0 * nsteps);
      ms[1] = sum[1] / (3.0 * nsteps);
      ms[2] = (double)tot / nsteps;
    }
  }
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  return st;
}

// ---------------------------------------------------------------------------
// Adjoint.  Tape layout (FP64 node arrays of the single member, N elements
// each): per step s of the segment the stage states w0 w1 w2 and psi0 psi1
// psi2 (6 arrays), then four work arrays X1 X2 P ACC.
// ---------------------------------------------------------------------------
cgp_status cgp_time_state(cgp_handle* h, double* out, void* stream) {
  if (check_handle(h) != CGP_OK) return CGP_ERR_INVALID;
  if (!out) return fail(CGP_ERR_INVALID, "out is NULL");
  HIP_TRY(time_state(h->d_md(), h->nm(), h->at<double>(h->plan.lay.ctl), out,
                     static_cast<hipStream_t>(stream)),
          "time state launch");
  return CGP_OK;
}

cgp_status cgp_tape_size(const cgp_config* cfg, int32_t nsteps, size_t* bytes) {
  cgp_status st = validate(cfg);
  if (st != CGP_OK) return st;
  if (!bytes || nsteps < 1) return fail(CGP_ERR_INVALID, "bad argument");
  if (cfg->cfl > 0)
    return fail(CGP_ERR_UNSUPPORTED, "the adjoint needs a fixed dt (cfl = 0)");
  if (cfg->solver != 0)
    return fail(CGP_ERR_UNSUPPORTED, "the adjoint needs the sine-transform solver");
  const size_t N = (size_t)(cfg->nx + 1) * (cfg->ny + 1);
  *bytes = (6 * (size_t)nsteps + 4) * N * sizeof(double);
  return CGP_OK;
}

cgp_status cgp_adjoint_step(cgp_handle* h, const void* omega_n, const void* forcing,
                            int32_t nsteps, void* lambda, void* grad_forcing, void* tape,
                            size_t tape_bytes, void* stream) {
  if (check_handle(h) != CGP_OK) return CGP_ERR_INVALID;
  if (h->nm() != 1 || h->plan.nlayers != 1 || h->plan.dtype != CGP_F64)
    return fail(CGP_ERR_UNSUPPORTED, "adjoint needs a one-layer FP64 single-basin handle");
  if (h->plan.md[0].cfl > 0)
    return fail(CGP_ERR_UNSUPPORTED, "the adjoint needs a fixed dt (cfl = 0)");
  if (h->plan.solver != 0)
    return fail(CGP_ERR_UNSUPPORTED, "the adjoint needs the sine-transform solver");
  if (!omega_n || !forcing || !lambda || !grad_forcing || !tape || nsteps < 1)
    return fail(CGP_ERR_INVALID, "bad argument");
  const MemberDesc& d = h->plan.md[0];
  const size_t N = (size_t)(d.nx + 1) * (d.ny + 1);
  const size_t need = (6 * (size_t)nsteps + 4) * N * sizeof(double);
  if (tape_bytes < need)
    return fail(CGP_ERR_INVALID, "tape too small: %zu < %zu", tape_bytes, need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* tp = static_cast<double*>(tape);
  auto slot = [&](int n, int k) { return tp + ((size_t)n * 6 + k) * N; };
  double* X1 = tp + (size_t)nsteps * 6 * N;
  double* X2 = X1 + N;
  double* P = X2 + N;
  double* ACC = P + N;
  const double* F = static_cast<const double*>(forcing);
  // forward recompute: step n reads w0(n) and leaves w_{n+1} in w0(n+1), or
  // in X1 for the last step (not needed afterwards).
  HIP_TRY(hipMemcpyAsync(slot(0, 0), omega_n, N * sizeof(double), hipMemcpyDeviceToDevice, s),
          "tape copy");
  if (h->plan.fused) {
    // the fused steps of the forward run, writing every stage into the tape
    HIP_TRY(enqueue_pass<double>(h, 0, slot(0, 0), nullptr, 0, s), "forward recompute");
    for (int n = 0; n < nsteps; ++n) {
      double* const w[3] = {slot(n, 0), slot(n, 1), slot(n, 2)};
      double* const ps[3] = {slot(n, 3), slot(n, 4), slot(n, 5)};
      HIP_TRY(enqueue_step_tape<double>(h, w, ps, (n + 1 < nsteps) ? slot(n + 1, 0) : X1, F, s),
              "forward recompute");
    }
  } else {
    for (int n = 0; n < nsteps; ++n) {
      double* next = (n + 1 < nsteps) ? slot(n + 1, 0) : X1;
      HIP_TRY(hipMemcpyAsync(next, slot(n, 0), N * sizeof(double), hipMemcpyDeviceToDevice, s),
              "tape copy");
      // enqueue_step updates its omega argument in place: run it on `next`
      // (holding w_n) so that w0(n) stays intact.
      HIP_TRY(enqueue_step<double>(h, next, F, s, slot(n, 1), slot(n, 2), slot(n, 3),
                                   slot(n, 4), slot(n, 5)),
              "forward recompute");
    }
  }
  // reverse sweep
  double* lam = static_cast<double*>(lambda);
  double* gF = static_cast<double*>(grad_forcing);
  const MemberDesc* md = h->d_md();
  const int nb = h->plan.nblk_d;
  if (h->plan.fused && d.c >= 2 && d.c <= 4) {
    // each stage: the fused adjoint kernel (which finishes the previous
    // stage's solve) and pass B on its source; pass C ends the sweep
    double* wt = h->at<double>(h->plan.lay.wt);
    double* wt2 = h->at<double>(h->plan.lay.wt2);
    const cplx<double>* tw = h->at<cplx<double>>(h->plan.lay.tw);
    bool prev = false;
    for (int n = nsteps - 1; n >= 0; --n) {
      const double* lin[3] = {X1, X2, lam};
      double* lout[3] = {lam, X1, X2};
      for (int st = 2; st >= 0; --st) {
        const int mode = st == 2 ? 0 : (st == 1 ? 1 : 2);
        for (int i = 0; i < h->ngroups(3); ++i)
          HIP_TRY(AdjLaunch::fused(md, h->group(3, i), prev ? wt2 : nullptr, wt, tw, lin[st],
                                   slot(n, st), slot(n, 3 + st), lout[st], ACC, gF, kRkA[st],
                                   kRkB[st], mode, s),
                  "adjoint stage");
        HIP_TRY(enqueue_pass<double>(h, 1, nullptr, nullptr, 0, s, nullptr, -1, 0),
                "adjoint solve");
        prev = true;
      }
    }
    HIP_TRY(enqueue_pass<double>(h, 2, nullptr, lam, 1, s), "adjoint solve");
    return CGP_OK;
  }
  for (int n = nsteps - 1; n >= 0; --n) {
    // stage 2: lam_3 = lam -> X2 ; stage 1: X2 -> X1 ; stage 0: X1 -> lam
    const double* lin[3] = {X1, X2, lam};
    double* lout[3] = {lam, X1, X2};
    for (int st = 2; st >= 0; --st) {
      const double* ws = slot(n, st);
      const double* ps = slot(n, 3 + st);
      const int mode = st == 2 ? 0 : (st == 1 ? 1 : 2);
      HIP_TRY(AdjLaunch::stencil(md, nb, lin[st], ws, ps, lout[st], P, ACC, gF, kRkA[st],
                                 kRkB[st], mode, s),
              "adjoint stencil");
      HIP_TRY(enqueue_solve<double>(h, P, lout[st], 1, s), "adjoint solve");
    }
  }
  return CGP_OK;
}

#ifdef CGP_PHASE_STAMPS
cgp_status cgp_phase_stamps(int32_t kind, uint64_t* host_out, int32_t nblocks,
                            int32_t* clock_khz) {
  if (kind != 0 && kind != 1) return fail(CGP_ERR_INVALID, "kind must be 0 or 1 (got %d)", kind);
  if (!host_out) return fail(CGP_ERR_INVALID, "host_out is NULL");
  if (nblocks < 1 || nblocks > kStampBlocks)
    return fail(CGP_ERR_INVALID, "nblocks must be in 1..%d (got %d)", kStampBlocks, nblocks);
  HIP_TRY(hipDeviceSynchronize(), "phase stamps sync");
  unsigned long long* out = reinterpret_cast<unsigned long long*>(host_out);
  HIP_TRY(kind == 0 ? stamps_copy_solve(out, nblocks) : stamps_copy_fused(out, nblocks),
          "phase stamps copy");
  if (clock_khz) {
    int dev = 0, khz = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev), "clock rate");
    *clock_khz = khz;
  }
  return CGP_OK;
}
#endif

}  // extern "C"
