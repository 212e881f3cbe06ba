// Host side of the C ABI declared in include/wect.h: metadata checks, work
// decomposition, workspace sizing, kernel dispatch, measurement hooks.
//
// Every hot-path entry point checks only host-side metadata, computes the
// decomposition from host-known totals and enqueues kernels; it never reads
// device memory, allocates or synchronises, so it can be captured.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "wect.h"
#include "wect_internal.h"

namespace {

using wect::Params;

constexpr int kW = wect::kWave;
constexpr size_t kLdsLimit = wect::kLdsBudget;

struct DeviceInfo {
  int cus = 0;
  bool ok = false;
};

std::mutex g_dev_mu;
std::vector<DeviceInfo> g_devs;

bool device_info(DeviceInfo* out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  std::lock_guard<std::mutex> lk(g_dev_mu);
  if ((int)g_devs.size() <= dev) g_devs.resize(dev + 1);
  DeviceInfo& di = g_devs[dev];
  if (!di.ok) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
    di.cus = prop.multiProcessorCount;
    di.ok = true;
  }
  *out = di;
  return true;
}

// launch shape (process-wide)
std::atomic<int> g_block{0};  // 0: chosen per request by auto_block()
std::atomic<int> g_bpc{0};  // 0: as many as LDS and wave slots allow
std::atomic<int> g_min_items{256};
std::atomic<int> g_decomp{0};  // wect_launch.decomposition
std::atomic<int> g_ttile{0};   // wect_launch.threshold_tile (0: automatic)
std::atomic<int> g_dpl{0};     // wect_launch.directions_per_lane (0: automatic)
std::atomic<int> g_rec{0};     // wect_launch.cubical_records (0: automatic, 1: off, 2: on, 3: on, two voxels per thread)
std::atomic<int> g_pack{0};    // wect_launch.cell_packing (0: automatic, 1: off)
std::atomic<int> g_stage{0};   // wect_launch.stage_entries (0: automatic)

// measurement
std::atomic<int> g_profile{0};
struct EvPair {
  hipEvent_t a, b;
  int bwd;
};
std::mutex g_prof_mu;
std::vector<EvPair> g_prof;

bool valid_block(int b) { return b == 256 || b == 512 || b == 1024; }

// Everything the host derives for one request.
struct Plan {
  Params p;
  // Thresholds are processed in tiles of consecutive entries, one launch per
  // tile: out[b][p][q] depends on thr[q] alone (the cells whose value is at
  // most thr[q]), so a launch given thr[q0 .. q0+t) computes exactly the
  // columns q0 .. q0+t of the output; the adjoint is a sum over the
  // thresholds, so its tiles add up.  One tile whenever the LDS histogram of
  // all T thresholds fits.
  int T_full = 0;
  const float* thr = nullptr;
  int tt_fwd = 0, tt_bwd = 0;  // threshold tile of the forward / adjoint launches
  int stage_fwd = 0, stage_bwd = 0;
  int block = 1024;
  size_t lds_fwd = 0, lds_bwd = 0;
  size_t partial_bytes = 0, dsum_bytes = 0, absmax_bytes = 0;
  size_t vb_bytes = 0;        // general-filter WECF: threshold indices of the filter values
  size_t rec_bytes = 0;       // cubical: per-voxel records of combined weights
  bool two_vox = false;       // cubical with records: two voxels per thread and tile
  bool split = false;
  bool group_mode = false;
  size_t ws_fwd = 0, ws_bwd = 0;
  int64_t elems = 0;  // stream elements per direction tile / group
  int G_fwd = 0, G_bwd = 0;
  int64_t S_fwd = 0, S_bwd = 0;
  int dg = 0, ngd = 0;
  int sm_block = 0, sm_stage = 0;  // adjoint of the sigmoid relaxation
};

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Staged entries per tile and LDS bytes of the forward kernel for a block
// size: the histogram and thresholds are fixed, the staging tile takes what is
// left (at most one entry per thread, a multiple of 64).  stage = 0: no fit.
// Accumulator width of the forward: float32 weights and the sigmoid relaxation
// accumulate in 64-bit fixed point, integer weights in 32 bits.
int acc_bytes_of(const wect_complex* c, bool smooth) {
  return (smooth || (c->kind == WECT_SIMPLICIAL && c->dtype == WECT_F32)) ? 8 : 4;
}

void fwd_stage_lds(const wect_complex* c, const wect_grid* g, int block, int* stage, size_t* lds,
                   bool smooth = false, int dpl = 1) {
  const int acc_bytes = acc_bytes_of(c, smooth);
  const size_t fixed = wect::forward_lds_fixed(g->T, c->kind, acc_bytes, dpl);
  const size_t entry = wect::forward_entry_bytes(c->kind, c->n);
  int st = fixed + 64 * entry > kLdsLimit ? 0 : (int)std::min<size_t>(block, (kLdsLimit - fixed) / entry) / 64 * 64;
  if (const int cap = g_stage.load(); cap > 0) {
    st = std::min(st, cap);
  } else if (c->kind == WECT_SIMPLICIAL && !smooth && block == 1024 && st == 1024) {
    // measured on MI355X (2D batches of 10^4 - 2 10^5 vertices, every weight
    // mode): 768 staged cells per 1024-thread block run 6 - 7 % faster than
    // 1024, with the same resident blocks
    st = 768;
  }
  *stage = st;
  *lds = fixed + (size_t)st * entry;
}

// Default block size.  Measured on MI355X: 512-thread blocks are fastest when
// they reach 16 or more resident wavefronts per CU (several independent blocks
// overlap their staging and histogram phases); otherwise the size with the
// most resident wavefronts (32 wave slots and 160 KiB of LDS per CU) wins.
int auto_block(const wect_complex* c, const wect_grid* g, bool bwd_only, bool smooth, int dpl) {
  if (bwd_only || g->T <= 0) return 1024;
  auto waves_of = [&](int b) {
    int stage = 0;
    size_t lds = 0;
    fwd_stage_lds(c, g, b, &stage, &lds, smooth, dpl);
    if (stage == 0) return 0;
    const int by_lds = (int)((160 * 1024) / (lds + 1024));
    return std::min(32 / (b / kW), by_lds) * (b / kW);
  };
  if (waves_of(512) >= 16) return 512;
  int best = 1024, best_waves = -1;
  for (int b : {1024, 512, 256}) {
    const int w = waves_of(b);
    if (w > best_waves) {
      best_waves = w;
      best = b;
    }
  }
  return best;
}

// Largest block whose vertex-centric relaxation kernel fits in LDS (the
// coface rows grow with the block); 0 when none does.
int ls_block(int T, bool bwd) {
  for (int b : {1024, 512, 256}) {
    const size_t lds = bwd ? wect::smooth_ls_backward_lds_bytes(T, b) : wect::smooth_ls_forward_lds_bytes(T, b);
    if (lds <= kLdsLimit) return b;
  }
  return 0;
}

// Largest t in [1, T] for which fits(t) holds (fits is monotone: true up to
// some length, false beyond); 0 when not even t = 1 fits.
template <typename F>
int largest_fit(int T, F fits) {
  if (T <= 0) return 0;
  if (fits(T)) return T;
  if (!fits(1)) return 0;
  int lo = 1, hi = T;
  while (hi - lo > 1) {
    const int mid = lo + (hi - lo) / 2;
    if (fits(mid)) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Threshold tile for T thresholds when at most tmax fit in one launch: the
// fewest tiles, of balanced length (a multiple of 4 when that still fits, so
// that output rows keep their vector stores).
int balanced_tile(int T, int tmax) {
  if (tmax <= 0 || T <= 0) return 0;
  if (T <= tmax) return T;
  const int nt = (int)ceil_div(T, tmax);
  const int t = (int)ceil_div(T, nt);
  const int t4 = (t + 3) & ~3;
  return t4 <= tmax ? t4 : t;
}

// Threshold tile of a launch family: with a user tile, at most that and at
// most what fits at all (fits_min); automatically, all T thresholds when they
// fit at all, else the largest tile that fits with a comfortable staging area
// (fits_good), balanced.
template <typename FMin, typename FGood>
int choose_tile(int T, FMin fits_min, FGood fits_good) {
  const int user = g_ttile.load();
  int tmax;
  if (user > 0) tmax = std::min(user, largest_fit(T, fits_min));
  else tmax = fits_min(T) ? T : largest_fit(T, fits_good);
  return balanced_tile(T, tmax);
}

// Check host metadata and build the plan.  need_bwd: backward requested.
// smooth: forward of the sigmoid relaxation (fixed-point accumulation for
// every weight mode, float32 output); its adjoint is planned by smooth_plan.
wect_status make_plan(const wect_complex* c, const wect_grid* g, bool need_fwd, bool need_bwd, Plan* pl,
                      bool smooth = false, bool ls = false, bool lean = false) {
  if (!c || !g) return WECT_ERR_ARG;
  if (c->kind != WECT_SIMPLICIAL && c->kind != WECT_CUBICAL) return WECT_ERR_ARG;
  if (c->B < 1) return WECT_ERR_ARG;
  if (c->wmode < WECT_W_ONES || c->wmode > WECT_W_VERTEX_MAX) return WECT_ERR_ARG;
  if (c->dtype != WECT_I32 && c->dtype != WECT_F32) return WECT_ERR_ARG;
  if (g->d < 0 || g->T < 0) return WECT_ERR_ARG;
  if (g->d > 0 && !g->dirs) return WECT_ERR_ARG;
  if (g->T > 0 && !g->thr) return WECT_ERR_ARG;
  Params& p = pl->p;
  std::memset(&p, 0, sizeof(p));
  p.kind = c->kind;
  p.n = c->n;
  p.B = c->B;
  p.wmode = c->wmode;
  p.dtype = c->dtype;
  p.dirs = g->dirs;
  p.d = g->d;
  p.T = g->T;
  p.thr = g->thr;
  int64_t elems = 0;
  if (c->kind == WECT_SIMPLICIAL) {
    if (c->n < 1 || c->n > 3) return WECT_ERR_ARG;
    if (c->top_dim < 0 || c->top_dim > 3) return WECT_ERR_ARG;
    if (c->wmode == WECT_W_ONES && c->dtype != WECT_I32) return WECT_ERR_ARG;
    if (c->wmode == WECT_W_VERTEX_MAX && c->dtype != WECT_F32) return WECT_ERR_ARG;
    for (int i = 0; i < 4; ++i) {
      if (c->count[i] < 0) return WECT_ERR_ARG;
      if (i > c->top_dim && c->count[i] != 0) return WECT_ERR_ARG;
      elems += c->count[i];
    }
    if (c->count[0] > 0 && !c->coords) return WECT_ERR_ARG;
    if (c->count[0] > INT32_MAX || c->count[0] * (int64_t)c->n > INT64_MAX / 4) return WECT_ERR_ARG;
    for (int i = 1; i <= c->top_dim; ++i)
      if (c->count[i] > 0 && !c->simplices[i]) return WECT_ERR_ARG;
    if (c->B > 1) {
      if (!c->vert_off) return WECT_ERR_ARG;
      for (int i = 1; i <= c->top_dim; ++i)
        if (!c->simp_off[i]) return WECT_ERR_ARG;
    }
    // a batch given with offsets for B == 1 must give all of them
    if (c->B == 1 && c->vert_off) {
      for (int i = 1; i <= c->top_dim; ++i)
        if (!c->simp_off[i]) return WECT_ERR_ARG;
    }
    if (c->wmode == WECT_W_EXPLICIT) {
      for (int i = 0; i <= c->top_dim; ++i)
        if (c->count[i] > 0 && !c->weights[i]) return WECT_ERR_ARG;
    }
    if (c->wmode == WECT_W_VERTEX_MAX && c->count[0] > 0 && !c->weights[0]) return WECT_ERR_ARG;
    p.top_dim = c->top_dim;
    p.coords = c->coords;
    p.vert_off = c->vert_off;
    for (int i = 0; i < 4; ++i) {
      p.count[i] = c->count[i];
      p.simp[i] = i >= 1 ? c->simplices[i] : nullptr;
      p.simp_off[i] = (i >= 1 && i <= c->top_dim) ? c->simp_off[i] : nullptr;
      p.weights[i] = c->weights[i];
    }
    if (c->B == 1 && !c->vert_off) {
      for (int i = 0; i < 4; ++i) p.simp_off[i] = nullptr;
    }
  } else {
    if (c->n != 2 && c->n != 3) return WECT_ERR_ARG;
    if (c->wmode == WECT_W_EXPLICIT) return WECT_ERR_UNSUPPORTED;
    if (c->dtype != WECT_I32) return WECT_ERR_ARG;
    if (c->total_voxels < 0) return WECT_ERR_ARG;
    if (!c->shape || !c->axis) return WECT_ERR_ARG;
    if (c->total_voxels > 0 && !c->intensity) return WECT_ERR_ARG;
    if (c->B > 1 && (!c->grid_off || !c->axis_off)) return WECT_ERR_ARG;
    if (c->include_above < -1 || c->include_above > 255) return WECT_ERR_ARG;
    p.shape = c->shape;
    p.grid_off = c->grid_off;
    p.intensity = c->intensity;
    p.axis = c->axis;
    p.axis_off = c->axis_off;
    p.total_voxels = c->total_voxels;
    p.include_above = c->include_above;
    elems = c->total_voxels;
  }
  const int64_t cells = elems;
  if (ls) elems = c->count[0];  // vertex-centric kernels: one stream element per vertex
  if (need_bwd) {
    if (c->kind != WECT_SIMPLICIAL) return WECT_ERR_UNSUPPORTED;
    if (c->dtype != WECT_F32 || c->wmode == WECT_W_ONES) return WECT_ERR_ARG;
  }

  // directions per lane of the forward: two (a tile of 128 directions, so
  // that every staged voxel serves two directions per lane) for cubical
  // complexes with more than one 64-direction tile, when two histogram
  // columns per lane fit LDS with 256 staged voxels; else one
  int dpl = 1;
  if (need_fwd && c->kind == WECT_CUBICAL && !smooth && !ls && g->T > 0) {
    const int user = g_dpl.load();
    const bool fits2 = wect::forward_lds_fixed(g->T, c->kind, 4, 2) +
                           256 * wect::forward_entry_bytes(c->kind, c->n) <= kLdsLimit;
    dpl = (user == 2 || (user == 0 && g->d > kW)) && fits2 ? 2 : 1;
  }
  p.dpl = dpl;
  // simplicial forward with at most 32 directions (or filter columns): 64 / dt
  // cells per wavefront instruction instead of lanes past d idling
  p.cpw = 1;
  p.dt = kW;
  if (need_fwd && c->kind == WECT_SIMPLICIAL && !smooth && !ls && g->d > 0 && g->d <= kW / 2 &&
      g_pack.load() != 1) {
    int dt = 1;
    while (dt < g->d) dt *= 2;
    p.dt = dt;
    p.cpw = kW / dt;
  }
  const int ntiles = (int)ceil_div(g->d, kW * dpl);
  DeviceInfo di;
  const bool have_dev = device_info(&di);
  const int cus = have_dev ? di.cus : 256;
  pl->T_full = g->T;
  pl->thr = g->thr;
  p.ldo = g->T;
  // forward threshold tile: all thresholds whenever their histogram fits LDS
  // with at least one wavefront's staging, else the fewest tiles that leave a
  // staging area of 256 entries (relaxation over the lower-star index: the
  // smallest block's coface rows)
  int tt_fwd = g->T;
  if (need_fwd && g->d > 0 && g->T > 0) {
    const int acc_bytes = acc_bytes_of(c, smooth);
    const size_t entry = wect::forward_entry_bytes(c->kind, c->n);
    auto fits_stage = [&](int t, size_t nst) {
      return ls ? wect::smooth_ls_forward_lds_bytes(t, 256) <= kLdsLimit
                : wect::forward_lds_fixed(t, c->kind, acc_bytes, dpl) + nst * entry <= kLdsLimit;
    };
    // one tile when all T thresholds fit next to a wavefront's staging area;
    // else the fewest balanced tiles that leave 448 staged cells (measured on
    // MI355X: with several passes anyway, one more pass for a larger staging
    // tile pays, e.g. 256 images of 128^2 at T = 4096: 8 tiles 0.89 ms
    // against 7 tiles 1.06 ms)
    tt_fwd = choose_tile(g->T, [&](int t) { return fits_stage(t, 64); }, [&](int t) { return fits_stage(t, 448); });
    if (tt_fwd == 0) return WECT_ERR_UNSUPPORTED;
  }
  wect_grid gt = *g;  // the grid of one forward launch: its threshold tile
  gt.T = tt_fwd;
  pl->tt_fwd = tt_fwd;
  // Automatic one block per group (complex, direction tile) when there is at
  // least one group per compute unit: every block finishes its own groups, so
  // there are no partial histograms and no reduction kernel.  Cubical groups
  // take 1024-thread blocks for 2048 voxels or more on average, else 512;
  // simplicial groups the block that auto_block picks (occupancy by LDS).
  // Measured on MI355X (64 directions, T = 128): 256 images of 128^2 102 us
  // (1024-thread groups) against 118-145 us split over blocks; 256 images of
  // 2^2 ... 64^2, 1024 of 28^2 and 4096 of 8^2 take 15 / 16 / 17 / 22 / 37 /
  // 45 / 101 us in groups against 332 / 35 / 21 / 41 / 54 / 74 / 179 us when a
  // few blocks share many small groups.
  const int64_t groups_fwd = (int64_t)c->B * ntiles;
  const int64_t S_fwd = (int64_t)ntiles * elems;
  const int decomp = g_decomp.load();
  const bool auto_group = need_fwd && decomp == 0 && g->T > 0 && S_fwd > 0 && groups_fwd >= cus;
  const int group_block = c->kind == WECT_CUBICAL ? (S_fwd >= groups_fwd * 2048 ? 1024 : 512) : 0;
  int block = g_block.load();
  if (ls) {
    // the coface rows of the vertex-centric kernels grow with the block:
    // at most the largest block that fits, also for a block set by the caller
    const int fit = ls_block(tt_fwd, false);
    block = block ? std::min(block, fit) : fit;
    if (block == 0) block = 256;
  } else if (!block) {
    block = auto_group && group_block ? group_block : auto_block(c, &gt, need_bwd && !need_fwd, smooth, dpl);
  }
  pl->block = block;
  pl->elems = elems;
  p.ntiles = ntiles;
  p.stage = block;
  p.T = tt_fwd;
  const int64_t min_items = std::max(1, g_min_items.load());
  // blocks resident per compute unit: 32 wavefronts and 160 KiB of LDS per CU
  auto blocks_per_cu = [&](size_t lds) -> int64_t {
    const int user = g_bpc.load();
    if (user > 0) return user;
    int64_t by_waves = 32 / (block / kW);
    int64_t by_lds = lds > 0 ? (int64_t)((160 * 1024) / (lds + 1024)) : by_waves;
    return std::max<int64_t>(1, std::min(by_waves, by_lds));
  };

  if (need_fwd && g->d > 0 && g->T > 0) {
    // forward LDS: histogram [T+1][64] + threshold pairs + staged entries
    const int acc_bytes = acc_bytes_of(c, smooth);
    int stage = 0;
    size_t lds = 0;
    if (ls) {  // per-wavefront coface rows instead of a block staging tile
      stage = block;
      lds = wect::smooth_ls_forward_lds_bytes(tt_fwd, block);
      if (lds > kLdsLimit) stage = 0;
    } else {
      fwd_stage_lds(c, &gt, block, &stage, &lds, smooth, dpl);
    }
    if (stage == 0) return WECT_ERR_UNSUPPORTED;
    pl->stage_fwd = stage;
    p.stage = stage;
    pl->lds_fwd = lds;
    const int64_t S = S_fwd;
    const int64_t max_blocks = (int64_t)cus * blocks_per_cu(pl->lds_fwd);
    int64_t G = std::min<int64_t>(max_blocks, std::max<int64_t>(1, ceil_div(S, min_items)));
    G = std::min<int64_t>(G, std::max<int64_t>(S, 1));
    const int64_t groups = groups_fwd;
    const bool fits = S > 0 && groups * block < ((int64_t)1 << 32);  // grid limit: 2^32 threads
    pl->group_mode = fits && (decomp == 2 || auto_group);
    if (pl->group_mode) G = groups;
    pl->G_fwd = (int)G;
    pl->S_fwd = S;
    p.group_mode = pl->group_mode ? 1 : 0;
    const int64_t slots = pl->group_mode ? 0 : G + groups;
    const size_t slot_bytes = (size_t)tt_fwd * kW * dpl * acc_bytes;
    // Slots a group may have (blocks meeting its stream range).  A batch's
    // per-complex sizes are on the device: the kernels decide per group, and
    // the separate slot summation is launched when the average group has many
    // slots.  Either way every group is summed correctly.
    const int64_t spg = c->B == 1 ? ceil_div(G, ntiles) + 1 : ceil_div(G, groups) + 1;
    pl->split = !pl->group_mode && spg > 16;  // kFusedSlots in the kernels
    pl->partial_bytes = align256((size_t)slots * slot_bytes);
    pl->dsum_bytes = pl->split ? align256((size_t)groups * slot_bytes) : 0;
    const bool absmax = acc_bytes == 8 && c->wmode != WECT_W_ONES;  // unit weights: M = 1
    pl->absmax_bytes = absmax ? align256(wect::kAbsmaxSlots * sizeof(float)) : 0;
    // Cubical: when every voxel would be staged more than once (several
    // direction or threshold tiles), its combined weights are formed once per
    // call into per-voxel records (8 or 16 bytes per voxel of workspace) and
    // the forward stages records instead of neighbourhoods.  Not in lean plans
    // (the workspace then stays at the partial histograms).
    const int64_t reuse = (int64_t)ntiles * ceil_div(g->T, tt_fwd);
    const int rec_knob = g_rec.load();
    if (c->kind == WECT_CUBICAL && !lean && rec_knob != 1 && (reuse >= 2 || rec_knob >= 2))
      pl->rec_bytes = align256((size_t)c->total_voxels * (c->n == 3 ? 16 : 8));
    // With records, a tile of 1.5 stages of voxels (two per thread, the
    // contributing ones past the stage in a second round) means fewer tiles
    // and block barriers per voxel; automatic for volumes whose blocks walk
    // many tiles (measured on MI355X: 16 volumes 64^3 - 192^3 at d = 512, 3.31
    // -> 3.27 ms; 3 volumes of sides 9 - 40, 34 -> 36 us, hence the bound; 256
    // images 128^2 at T = 1000, 0.23 -> 0.25 ms, hence volumes only)
    if (pl->rec_bytes)
      pl->two_vox = rec_knob == 3 || (rec_knob == 0 && c->n == 3 &&
                                       pl->S_fwd >= 16 * (int64_t)pl->stage_fwd * std::max(1, pl->G_fwd));
    pl->ws_fwd = pl->partial_bytes + pl->dsum_bytes + pl->absmax_bytes + pl->rec_bytes;
    p.nabsmax = absmax ? wect::kAbsmaxSlots : 0;
    p.cells_total = (double)std::max<int64_t>(cells, 1);
  }
  if (need_bwd && g->d > 0 && g->T > 0) {
    // adjoint threshold tile: the reverse-scanned grad_out of one direction
    // tile and a 256-entry staging area must fit
    const int tt = choose_tile(
        g->T, [&](int t) { return wect::backward_lds_bytes(t, 256, 1) <= kLdsLimit; },
        [&](int t) { return wect::backward_lds_bytes(t, 256, 1) <= kLdsLimit; });
    if (tt == 0) return WECT_ERR_UNSUPPORTED;
    pl->tt_bwd = tt;
    int dg = std::min(ntiles, 4);
    int stage = block;
    while (dg > 0 && wect::backward_lds_bytes(tt, stage, dg) > kLdsLimit) --dg;
    if (dg == 0) {
      dg = 1;
      while (stage > 256 && wect::backward_lds_bytes(tt, stage, dg) > kLdsLimit) stage /= 2;
      if (wect::backward_lds_bytes(tt, stage, dg) > kLdsLimit) return WECT_ERR_UNSUPPORTED;
    }
    pl->dg = dg;
    pl->ngd = (int)ceil_div(ntiles, dg);
    pl->stage_bwd = stage;
    pl->lds_bwd = wect::backward_lds_bytes(tt, stage, dg);
    const int64_t S = (int64_t)pl->ngd * elems;
    const int64_t max_blocks = (int64_t)cus * blocks_per_cu(pl->lds_bwd);
    int64_t G = std::min<int64_t>(max_blocks, std::max<int64_t>(1, ceil_div(S, min_items)));
    G = std::min<int64_t>(G, std::max<int64_t>(S, 1));
    pl->G_bwd = (int)G;
    pl->S_bwd = S;
    pl->ws_bwd = 0;
  }
  p.T = g->T;  // the launches set their tile's thresholds
  return WECT_OK;
}

thread_local char g_last_error[256] = "";

// Remember a failed HIP call for wect_last_error() and map it to WECT_ERR_DEVICE.
wect_status device_error(hipError_t e, const char* where) {
  snprintf(g_last_error, sizeof(g_last_error), "%s: %s (%d)", where, hipGetErrorString(e), (int)e);
  return WECT_ERR_DEVICE;
}

// Creates and records a timing event; on failure nothing is left allocated.
hipError_t record(hipEvent_t* e, hipStream_t s) {
  hipError_t r = hipEventCreate(e);
  if (r != hipSuccess) {
    *e = nullptr;
    return r;
  }
  r = hipEventRecord(*e, s);
  if (r != hipSuccess) {
    (void)hipEventDestroy(*e);
    *e = nullptr;
  }
  return r;
}

wect_status run_forward(const Plan& pl0, void* out, void* ws, size_t ws_bytes, hipStream_t s) {
  Plan pl = pl0;
  Params& p = pl.p;
  const int Tfull = pl.T_full;
  const int64_t nout = (int64_t)p.B * p.d * Tfull;
  if (nout == 0) return WECT_OK;
  if (!out) return WECT_ERR_ARG;
  if (pl.ws_fwd > 0 && (!ws || ws_bytes < pl.ws_fwd)) return WECT_ERR_WORKSPACE;
  if (ws && (reinterpret_cast<uintptr_t>(ws) & 15)) return WECT_ERR_ARG;
  unsigned char* w8 = static_cast<unsigned char*>(ws);
  p.partial = w8;
  p.dsum = pl.dsum_bytes ? w8 + pl.partial_bytes : nullptr;
  p.split = pl.split ? 1 : 0;
  p.absmax = pl.absmax_bytes ? reinterpret_cast<float*>(w8 + pl.partial_bytes + pl.dsum_bytes) : nullptr;
  p.vbuckets = pl.vb_bytes ? w8 + pl.partial_bytes + pl.dsum_bytes + pl.absmax_bytes : nullptr;
  p.cub_rec = pl.rec_bytes ? w8 + pl.partial_bytes + pl.dsum_bytes + pl.absmax_bytes : nullptr;
  p.G = pl.G_fwd;
  p.S = pl.S_fwd;
  p.stage = pl.stage_fwd;
  // 1.5 stages of voxels per tile: about 55 % of the voxels of a volume contribute, so the stage rarely
  // overflows into the second round
  p.stage_vox = pl.two_vox ? std::min(2 * pl.block, (3 * pl.stage_fwd / 2) / 64 * 64) : 0;
  if (p.stage_vox <= p.stage) p.stage_vox = 0;
  p.ldo = Tfull;
  const bool prof = g_profile.load() != 0;
  if (p.nabsmax > 0) {
    if (hipError_t e = wect::launch_absmax(p, s); e != hipSuccess) return device_error(e, "abs-max kernel");
  }
  if (p.cub_rec && p.S > 0) {
    if (hipError_t e = wect::launch_cub_records(p, s); e != hipSuccess) return device_error(e, "voxel records kernel");
  }
  for (int q0 = 0; q0 < Tfull; q0 += pl.tt_fwd) {
    p.T = std::min(pl.tt_fwd, Tfull - q0);
    p.thr = pl.thr + q0;
    p.out = static_cast<unsigned char*>(out) + (size_t)q0 * 4;  // int32 or float32 entries
    if (p.n == 0 && p.S > 0) {
      if (hipError_t e = wect::launch_vertex_buckets(p, p.count[0] * (int64_t)p.d, s); e != hipSuccess)
        return device_error(e, "vertex index kernel");
    }
    if (p.S > 0) {
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (prof && record(&e0, s) != hipSuccess) return WECT_ERR_DEVICE;
      const hipError_t le = p.ls ? wect::launch_smooth_ls_forward(p, pl.block, pl.lds_fwd, s)
                                 : wect::launch_forward_main(p, pl.block, pl.lds_fwd, s);
      if (le != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return device_error(le, "forward kernel");
      }
      if (prof) {
        if (record(&e1, s) != hipSuccess) {
          (void)hipEventDestroy(e0);
          return WECT_ERR_DEVICE;
        }
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof.push_back({e0, e1, 0});
      }
    }
    if (hipError_t e = wect::launch_forward_reduce(p, s); e != hipSuccess) return device_error(e, "reduce kernel");
  }
  return WECT_OK;
}

wect_status run_backward(const Plan& pl0, const float* grad_out, float* const grad_w[4], float* grad_vertex,
                         hipStream_t s) {
  Plan pl = pl0;
  Params& p = pl.p;
  const int Tfull = pl.T_full;
  if (!grad_out && (int64_t)p.B * p.d * Tfull > 0) return WECT_ERR_ARG;
  if (p.wmode == WECT_W_VERTEX_MAX) {
    if (!grad_vertex && p.count[0] > 0) return WECT_ERR_ARG;
    p.grad_vertex = grad_vertex;
  } else {
    for (int i = 0; i < 4; ++i) p.grad_w[i] = grad_w ? grad_w[i] : nullptr;
  }
  p.cpw = 1;  // the adjoint keeps one cell per instruction
  p.dt = kW;
  p.dg = pl.dg;
  p.ngroups_dir = pl.ngd;
  p.G = pl.G_bwd;
  p.S = pl.S_bwd;
  p.stage = pl.stage_bwd;
  p.ldo = Tfull;
  const bool work = p.d > 0 && Tfull > 0 && p.S > 0;
  const int ntt = work ? (int)ceil_div(Tfull, pl.tt_bwd) : 0;
  // Outputs that are accumulated with atomics start from zero; with a single
  // direction group and a single threshold tile every explicit-weight
  // gradient is written exactly once.
  const bool atomic_explicit = pl.ngd > 1 || ntt > 1;
  p.bwd_atomic = atomic_explicit ? 1 : 0;
  if (p.wmode == WECT_W_VERTEX_MAX) {
    if (wect::launch_fill_zero(grad_vertex, p.count[0], s) != hipSuccess) return WECT_ERR_DEVICE;
  } else if (atomic_explicit || !work) {
    for (int i = 0; i <= p.top_dim; ++i)
      if (p.grad_w[i] && wect::launch_fill_zero(p.grad_w[i], p.count[i], s) != hipSuccess) return WECT_ERR_DEVICE;
  }
  if (!work) return WECT_OK;
  const bool prof = g_profile.load() != 0;
  for (int q0 = 0; q0 < Tfull; q0 += pl.tt_bwd) {
    p.T = std::min(pl.tt_bwd, Tfull - q0);
    p.thr = pl.thr + q0;
    p.grad_out = grad_out + q0;
    if (p.n == 0) {  // general vertex filter: threshold index of every filter value first
      if (hipError_t e = wect::launch_vertex_buckets(p, p.count[0] * (int64_t)p.d, s); e != hipSuccess)
        return device_error(e, "vertex index kernel");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (prof && record(&e0, s) != hipSuccess) return WECT_ERR_DEVICE;
    if (hipError_t e = wect::launch_backward_main(p, pl.block, pl.lds_bwd, s); e != hipSuccess) {
      if (e0) (void)hipEventDestroy(e0);
      return device_error(e, "adjoint kernel");
    }
    if (prof) {
      if (record(&e1, s) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return WECT_ERR_DEVICE;
      }
      std::lock_guard<std::mutex> lk(g_prof_mu);
      g_prof.push_back({e0, e1, 1});
    }
  }
  return WECT_OK;
}

// ---------------------------------------------------------------------------
// image ECF
// ---------------------------------------------------------------------------

// WECF of a general vertex filter on a simplicial complex: planned as a
// forward over m columns whose heights are read from fvals [V, m] (n = 0 in
// the kernels), so decomposition, staging and reduction are shared.  With
// sizing set, only the sizes are planned and fvals / thr may be null.
wect_status wecf_plan(const wect_complex* c, const float* fvals, int32_t m, const float* thr, int32_t T, Plan* pl,
                      bool bwd = false, bool sizing = false) {
  if (!c || c->kind != WECT_SIMPLICIAL || m < 0 || T < 0) return WECT_ERR_ARG;
  if (!sizing && m > 0 && c->count[0] > 0 && !fvals) return WECT_ERR_ARG;
  if (c->count[0] > 0 && m > 0 && c->count[0] > INT64_MAX / m) return WECT_ERR_ARG;
  // make_plan checks pointers it would read; here the coordinates are not
  // read and the directions are the filter columns, so stand-ins for the
  // pointers make_plan requires are passed and then cleared
  static const float kStandIn = 0.0f;
  wect_complex cc = *c;
  cc.n = 1;
  cc.coords = &kStandIn;
  const wect_grid gg = {&kStandIn, m, T, (thr || !sizing) ? thr : &kStandIn};
  if (wect_status st = make_plan(&cc, &gg, !bwd, bwd, pl); st != WECT_OK) return st;
  pl->p.n = 0;
  pl->p.coords = nullptr;
  pl->p.dirs = nullptr;
  pl->p.fvals = fvals;
  pl->thr = thr;
  pl->p.thr = thr;
  // threshold index of every filter value (within a launch's threshold tile,
  // at most T), one byte while T < 255
  pl->p.vb_bytes = T < 255 ? 1 : 2;
  if (pl->ws_fwd > 0 || (m > 0 && T > 0)) {
    pl->vb_bytes = align256((size_t)c->count[0] * (size_t)m * (size_t)pl->p.vb_bytes);
    if (!bwd) pl->ws_fwd += pl->vb_bytes;
  }
  return WECT_OK;
}

// Sigmoid relaxation (simplicial): the forward is planned like the WECT's with
// fixed-point accumulation; the adjoint takes one direction tile per block
// pass (g and its reverse scan in LDS) over the stream of ntiles x cells.
wect_status smooth_plan(const wect_complex* c, const wect_grid* g, float lam, bool need_fwd, bool need_bwd,
                        Plan* pl, bool ls = false) {
  if (!c || !g) return WECT_ERR_ARG;
  if (!(lam >= 0.0f) || !std::isfinite(lam)) return WECT_ERR_ARG;
  if (c->kind != WECT_SIMPLICIAL) return WECT_ERR_UNSUPPORTED;
  if (c->wmode == WECT_W_EXPLICIT && c->dtype != WECT_F32) return WECT_ERR_UNSUPPORTED;
  if (wect_status st = make_plan(c, g, need_fwd, false, pl, true, ls); st != WECT_OK) return st;
  pl->p.ls = ls ? 1 : 0;
  Params& p = pl->p;
  p.smooth = 1;
  p.dtype = WECT_F32;  // float32 output from 64-bit fixed point
  p.sm_lam = lam;
  p.sm_k = (float)((double)lam * 1.4426950408889634);  // lam log2(e)
  const double r = lam > 0.0f ? wect::kSmoothW / (double)lam : (double)FLT_MAX;
  p.sm_r = (float)std::min(r, (double)FLT_MAX);
  if (need_bwd && g->d > 0 && g->T > 0) {
    // threshold tile of the adjoint: all thresholds when they fit (per-cell
    // kernel: staging down to 64 cells; vertex-centric: 256-thread blocks),
    // else the fewest tiles that leave 256 staged cells
    auto fits = [&](int t, int st) {
      return ls ? wect::smooth_ls_backward_lds_bytes(t, 256) <= kLdsLimit
                : wect::smooth_backward_lds_bytes(t, st) <= kLdsLimit;
    };
    const int tt = choose_tile(g->T, [&](int t) { return fits(t, 64); }, [&](int t) { return fits(t, 256); });
    if (tt == 0) return WECT_ERR_UNSUPPORTED;
    pl->tt_bwd = tt;
    int block = g_block.load();
    if (ls) {  // at most the largest block whose coface rows fit, also for a caller's block
      const int fit = ls_block(tt, true);
      block = block ? std::min(block, fit) : fit;
    } else if (!block) {
      block = 1024;
    }
    if (block == 0) return WECT_ERR_UNSUPPORTED;
    int stage = block;
    size_t lds = 0;
    if (ls) {
      lds = wect::smooth_ls_backward_lds_bytes(tt, block);
    } else {
      while (stage > 64 && wect::smooth_backward_lds_bytes(tt, stage) > kLdsLimit) stage /= 2;
      lds = wect::smooth_backward_lds_bytes(tt, stage);
    }
    if (lds > kLdsLimit) return WECT_ERR_UNSUPPORTED;
    DeviceInfo di;
    const int cus = device_info(&di) ? di.cus : 256;
    const int user = g_bpc.load();
    const int64_t bpc = user > 0 ? user
                                 : std::max<int64_t>(1, std::min<int64_t>(32 / (block / kW),
                                                                          (int64_t)((160 * 1024) / (lds + 1024))));
    const int64_t S = (int64_t)p.ntiles * pl->elems;
    int64_t G = std::min<int64_t>((int64_t)cus * bpc, std::max<int64_t>(1, ceil_div(S, std::max(1, g_min_items.load()))));
    G = std::min<int64_t>(G, std::max<int64_t>(S, 1));
    pl->sm_block = block;
    pl->sm_stage = stage;
    pl->lds_bwd = lds;
    pl->G_bwd = (int)G;
    pl->S_bwd = S;
  }
  return WECT_OK;
}

wect_status run_smooth_backward(const Plan& pl0, const float* grad_out, float* grad_coords, float* grad_dirs,
                                float* const grad_w[4], float* grad_vertex, hipStream_t s) {
  Plan pl = pl0;
  Params& p = pl.p;
  const int Tfull = pl.T_full;
  if (!grad_out && (int64_t)p.B * p.d * Tfull > 0) return WECT_ERR_ARG;
  p.grad_coords = grad_coords;
  p.grad_dirs = grad_dirs;
  if (p.wmode == WECT_W_VERTEX_MAX) p.grad_vertex = grad_vertex;
  else if (p.wmode == WECT_W_EXPLICIT)
    for (int i = 0; i < 4; ++i) p.grad_w[i] = grad_w ? grad_w[i] : nullptr;
  p.G = pl.G_bwd;
  p.S = pl.S_bwd;
  p.stage = pl.sm_stage;
  p.ldo = Tfull;
  const bool work = p.d > 0 && Tfull > 0 && p.S > 0;
  const int ntt = work ? (int)ceil_div(Tfull, pl.tt_bwd) : 0;
  // explicit-weight gradients are written once when there is one direction
  // tile and one threshold tile
  p.bwd_atomic = (p.ntiles > 1 || ntt > 1) ? 1 : 0;
  auto zero = [&](float* x, int64_t n) { return x ? wect::launch_fill_zero(x, n, s) : hipSuccess; };
  if (zero(grad_coords, p.count[0] * (int64_t)p.n) != hipSuccess) return WECT_ERR_DEVICE;
  if (zero(grad_dirs, (int64_t)p.d * p.n) != hipSuccess) return WECT_ERR_DEVICE;
  if (p.wmode == WECT_W_VERTEX_MAX && zero(grad_vertex, p.count[0]) != hipSuccess) return WECT_ERR_DEVICE;
  // the vertex-centric adjoint adds a cell's gradient from each of its vertices
  if (p.wmode == WECT_W_EXPLICIT && (p.bwd_atomic || p.ls || !work)) {
    for (int i = 0; i <= p.top_dim; ++i)
      if (zero(p.grad_w[i], p.count[i]) != hipSuccess) return WECT_ERR_DEVICE;
  }
  if (!work) return WECT_OK;
  const bool prof = g_profile.load() != 0;
  for (int q0 = 0; q0 < Tfull; q0 += pl.tt_bwd) {
    p.T = std::min(pl.tt_bwd, Tfull - q0);
    p.thr = pl.thr + q0;
    p.grad_out = grad_out + q0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (prof && record(&e0, s) != hipSuccess) return WECT_ERR_DEVICE;
    const hipError_t le = p.ls ? wect::launch_smooth_ls_backward(p, pl.sm_block, pl.lds_bwd, s)
                              : wect::launch_smooth_backward(p, pl.sm_block, pl.lds_bwd, s);
    if (le != hipSuccess) {
      if (e0) (void)hipEventDestroy(e0);
      return device_error(le, "relaxation adjoint kernel");
    }
    if (prof) {
      if (record(&e1, s) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return WECT_ERR_DEVICE;
      }
      std::lock_guard<std::mutex> lk(g_prof_mu);
      g_prof.push_back({e0, e1, 1});
    }
  }
  return WECT_OK;
}

// Lower-star index of a simplicial complex: layout from host counts.
wect_status ls_check(const wect_complex* c, wect::LsLayout* L) {
  if (!c || c->kind != WECT_SIMPLICIAL) return WECT_ERR_ARG;
  const wect_grid g0 = {nullptr, 0, 0, nullptr};
  Plan pl;
  if (wect_status st = make_plan(c, &g0, false, false, &pl); st != WECT_OK) return st;
  *L = wect::ls_layout(c->count[0], c->count, c->top_dim);
  return WECT_OK;
}

// Binds a caller's index to a relaxation plan (vertex-centric kernels).
wect_status ls_attach(const wect_complex* c, const void* index, size_t index_bytes, Plan* pl) {
  wect::LsLayout L;
  if (wect_status st = ls_check(c, &L); st != WECT_OK) return st;
  if (!index || index_bytes < L.total || (reinterpret_cast<uintptr_t>(index) & 15)) return WECT_ERR_ARG;
  wect::ls_bind(pl->p, const_cast<void*>(index), L);
  return WECT_OK;
}

struct EcfPlan {
  Params p;
  int block = 1024;
  size_t ws = 0;
};

wect_status ecf_plan(const wect_complex* c, int32_t T, const float* thr, EcfPlan* pl) {
  if (!c || T < 0 || (T > 0 && !thr)) return WECT_ERR_ARG;
  if (c->kind != WECT_CUBICAL || (c->n != 2 && c->n != 3) || c->B < 1) return WECT_ERR_ARG;
  if (c->wmode == WECT_W_EXPLICIT) return WECT_ERR_UNSUPPORTED;
  if (c->wmode != WECT_W_ONES && c->wmode != WECT_W_VERTEX_MAX) return WECT_ERR_ARG;
  if (c->dtype != WECT_I32 || c->total_voxels < 0 || !c->shape) return WECT_ERR_ARG;
  if (c->total_voxels > 0 && !c->intensity) return WECT_ERR_ARG;
  if (c->B > 1 && !c->grid_off) return WECT_ERR_ARG;
  if (c->include_above < -1 || c->include_above > 255) return WECT_ERR_ARG;
  Params& p = pl->p;
  std::memset(&p, 0, sizeof(p));
  p.dpl = 1;
  p.kind = WECT_CUBICAL;
  p.n = c->n;
  p.B = c->B;
  p.wmode = c->wmode;
  p.dtype = WECT_I32;
  p.shape = c->shape;
  p.grid_off = c->grid_off;
  p.intensity = c->intensity;
  p.total_voxels = c->total_voxels;
  p.include_above = c->include_above;
  p.thr = thr;
  p.T = T;
  p.ntiles = 1;  // one group per image
  DeviceInfo di;
  const int cus = device_info(&di) ? di.cus : 256;
  const int64_t S = c->total_voxels;
  // 1024-thread blocks, two per compute unit, at least 8192 voxels each
  const int64_t G = std::max<int64_t>(1, std::min<int64_t>(2LL * cus, ceil_div(S, 8192)));
  p.S = S;
  p.G = (int)G;
  pl->ws = align256((size_t)c->B * wect::kEcfRowBytes);
  return WECT_OK;
}

}  // namespace

namespace wect {
void set_last_error(const char* msg) { snprintf(g_last_error, sizeof(g_last_error), "%s", msg); }

size_t workspace_bytes_lean(const wect_complex* c, const wect_grid* g) {
  Plan pl;
  if (make_plan(c, g, true, false, &pl, false, false, true) != WECT_OK) return 0;
  return pl.ws_fwd;
}

wect_status forward_lean(const wect_complex* c, const wect_grid* g, void* out, void* ws, size_t ws_bytes,
                         void* hip_stream) {
  Plan pl;
  wect_status st = make_plan(c, g, true, false, &pl, false, false, true);
  if (st != WECT_OK) return st;
  return run_forward(pl, out, ws, ws_bytes, (hipStream_t)hip_stream);
}
}  // namespace wect

extern "C" {

const char* wect_status_string(wect_status s) {
  switch (s) {
    case WECT_OK: return "ok";
    case WECT_ERR_ARG: return "invalid argument";
    case WECT_ERR_INDEX: return "vertex id, offset or shape out of range";
    case WECT_ERR_THRESHOLDS: return "thresholds not non-decreasing or axis not strictly increasing";
    case WECT_ERR_NONFINITE: return "NaN or Inf in the input";
    case WECT_ERR_WORKSPACE: return "workspace missing or too small";
    case WECT_ERR_UNSUPPORTED: return "unsupported request";
    case WECT_ERR_DEVICE: return "HIP runtime error";
  }
  return "unknown status";
}

const char* wect_version(void) { return "wect 0.1 gfx950"; }

const char* wect_last_error(void) { return g_last_error; }

size_t wect_workspace_bytes(const wect_complex* c, const wect_grid* g, int with_backward) {
  Plan pl;
  if (make_plan(c, g, true, with_backward != 0, &pl) != WECT_OK) return 0;
  return std::max(pl.ws_fwd, pl.ws_bwd);
}

wect_status wect_forward(const wect_complex* c, const wect_grid* g, void* out, void* ws, size_t ws_bytes,
                         void* hip_stream) {
  Plan pl;
  wect_status st = make_plan(c, g, true, false, &pl);
  if (st != WECT_OK) return st;
  return run_forward(pl, out, ws, ws_bytes, (hipStream_t)hip_stream);
}

wect_status wect_backward(const wect_complex* c, const wect_grid* g, const float* grad_out,
                          float* const grad_w[4], float* grad_vertex, void* ws, size_t ws_bytes, void* hip_stream) {
  (void)ws;
  (void)ws_bytes;
  Plan pl;
  wect_status st = make_plan(c, g, false, true, &pl);
  if (st != WECT_OK) return st;
  return run_backward(pl, grad_out, grad_w, grad_vertex, (hipStream_t)hip_stream);
}

wect_status wect_batched(const wect_complex* c, const wect_grid* g, void* out, const float* grad_out,
                         float* const grad_w[4], float* grad_vertex, void* ws, size_t ws_bytes, void* hip_stream) {
  const bool bwd = grad_out != nullptr;
  Plan pl;
  wect_status st = make_plan(c, g, true, bwd, &pl);
  if (st != WECT_OK) return st;
  // all metadata checks of the backward happen before anything is enqueued
  if (bwd) {
    if (c->wmode == WECT_W_VERTEX_MAX && !grad_vertex && c->count[0] > 0) return WECT_ERR_ARG;
  }
  if ((int64_t)c->B * g->d * g->T > 0 && !out) return WECT_ERR_ARG;
  if (pl.ws_fwd > 0 && (!ws || ws_bytes < pl.ws_fwd)) return WECT_ERR_WORKSPACE;
  st = run_forward(pl, out, ws, ws_bytes, (hipStream_t)hip_stream);
  if (st != WECT_OK || !bwd) return st;
  return run_backward(pl, grad_out, grad_w, grad_vertex, (hipStream_t)hip_stream);
}

wect_status wect_validate(const wect_complex* c, const wect_grid* g, void* hip_stream) {
  Plan pl;
  wect_status st = make_plan(c, g, false, false, &pl);
  if (st != WECT_OK) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  int* dflags = nullptr;
  if (hipMalloc(&dflags, sizeof(int)) != hipSuccess) return WECT_ERR_DEVICE;
  int flags = 0;
  bool ok = hipMemcpyAsync(dflags, &flags, sizeof(int), hipMemcpyHostToDevice, s) == hipSuccess;
  ok = ok && wect::launch_validate(pl.p, dflags, s) == hipSuccess;
  ok = ok && hipMemcpyAsync(&flags, dflags, sizeof(int), hipMemcpyDeviceToHost, s) == hipSuccess;
  ok = ok && hipStreamSynchronize(s) == hipSuccess;
  (void)hipFree(dflags);
  if (!ok) return WECT_ERR_DEVICE;
  if (flags & wect::kFlagIndex) return WECT_ERR_INDEX;
  if (flags & wect::kFlagThr) return WECT_ERR_THRESHOLDS;
  if (flags & wect::kFlagNonfinite) return WECT_ERR_NONFINITE;
  return WECT_OK;
}

wect_status wect_set_launch(const wect_launch* l) {
  if (!l) return WECT_ERR_ARG;
  if (l->block != 0 && !valid_block(l->block)) return WECT_ERR_ARG;
  if (l->blocks_per_cu < 0 || l->blocks_per_cu > 64 || l->min_items_per_block < 0) return WECT_ERR_ARG;
  if (l->decomposition < 0 || l->decomposition > 2) return WECT_ERR_ARG;
  if (l->threshold_tile < 0) return WECT_ERR_ARG;
  if (l->directions_per_lane < 0 || l->directions_per_lane > 2) return WECT_ERR_ARG;
  if (l->cubical_records < 0 || l->cubical_records > 3) return WECT_ERR_ARG;
  if (l->cell_packing < 0 || l->cell_packing > 1) return WECT_ERR_ARG;
  if (l->stage_entries < 0 || l->stage_entries > 1024 || l->stage_entries % 64 != 0) return WECT_ERR_ARG;
  g_stage.store(l->stage_entries);
  g_pack.store(l->cell_packing);
  g_rec.store(l->cubical_records);
  g_decomp.store(l->decomposition);
  g_ttile.store(l->threshold_tile);
  g_dpl.store(l->directions_per_lane);
  g_block.store(l->block);
  g_bpc.store(l->blocks_per_cu);
  g_min_items.store(l->min_items_per_block ? l->min_items_per_block : 256);
  return WECT_OK;
}

wect_status wect_get_launch(wect_launch* l) {
  if (!l) return WECT_ERR_ARG;
  l->block = g_block.load();
  l->blocks_per_cu = g_bpc.load();
  l->min_items_per_block = g_min_items.load();
  l->decomposition = g_decomp.load();
  l->threshold_tile = g_ttile.load();
  l->directions_per_lane = g_dpl.load();
  l->cubical_records = g_rec.load();
  l->cell_packing = g_pack.load();
  l->stage_entries = g_stage.load();
  return WECT_OK;
}

wect_status wect_profile_enable(int on) {
  g_profile.store(on ? 1 : 0);
  return WECT_OK;
}

wect_status wect_profile_read(double* fwd_ms, int64_t* fwd_launches, double* bwd_ms, int64_t* bwd_launches,
                              int reset) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  double ms[2] = {0.0, 0.0};
  int64_t cnt[2] = {0, 0};
  for (auto& e : g_prof) {
    if (hipEventSynchronize(e.b) != hipSuccess) return WECT_ERR_DEVICE;
    float t = 0.0f;
    if (hipEventElapsedTime(&t, e.a, e.b) != hipSuccess) return WECT_ERR_DEVICE;
    ms[e.bwd] += t;
    cnt[e.bwd] += 1;
  }
  if (fwd_ms) *fwd_ms = ms[0];
  if (fwd_launches) *fwd_launches = cnt[0];
  if (bwd_ms) *bwd_ms = ms[1];
  if (bwd_launches) *bwd_launches = cnt[1];
  if (reset) {
    for (auto& e : g_prof) {
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
    g_prof.clear();
  }
  return WECT_OK;
}

size_t wect_wecf_workspace_bytes(const wect_complex* c, int32_t m, int32_t T) {
  Plan pl;
  if (wecf_plan(c, nullptr, m, nullptr, T, &pl, false, true) != WECT_OK) return 0;
  return pl.ws_fwd;
}

wect_status wect_wecf_forward(const wect_complex* c, const float* fvals, int32_t m, const float* thr, int32_t T,
                              void* out, void* ws, size_t ws_bytes, void* hip_stream) {
  Plan pl;
  if (wect_status st = wecf_plan(c, fvals, m, thr, T, &pl); st != WECT_OK) return st;
  return run_forward(pl, out, ws, ws_bytes, (hipStream_t)hip_stream);
}

wect_status wect_wecf_backward(const wect_complex* c, const float* fvals, int32_t m, const float* thr, int32_t T,
                               const float* grad_out, float* const grad_w[4], float* grad_vertex, void* ws,
                               size_t ws_bytes, void* hip_stream) {
  Plan pl;
  if (wect_status st = wecf_plan(c, fvals, m, thr, T, &pl, true); st != WECT_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const bool work = (int64_t)c->B * m * T > 0 && pl.S_bwd > 0;
  if (work) {
    if (!ws || ws_bytes < pl.vb_bytes) return WECT_ERR_WORKSPACE;
    if (reinterpret_cast<uintptr_t>(ws) & 15) return WECT_ERR_ARG;
    if (c->wmode == WECT_W_VERTEX_MAX && !grad_vertex && c->count[0] > 0) return WECT_ERR_ARG;
    if (!grad_out) return WECT_ERR_ARG;
    // run_backward forms the threshold index of every filter value for each
    // threshold tile first (Algorithm 1's order), then runs the adjoint
    pl.p.vbuckets = ws;
  }
  return run_backward(pl, grad_out, grad_w, grad_vertex, s);
}

wect_status wect_freudenthal_counts(int32_t B, const int32_t* shape_host, int64_t counts[3]) {
  if (B < 1 || !shape_host || !counts) return WECT_ERR_ARG;
  int64_t v = 0, e = 0, t = 0;
  for (int32_t b = 0; b < B; ++b) {
    const int64_t n0 = shape_host[3 * b], n1 = shape_host[3 * b + 1];
    if (n0 < 1 || n1 < 1 || shape_host[3 * b + 2] != 1 || n0 * n1 > INT32_MAX) return WECT_ERR_ARG;
    v += n0 * n1;
    e += (n0 - 1) * n1 + n0 * (n1 - 1) + (n0 - 1) * (n1 - 1);
    t += 2 * (n0 - 1) * (n1 - 1);
  }
  counts[0] = v;
  counts[1] = e;
  counts[2] = t;
  return WECT_OK;
}

wect_status wect_freudenthal_build(const wect_complex* c, float* coords, float* vweights, int32_t* edges,
                                   int32_t* tris, int64_t* vert_off, int64_t* edge_off, int64_t* tri_off,
                                   void* hip_stream) {
  if (!c || c->kind != WECT_CUBICAL || c->n != 2 || c->B < 1 || !c->shape || !c->axis) return WECT_ERR_ARG;
  if (c->total_voxels < 0 || (c->B > 1 && (!c->grid_off || !c->axis_off))) return WECT_ERR_ARG;
  if (!vert_off || !edge_off || !tri_off) return WECT_ERR_ARG;
  if (c->total_voxels > 0 && (!c->intensity || !coords || !vweights || !edges || !tris)) return WECT_ERR_ARG;
  Params p;
  std::memset(&p, 0, sizeof(p));
  p.dpl = 1;
  p.kind = WECT_CUBICAL;
  p.n = 2;
  p.B = c->B;
  p.shape = c->shape;
  p.grid_off = c->grid_off;
  p.intensity = c->intensity;
  p.axis = c->axis;
  p.axis_off = c->axis_off;
  p.total_voxels = c->total_voxels;
  if (hipError_t e = wect::launch_freudenthal(p, vert_off, edge_off, tri_off, coords, vweights, edges, tris,
                                              static_cast<hipStream_t>(hip_stream));
      e != hipSuccess)
    return device_error(e, "Freudenthal builder");
  return WECT_OK;
}

size_t wect_smooth_workspace_bytes(const wect_complex* c, const wect_grid* g, float lam) {
  Plan pl;
  if (smooth_plan(c, g, lam, true, false, &pl) != WECT_OK) return 0;
  return pl.ws_fwd;
}

wect_status wect_smooth_forward(const wect_complex* c, const wect_grid* g, float lam, float* out, void* ws,
                                size_t ws_bytes, void* hip_stream) {
  Plan pl;
  if (wect_status st = smooth_plan(c, g, lam, true, false, &pl); st != WECT_OK) return st;
  return run_forward(pl, out, ws, ws_bytes, (hipStream_t)hip_stream);
}

wect_status wect_smooth_backward(const wect_complex* c, const wect_grid* g, float lam, const float* grad_out,
                                 float* grad_coords, float* grad_dirs, float* const grad_w[4], float* grad_vertex,
                                 void* hip_stream) {
  Plan pl;
  if (wect_status st = smooth_plan(c, g, lam, false, true, &pl); st != WECT_OK) return st;
  return run_smooth_backward(pl, grad_out, grad_coords, grad_dirs, grad_w, grad_vertex, (hipStream_t)hip_stream);
}

size_t wect_lower_star_bytes(const wect_complex* c) {
  wect::LsLayout L;
  if (ls_check(c, &L) != WECT_OK) return 0;
  return L.total;
}

wect_status wect_lower_star_build(const wect_complex* c, void* index, size_t index_bytes, void* hip_stream) {
  wect::LsLayout L;
  if (wect_status st = ls_check(c, &L); st != WECT_OK) return st;
  if (!index || index_bytes < L.total || (reinterpret_cast<uintptr_t>(index) & 15)) return WECT_ERR_ARG;
  const wect_grid g0 = {nullptr, 0, 0, nullptr};
  Plan pl;
  if (wect_status st = make_plan(c, &g0, false, false, &pl); st != WECT_OK) return st;
  wect::ls_bind(pl.p, index, L);
  if (hipError_t e = wect::launch_lower_star_build(pl.p, L, static_cast<hipStream_t>(hip_stream)); e != hipSuccess)
    return device_error(e, "lower-star index build");
  return WECT_OK;
}

size_t wect_smooth_ls_workspace_bytes(const wect_complex* c, const wect_grid* g, float lam) {
  Plan pl;
  if (smooth_plan(c, g, lam, true, false, &pl, true) != WECT_OK) return 0;
  return pl.ws_fwd;
}

wect_status wect_smooth_ls_forward(const wect_complex* c, const wect_grid* g, float lam, const void* index,
                                   size_t index_bytes, float* out, void* ws, size_t ws_bytes, void* hip_stream) {
  Plan pl;
  if (wect_status st = smooth_plan(c, g, lam, true, false, &pl, true); st != WECT_OK) return st;
  if (wect_status st = ls_attach(c, index, index_bytes, &pl); st != WECT_OK) return st;
  return run_forward(pl, out, ws, ws_bytes, (hipStream_t)hip_stream);
}

wect_status wect_smooth_ls_backward(const wect_complex* c, const wect_grid* g, float lam, const void* index,
                                    size_t index_bytes, const float* grad_out, float* grad_coords, float* grad_dirs,
                                    float* const grad_w[4], float* grad_vertex, void* hip_stream) {
  Plan pl;
  if (wect_status st = smooth_plan(c, g, lam, false, true, &pl, true); st != WECT_OK) return st;
  if (wect_status st = ls_attach(c, index, index_bytes, &pl); st != WECT_OK) return st;
  return run_smooth_backward(pl, grad_out, grad_coords, grad_dirs, grad_w, grad_vertex, (hipStream_t)hip_stream);
}

size_t wect_image_ecf_workspace_bytes(const wect_complex* c) {
  EcfPlan pl;
  if (ecf_plan(c, 0, nullptr, &pl) != WECT_OK) return 0;
  return pl.ws;
}

wect_status wect_image_ecf(const wect_complex* c, const float* thr, int32_t T, int32_t* out, void* ws,
                           size_t ws_bytes, void* hip_stream) {
  EcfPlan pl;
  if (wect_status st = ecf_plan(c, T, thr, &pl); st != WECT_OK) return st;
  if ((int64_t)c->B * T == 0) return WECT_OK;
  if (!out) return WECT_ERR_ARG;
  if (!ws || ws_bytes < pl.ws) return WECT_ERR_WORKSPACE;
  pl.p.out = out;
  pl.p.partial = ws;
  if (hipError_t e = wect::launch_image_ecf(pl.p, pl.block, static_cast<hipStream_t>(hip_stream)); e != hipSuccess)
    return device_error(e, "image ECF kernels");
  return WECT_OK;
}

}  // extern "C"
