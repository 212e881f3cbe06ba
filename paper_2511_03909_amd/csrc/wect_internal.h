// Internal interface between the host runtime (wect_api.cpp) and the HIP
// kernels (k_*.hip, with device helpers in wect_device.h).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wect {

constexpr int kWave = 64;          // lanes per wavefront on gfx950; one lane = one direction
constexpr size_t kLdsBudget = 160 * 1024 - 1024;  // dynamic LDS per workgroup on gfx950 (160 KiB, less static use)
constexpr int kMaxStride = 16;     // floats per staged simplicial entry (4 vertices x 3 + weight + owner)

// Everything a kernel needs, passed by value.
struct Params {
  // complex
  int32_t kind, n, B, top_dim, wmode, dtype;
  const float* coords;
  const float* fvals;    // n = 0: vertex filter values [V, d] row-major (WECF of a general filter)
  void* vbuckets;        // n = 0: threshold index of every filter value [V, d], uint8 or uint16
  int32_t vb_bytes;      // 1 (T < 255) or 2
  const int64_t* vert_off;
  int64_t count[4];
  const int32_t* simp[4];
  const int64_t* simp_off[4];
  const void* weights[4];
  const int32_t* shape;
  const int64_t* grid_off;
  const uint8_t* intensity;
  const float* axis;
  const int64_t* axis_off;
  int64_t total_voxels;
  int32_t include_above;
  void* cub_rec;         // cubical: per-voxel records of combined weights (k_cub_records), or null
  // sampling grid
  const float* dirs;
  int32_t d, T;          // T: thresholds of this launch (one tile of the request's thresholds)
  const float* thr;      // the launch's thresholds (first entry of its tile)
  int32_t ldo;           // row stride of out and grad_out: the request's full threshold count
  // decomposition
  int32_t ntiles;        // direction tiles of 64 * dpl (forward) / per group (backward)
  int32_t dpl;           // directions per lane: 1, or 2 (cubical forward: a tile of 128 directions, two
                         // histogram columns per lane, so each staged voxel serves both)
  int32_t cpw, dt;       // simplicial forward with d <= 32: cells per wavefront instruction (64 / dt) and
                         // the power of two dt >= d of columns per cell; lane l serves column l % dt of
                         // cell l / dt (cpw = 1, dt = 64: one cell per instruction)
  int32_t G;             // blocks of the main kernel
  int64_t S;             // stream length: sum over groups of the stream elements
  int32_t stage;         // staged entries per tile (<= blockDim.x)
  int32_t stage_vox;     // cubical forward with voxel records: voxels per tile, stage < stage_vox <=
                         // min(2 stage, 2 blockDim.x) (two per thread; the contributing ones past the
                         // stage go in a second round); otherwise 0 (one voxel per thread, stage of them)
  int32_t dg;            // backward: direction tiles held in LDS at once
  int32_t ngroups_dir;   // backward: number of direction groups ( = ceil(ntiles / dg) )
  void* partial;         // forward: [slots][T][64] uint32 (integer weights) / uint64 (fixed point)
  void* dsum;            // forward, split reduction: [groups][T][64] slot sums
  int32_t split;         // 1: k_slot_sum first, then the scan reads dsum
  int32_t group_mode;    // 1: block k handles exactly group k (G = groups), no reduction kernel
  float* absmax;         // float32 weights: per-block max |w| ([nabsmax])
  int32_t nabsmax;
  double cells_total;    // bound on the cells of any complex (fixed-point scale)
  void* out;             // forward: [B][d][T]
  // backward
  const float* grad_out;         // [B][d][T]
  float* grad_w[4];
  float* grad_vertex;
  int32_t bwd_atomic;            // 1: accumulate with atomics (output pre-zeroed)
  // sigmoid relaxation: sig(lam (thr - h)) in place of the step [h <= thr]
  int32_t smooth;                // 1: smooth forward / adjoint
  float sm_lam;                  // lam
  float sm_k;                    // lam log2(e), the exponent scale for exp2
  float sm_r;                    // window half-width in height units (kSmoothW / lam, capped at FLT_MAX)
  float* grad_coords;            // smooth adjoint: [count0, n], accumulated (pre-zeroed); may be null
  float* grad_dirs;              // smooth adjoint: [d, n], accumulated (pre-zeroed); may be null
  // lower-star index (relaxation, vertex-centric kernels): the stream runs over vertices
  int32_t ls;                    // 1: stream elements are vertices, cofaces read from the index
  int64_t* ls_hdr;               // [4]: [1] largest vertex degree (device-written), others reserved
  int64_t* ls_off;               // [V+1] CSR offsets of each vertex's cofaces
  int64_t* ls_cur;               // [V] build: counts, then fill cursors
  int64_t* ls_part;              // build: scan partial sums
  int32_t* ls_ent;               // [entries][4]: dim, then the other vertices' global rows (-1 pad)
  int64_t* ls_row;               // [entries]: the coface's row within its dimension
  uint32_t* ls_mask;             // [entries]: the coface's other vertices as bits over the vertex's edges
  int32_t* ls_nbc;               // [V]: the vertex's edge count when every coface maps to bits, else -1
};

// Sigmoid terms with |lam (thr - h)| > kSmoothW are taken as 0 (below) or 1
// (above): each such term is then off by less than exp(-17) < 2^-24.
constexpr double kSmoothW = 17.0;

// Launchers (enqueue only, return hipError_t of the launch).
hipError_t launch_forward_main(const Params& p, int block, size_t lds_bytes, hipStream_t s);
// the two kinds of forward main kernel, which launch_forward_main dispatches to
hipError_t launch_forward_simp(const Params& p, int block, size_t lds_bytes, hipStream_t s);
hipError_t launch_forward_cub(const Params& p, int block, size_t lds_bytes, hipStream_t s);
// Per-voxel records of the cubical forward (p.cub_rec, total_voxels entries of
// 8 (n = 2) or 16 (n = 3) bytes).
hipError_t launch_cub_records(const Params& p, hipStream_t s);
hipError_t launch_forward_reduce(const Params& p, hipStream_t s);
hipError_t launch_backward_main(const Params& p, int block, size_t lds_bytes, hipStream_t s);
// Adjoint of the sigmoid relaxation (p.G blocks over p.S = ntiles * cells).
hipError_t launch_smooth_backward(const Params& p, int block, size_t lds_bytes, hipStream_t s);
hipError_t launch_fill_zero(float* ptr, int64_t n, hipStream_t s);
hipError_t launch_validate(const Params& p, int* flags, hipStream_t s);
// Freudenthal complexes of a 2D image batch: CSR offsets (device), then the
// per-pixel coordinates, weights, edges and triangles.
hipError_t launch_freudenthal(const Params& p, int64_t* voff, int64_t* eoff, int64_t* toff, float* coords,
                              float* vw, int32_t* edges, int32_t* tris, hipStream_t s);
// Image ECF: main kernel (p.G blocks of `block` threads, when p.S > 0) and the
// per-image finish (p.B blocks).
hipError_t launch_image_ecf(const Params& p, int block, hipStream_t s);
constexpr int kEcfRowBytes = 256 * 4;  // one image's sums over the intensity values

hipError_t launch_absmax(const Params& p, hipStream_t s);
// n = 0: threshold index of every filter value (first pass of the general-filter WECF).
hipError_t launch_vertex_buckets(const Params& p, int64_t nvals, hipStream_t s);

// Lower-star index: layout inside one caller buffer, and its build (count,
// scan, fill: five kernels, no allocation).
struct LsLayout {
  size_t hdr, off, cur, part, ent, row, mask, nbc, total;
  int64_t nent, nparts;
};
LsLayout ls_layout(int64_t V, const int64_t count[4], int top_dim);
void ls_bind(Params& p, void* base, const LsLayout& L);
hipError_t launch_lower_star_build(const Params& p, const LsLayout& L, hipStream_t s);
// Vertex-centric relaxation kernels (p.ls = 1).
hipError_t launch_smooth_ls_forward(const Params& p, int block, size_t lds_bytes, hipStream_t s);
hipError_t launch_smooth_ls_backward(const Params& p, int block, size_t lds_bytes, hipStream_t s);
size_t smooth_ls_forward_lds_bytes(int T, int block);
size_t smooth_ls_backward_lds_bytes(int T, int block);
constexpr int kLsChunk = 8192;  // elements per block of the build's scan

// LDS bytes of the forward kernels: fixed part (histogram, thresholds) plus
// forward_entry_bytes per staged entry; of the backward kernel in total.
size_t forward_lds_fixed(int T, int kind, int acc_bytes, int dpl = 1);
size_t forward_entry_bytes(int kind, int n);
size_t backward_lds_bytes(int T, int stage, int dg);
size_t smooth_backward_lds_bytes(int T, int stage);

constexpr int kAbsmaxSlots = 256;  // blocks of k_absmax, one partial maximum each

// Records the description returned by wect_last_error() on the calling thread.
void set_last_error(const char* msg);

}  // namespace wect

#include "wect.h"

namespace wect {

// wect_workspace_bytes(c, g, 0) / wect_forward for a plan whose workspace holds
// the partial histograms only (no per-voxel records of the cubical forward):
// the allocation-free entry point's plan.
size_t workspace_bytes_lean(const wect_complex* c, const wect_grid* g);
wect_status forward_lean(const wect_complex* c, const wect_grid* g, void* out, void* ws, size_t ws_bytes,
                         void* hip_stream);

// Validation flags (bit set = failure).
enum : int { kFlagIndex = 1, kFlagThr = 2, kFlagNonfinite = 4 };

}  // namespace wect
