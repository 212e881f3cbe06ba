// Cubical forward: implicit cells of images and volumes.

#include "wect_device.h"

#include <type_traits>

namespace wect {
namespace {

// ---------------------------------------------------------------------------
// forward, cubical (implicit cells of an image / volume)
// ---------------------------------------------------------------------------
//
// Heights of a grid vertex are ((x_i*sx) + (y_j*sy)) + (z_k*sz).  Rounding is
// monotone, so for sx >= 0 the height never decreases with i (and never
// increases for sx < 0), and the same for the other axes: the maximum height
// of a cell is attained at its "top" corner, the corner furthest along the
// sign pattern of the direction.  Each vertex therefore adds, per direction,
// one combined weight: the signed weights of the 2^n cells (itself, its
// edges, squares, cubes) that it tops for that sign pattern ("orthant").  The
// 2^n combined weights of a vertex are computed once when it is staged; each
// lane then reads the one for its direction's orthant.  With a zero component
// the heights along that axis are equal, so either corner gives the same index.

// Staged entry of a contributing vertex (8 words): its axis coordinates, then
// its 2^N combined weights, int32 in 2D and int16 pairs in 3D (|weight| <=
// 2^(N-1) * 255 < 2^15, the layout of a voxel record), and in 3D the index
// i1 + n1 i2 of its grid row.  The 32-byte 3D entry leaves room for a larger
// staging tile next to the histogram of two directions per lane; a lane
// extracts its orthant's half with one bitfield extract.  Entries of one row
// share y s_y and z s_z, so each wavefront walks a contiguous run of entries,
// two at a time, keeps the row terms once for the first and once for the
// second entry of its pairs, and recomputes them only when the row changes:
// the height ((x s_x) + (y s_y)) + (z s_z) keeps its operations and their
// order.
template <int N>
struct CubLayout {
  static constexpr int NO = 1 << N;                 // orthants
  static constexpr bool PACKED = N == 3;            // int16 pairs
  static constexpr int COFF = N;                    // first weight word
  static constexpr int ROW = 7;                     // 3D: grid row of the vertex
  static constexpr int STRIDE = 8;
};

// Raw neighbourhood of one voxel, loaded one tile ahead of its use: the
// intensities of the 3^N voxels around it, its axis coordinates and which of
// its neighbours lie inside the grid.  Coordinates are clamped into the grid,
// so every load is unconditional and in bounds; cub_weights masks the
// neighbours outside (bits of `inside`: i0 > 0, i0 < n0-1, i1 > 0, i1 < n1-1,
// i2 > 0, i2 < n2-1).
template <int N>
struct CubFetch {
  static constexpr int M = N == 2 ? 9 : 27;
  int nb[M];
  float cx, cy, cz;
  uint32_t inside;
  bool valid;

  __device__ __forceinline__ void load(const uint8_t* vol, const float* ax0, const float* ax1, const float* ax2,
                                       int n0, int n1, int n2, int i0, int i1, int i2, bool active) {
    valid = active;
    i0 = min(i0, n0 - 1);  // past the end of the range: any in-bounds voxel
    i1 = min(i1, n1 - 1);
    i2 = min(i2, n2 - 1);
    const uint32_t col[3] = {(uint32_t)max(i0 - 1, 0), (uint32_t)i0, (uint32_t)min(i0 + 1, n0 - 1)};
    const int row[3] = {max(i1 - 1, 0), i1, min(i1 + 1, n1 - 1)};
    const int lay[3] = {max(i2 - 1, 0), i2, min(i2 + 1, n2 - 1)};
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int d0 = m % 3, d1 = (m / 3) % 3, d2 = N == 3 ? m / 9 : 1;
      nb[m] = vol[(uint32_t)(lay[d2] * n1 + row[d1]) * (uint32_t)n0 + col[d0]];
    }
    inside = (uint32_t)(i0 > 0) | (uint32_t)(i0 < n0 - 1) << 1 | (uint32_t)(i1 > 0) << 2 |
             (uint32_t)(i1 < n1 - 1) << 3 | (uint32_t)(i2 > 0) << 4 | (uint32_t)(i2 < n2 - 1) << 5;
    cx = ax0[i0];
    cy = ax1[i1];
    cz = N == 3 ? ax2[i2] : 0.0f;
  }
};

// Combined weights of a staged vertex for the 2^N orthants, from its raw
// neighbourhood.  Orthant bit k set means s_k < 0: the cells topped by v then
// extend towards +k, otherwise towards -k.  Each distinct cell containing v
// (2N edges, the squares of each axis pair, the 2^N cubes) is evaluated once.
template <int N, int WM>
__device__ __forceinline__ void cub_weights(const CubFetch<N>& f, int include_above, int32_t* cw) {
  constexpr int M = CubFetch<N>::M;
  auto nbi = [](int d0, int d1, int d2) { return (d0 + 1) + 3 * (d1 + 1) + (N == 3 ? 9 * (d2 + 1) : 0); };
  // neighbour present: inside the grid and a vertex (lane masks, no arithmetic)
  bool pr[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int d0 = m % 3 - 1, d1 = (m / 3) % 3 - 1, d2 = N == 3 ? m / 9 - 1 : 0;
    const bool in = (d0 < 0 ? (f.inside & 1) : d0 > 0 ? (f.inside & 2) : 1) &&
                    (d1 < 0 ? (f.inside & 4) : d1 > 0 ? (f.inside & 8) : 1) &&
                    (d2 < 0 ? (f.inside & 16) : d2 > 0 ? (f.inside & 32) : 1);
    pr[m] = in && f.nb[m] > include_above;
  }
  const int x = f.nb[nbi(0, 0, 0)];  // the voxel itself (a vertex: the caller checked)
  // a cell's weight: 1, or (vertex-max) the largest corner intensity; x is a corner of every cell here
  auto val = [&](bool present, int mx) { return present ? (WM == WM_ONES ? 1 : mx) : 0; };
  auto at = [&](int d0, int d1, int d2) { return f.nb[nbi(d0, d1, d2)]; };
  auto has = [&](int d0, int d1, int d2) { return pr[nbi(d0, d1, d2)]; };
  // edges E[axis][side] (side 0: towards -axis)
  int E[N][2], Emx[N][2];
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      const int s = sd ? 1 : -1;
      const int d0 = a == 0 ? s : 0, d1 = a == 1 ? s : 0, d2 = a == 2 ? s : 0;
      Emx[a][sd] = max(x, at(d0, d1, d2));
      E[a][sd] = val(has(d0, d1, d2), Emx[a][sd]);
    }
  const int vx = WM == WM_ONES ? 1 : x;
  if constexpr (N == 2) {
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      const int s0 = o & 1, s1 = (o >> 1) & 1;
      const int a0 = s0 ? 1 : -1, a1 = s1 ? 1 : -1;
      const bool sq = has(a0, 0, 0) && has(0, a1, 0) && has(a0, a1, 0);
      const int sqv = val(sq, max(max(Emx[0][s0], at(0, a1, 0)), at(a0, a1, 0)));
      cw[o] = vx - E[0][s0] - E[1][s1] + sqv;
    }
  } else {
    // squares F01[s0][s1], F02[s0][s2], F12[s1][s2]: presence and largest corner
    int F01[2][2], F02[2][2], F12[2][2], M01[2][2], M12[2][2];
    bool P01[2][2], P12[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int sa = a ? 1 : -1, sb = b ? 1 : -1;
        P01[a][b] = has(sa, 0, 0) && has(0, sb, 0) && has(sa, sb, 0);
        M01[a][b] = max(max(Emx[0][a], at(0, sb, 0)), at(sa, sb, 0));
        F01[a][b] = val(P01[a][b], M01[a][b]);
        const bool p02 = has(sa, 0, 0) && has(0, 0, sb) && has(sa, 0, sb);
        F02[a][b] = val(p02, max(max(Emx[0][a], at(0, 0, sb)), at(sa, 0, sb)));
        P12[a][b] = has(0, sa, 0) && has(0, 0, sb) && has(0, sa, sb);
        M12[a][b] = max(max(Emx[1][a], at(0, 0, sb)), at(0, sa, sb));
        F12[a][b] = val(P12[a][b], M12[a][b]);
      }
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      const int s0 = o & 1, s1 = (o >> 1) & 1, s2 = (o >> 2) & 1;
      const int a0 = s0 ? 1 : -1, a1 = s1 ? 1 : -1, a2 = s2 ? 1 : -1;
      // the cube's corners: those of F01 and F12 plus the 0-2 diagonal and the far corner
      const bool pc = P01[s0][s1] && P12[s1][s2] && has(a0, 0, a2) && has(a0, a1, a2);
      const int cube = val(pc, max(max(M01[s0][s1], M12[s1][s2]), max(at(a0, 0, a2), at(a0, a1, a2))));
      cw[o] = vx - E[0][s0] - E[1][s1] - E[2][s2] + F01[s0][s1] + F02[s0][s2] + F12[s1][s2] - cube;
    }
  }
}

// Voxel records: the 2^N combined weights of a voxel as int16 (|weight| is at
// most 2^(N-1) * 255 < 2^15), in grid order, all zero for a voxel that is not a
// vertex.  With several direction or threshold tiles the forward would stage
// every voxel once per tile; k_cub_records forms them once per call and the
// forward's staging then loads one 8- or 16-byte record per voxel instead of
// its 3^N neighbourhood.
template <int N>
struct CubRec {
  using R = typename std::conditional<N == 2, uint2, uint4>::type;
  static constexpr int NO = 1 << N;
  R r;
  float cx, cy, cz;
  bool valid;

  __device__ __forceinline__ void load(const R* rec, const float* ax0, const float* ax1, const float* ax2, int n0,
                                       int n1, int n2, int i0, int i1, int i2, uint32_t v, bool active) {
    valid = active;
    if (active) r = rec[v];
    i0 = min(i0, n0 - 1);
    i1 = min(i1, n1 - 1);
    i2 = min(i2, n2 - 1);
    cx = ax0[i0];
    cy = ax1[i1];
    cz = N == 3 ? ax2[i2] : 0.0f;
  }
  // the record's words (int16 pairs); false when all are zero (or the voxel is not staged)
  __device__ __forceinline__ bool packed(uint32_t* pk) const {
    if (!valid) return false;
    const uint32_t* w = reinterpret_cast<const uint32_t*>(&r);
    uint32_t any = 0;
#pragma unroll
    for (int k = 0; k < NO / 2; ++k) {
      any |= w[k];
      pk[k] = w[k];
    }
    return any != 0;
  }
  // combined weights; false when all are zero (or the voxel is not staged)
  __device__ __forceinline__ bool weights(int32_t* cw) const {
    if (!valid) return false;
    const uint32_t* w = reinterpret_cast<const uint32_t*>(&r);
    uint32_t any = 0;
#pragma unroll
    for (int k = 0; k < NO / 2; ++k) {
      any |= w[k];
      cw[2 * k] = (int32_t)(int16_t)(w[k] & 0xffffu);
      cw[2 * k + 1] = (int32_t)w[k] >> 16;
    }
    return any != 0;
  }
};

// q = floor(v / n) and v - q n for v, n < 2^32, n > 0: the double-precision
// quotient is within 2^-20 of v / n, so one correction step in either
// direction makes it exact.
__device__ __forceinline__ uint32_t divmod_u32(uint32_t v, uint32_t n, double inv, uint32_t& r) {
  int64_t q = (int64_t)((double)v * inv);
  int64_t rr = (int64_t)v - q * (int64_t)n;
  if (rr >= (int64_t)n) { ++q; rr -= n; }
  if (rr < 0) { --q; rr += n; }
  r = (uint32_t)rr;
  return (uint32_t)q;
}

// One thread per voxel: block (x, y) takes the voxels x * 256 + t,
// + gridDim.x * 256, ... of complexes y, y + gridDim.y, ...; the grid
// position comes from two exact double-precision divisions.
template <int N, int WM>
__global__ __launch_bounds__(256) void k_cub_records(Params p) {
  using RT = typename CubRec<N>::R;
  constexpr int NO = 1 << N;
  for (int b = blockIdx.y; b < p.B; b += gridDim.y) {
    const int n0 = p.shape[3 * b], n1 = p.shape[3 * b + 1], n2 = N == 3 ? p.shape[3 * b + 2] : 1;
    const int64_t goff = off_or(p.grid_off, b, p.total_voxels);
    const int64_t aoff = p.axis_off ? p.axis_off[b] : 0;
    const uint32_t nvox = (uint32_t)n0 * (uint32_t)n1 * (uint32_t)n2;
    const double inv0 = 1.0 / (double)n0, inv1 = 1.0 / (double)n1;
    const float* ax0 = p.axis + aoff;
    RT* rec = (RT*)p.cub_rec + goff;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += gridDim.x * blockDim.x) {
      uint32_t i0, i1;
      const uint32_t row = divmod_u32(v, (uint32_t)n0, inv0, i0);
      const uint32_t i2 = divmod_u32(row, (uint32_t)n1, inv1, i1);
      CubFetch<N> f;
      f.load(p.intensity + goff, ax0, ax0 + n0, ax0 + n0 + n1, n0, n1, n2, (int)i0, (int)i1, (int)i2, true);
      int32_t cw[NO];
#pragma unroll
      for (int o = 0; o < NO; ++o) cw[o] = 0;
      if (f.nb[(CubFetch<N>::M - 1) / 2] > p.include_above) cub_weights<N, WM>(f, p.include_above, cw);
      uint32_t w[NO / 2];
#pragma unroll
      for (int k = 0; k < NO / 2; ++k) w[k] = ((uint32_t)cw[2 * k] & 0xffffu) | ((uint32_t)cw[2 * k + 1] << 16);
      RT out;
      __builtin_memcpy(&out, w, sizeof(RT));
      rec[v] = out;
    }
  }
}

// Forward over the voxels [lo, hi) of complex b for one direction tile (DPL
// directions per lane): the neighbourhoods (or records, PRE) of tile t+1 are
// loaded while the histogram of tile t runs.
template <int N, int WM, bool FAST, int DPL, bool PRE, bool TWO>
__device__ void cub_fwd_range(const Params& p, int b, int64_t lo, int64_t hi, const float (&sx)[DPL],
                              const float (&sy)[DPL], const float (&sz)[DPL], const int (&orth)[DPL],
                              uint32_t* hist, float* stage, int* counter, const Thr& th) {
  using L = CubLayout<N>;
  const int tid = threadIdx.x, lane = tid & (W - 1);
  const int wave = uniform(tid >> 6), nw = blockDim.x >> 6;
  const int TS = p.stage;
  const int n0 = p.shape[3 * b], n1 = p.shape[3 * b + 1], n2 = N == 3 ? p.shape[3 * b + 2] : 1;
  const int64_t goff = off_or(p.grid_off, b, p.total_voxels);
  const int64_t aoff = p.axis_off ? p.axis_off[b] : 0;
  const uint8_t* vol = p.intensity + goff;
  const float* ax0 = p.axis + aoff;
  const float* ax1 = ax0 + n0;
  const float* ax2 = ax1 + n1;
  int arith = th.arith;
  // 3D: y s_y and z s_z of the row last seen, one cache per entry slot of a
  // pair (no row yet: row indices are below 2^31)
  uint32_t row[2] = {0xffffffffu, 0xffffffffu};
  float ysy[2][DPL], zsz[2][DPL];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int k = 0; k < DPL; ++k) ysy[j][k] = zsz[j][k] = 0.0f;
  // voxels per tile: TS (one per thread), or with TWO up to two per thread
  // (lo + tid and lo + blockDim + tid); the contributing vertices past the
  // stage's TS entries then go in a second round of the same tile
  const int BD = blockDim.x;
  const int TV = TWO ? min(p.stage_vox, min(2 * TS, 2 * BD)) : TS;
  const int TV0 = min(TV, BD);
  // grid position of the thread's voxel lo + tid, advanced by TV voxels per
  // tile without division (voxel counts of one complex are below 2^31)
  const uint32_t ts = (uint32_t)TV;
  const uint32_t s0 = ts % (uint32_t)n0, s1 = (ts / (uint32_t)n0) % (uint32_t)n1;
  const uint32_t s2 = ts / ((uint32_t)n0 * (uint32_t)n1);
  uint32_t v = (uint32_t)(lo + tid);
  int i0 = (int)(v % (uint32_t)n0), i1 = (int)((v / (uint32_t)n0) % (uint32_t)n1);
  int i2 = (int)(v / ((uint32_t)n0 * (uint32_t)n1));
  // TWO: the second voxel v + BD
  uint32_t v2 = v + (uint32_t)BD;
  int j0 = 0, j1 = 0, j2 = 0;
  if constexpr (TWO) {
    j0 = (int)(v2 % (uint32_t)n0);
    j1 = (int)((v2 / (uint32_t)n0) % (uint32_t)n1);
    j2 = (int)(v2 / ((uint32_t)n0 * (uint32_t)n1));
  }
  using Fetch = typename std::conditional<PRE, CubRec<N>, CubFetch<N>>::type;
  const typename CubRec<N>::R* rec = (const typename CubRec<N>::R*)p.cub_rec + goff;
  Fetch f, f2;
  auto fetch = [&]() {
    const bool active = v < (uint32_t)hi && tid < TV0;
    if constexpr (PRE) f.load(rec, ax0, ax1, ax2, n0, n1, n2, i0, i1, i2, v, active);
    else f.load(vol, ax0, ax1, ax2, n0, n1, n2, i0, i1, i2, active);
    if constexpr (TWO) f2.load(rec, ax0, ax1, ax2, n0, n1, n2, j0, j1, j2, v2, v2 < (uint32_t)hi && BD + tid < TV);
  };
  fetch();
  // the staged entry of a contributing vertex: coordinates, grid row and
  // combined weights (packed int16 pairs in 3D, int32 in 2D)
  auto put = [&](int slot, float cx, float cy, float cz, int a1, int a2, const uint32_t* pk, const int32_t* cw) {
    float* E = stage + slot * L::STRIDE;
    E[0] = cx;
    E[1] = cy;
    if constexpr (N == 3) {
      E[2] = cz;
      E[L::ROW] = bitcast<float>((uint32_t)a1 + (uint32_t)n1 * (uint32_t)a2);
    }
    if constexpr (L::PACKED) {
#pragma unroll
      for (int k = 0; k < L::NO / 2; ++k) E[L::COFF + k] = bitcast<float>(pk[k]);
    } else {
#pragma unroll
      for (int o = 0; o < L::NO; ++o) E[L::COFF + o] = bitcast<float>(cw[o]);
    }
  };
  // the lane's combined weight within an entry: word wo[k], bits sh[k] .. sh[k] + 15 when packed
  int wo[DPL], sh[DPL];
#pragma unroll
  for (int k = 0; k < DPL; ++k) {
    wo[k] = L::COFF + (L::PACKED ? orth[k] >> 1 : orth[k]);
    sh[k] = L::PACKED ? (orth[k] & 1) * 16 : 0;
  }
  auto weight = [&](const float* E, int k) -> uint32_t {
    const uint32_t x = bitcast<uint32_t>(E[wo[k]]);
    if constexpr (L::PACKED) return (uint32_t)__builtin_amdgcn_sbfe((int)x, (unsigned)sh[k], 16u);
    else return x;
  };
  auto row_terms = [&](const float* E, int j) {
    if constexpr (N == 3) {
      const uint32_t r = __builtin_amdgcn_readfirstlane(bitcast<uint32_t>(E[L::ROW]));
      if (r != row[j]) {
        row[j] = r;
#pragma unroll
        for (int k = 0; k < DPL; ++k) {
          ysy[j][k] = E[1] * sy[k];
          zsz[j][k] = E[2] * sz[k];
        }
      }
    }
  };
  auto hgt = [&](const float* E, int j, int k) -> float {
    if constexpr (N == 3) return (E[0] * sx[k] + ysy[j][k]) + zsz[j][k];
    else return height<N>(E, sx[k], sy[k], sz[k]);
  };
  // the histogram of the ne entries in the stage
  auto histogram = [&](int ne) {
    // the stage's address held in a vector register, so that the entry reads
    // of one step share one address register instead of copying a scalar one
    uint32_t vz;
    asm volatile("v_mov_b32 %0, 0" : "=v"(vz));
    const float* vstage = stage + vz;
    if constexpr (DPL == 1) {
      hist_entries<FAST, uint32_t>(hist + lane, 2 * wave, 2 * nw, ne, th, &arith,
                                   [&](int e, float& h, uint32_t& w) {
                                     const float* E = stage + e * L::STRIDE;
                                     row_terms(E, 0);
                                     h = hgt(E, 0, 0);
                                     w = weight(E, 0);
                                   });
    } else {
      // 3D: every wavefront takes a contiguous run of entries, so that its
      // row terms change only where the run crosses a grid row
      int first = 2 * wave, step = 2 * nw, last = ne;
      if constexpr (N == 3) {
        const int run = 2 * ((ne + 2 * nw - 1) / (2 * nw));
        first = min(ne, wave * run);
        last = min(ne, first + run);
        step = 2;
      }
      hist_entries2<FAST, uint32_t>(hist + lane, first, step, last, th, &arith,
                                    [&](int e, int j, int k, float& h, uint32_t& w) {
                                      const float* E = vstage + e * L::STRIDE;
                                      if (k == 0) row_terms(E, j);  // k = 1 follows for the same entry
                                      h = hgt(E, j, k);
                                      w = weight(E, k);
                                    });
    }
  };
  // every wavefront has used the values of all its reads of the stage (they
  // fed its atomics), so the stage may be overwritten once all have arrived;
  // the histogram additions still in flight need no wait
  auto stage_free = [&]() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };
  const double inv0 = 1.0 / (double)n0, inv1 = 1.0 / (double)n1;
  // two compaction counters take turns, so that clearing one needs no block
  // barrier of its own: a tile has two, after its staging and after its
  // histogram
  if (tid == 0) counter[0] = counter[1] = 0;
  __syncthreads();
  int par = 0;
  for (int64_t t0 = lo; t0 < hi; t0 += TV, par ^= 1) {
    bool keep = false, keep2 = false;
    int32_t cw[L::NO], cw2[L::NO];
    uint32_t pk[L::NO / 2], pk2[L::NO / 2];
    if constexpr (PRE && L::PACKED) {
      keep = f.packed(pk);
      if constexpr (TWO) keep2 = f2.packed(pk2);
    } else if constexpr (PRE) {
      keep = f.weights(cw);
      if constexpr (TWO) keep2 = f2.weights(cw2);
    } else if (f.valid && f.nb[(CubFetch<N>::M - 1) / 2] > p.include_above) {
      cub_weights<N, WM>(f, p.include_above, cw);
      bool nz = false;
#pragma unroll
      for (int o = 0; o < L::NO; ++o) nz = nz || (cw[o] != 0);
      keep = nz;
    }
    if constexpr (L::PACKED && !PRE) {
#pragma unroll
      for (int k = 0; k < L::NO / 2; ++k) pk[k] = ((uint32_t)cw[2 * k] & 0xffffu) | ((uint32_t)cw[2 * k + 1] << 16);
    }
    // compact the contributing vertices: this thread's first voxel, then (TWO)
    // its second, each wavefront reserving one range for both
    const uint64_t bal = __ballot(keep);
    const uint64_t bal2 = TWO ? __ballot(keep2) : 0ull;
    int base = 0;
    if (lane == 0 && (bal | bal2)) base = atomicAdd(counter + par, __popcll(bal) + __popcll(bal2));
    base = __shfl(base, 0);
    const uint64_t below = (1ull << lane) - 1ull;
    const int slot = base + __popcll(bal & below);
    const int slot2 = base + __popcll(bal) + __popcll(bal2 & below);
    // TWO: entries past the stage wait for the second round (slot - TS)
    uint32_t dv = 0, dv2 = 0;
    int dslot = -1, dslot2 = -1;
    if (keep) {
      if (!TWO || slot < TS) put(slot, f.cx, f.cy, f.cz, i1, i2, pk, cw);
      else dslot = slot - TS, dv = v;
    }
    if constexpr (TWO) {
      if (keep2) {
        if (slot2 < TS) put(slot2, f2.cx, f2.cy, f2.cz, j1, j2, pk2, cw2);
        else dslot2 = slot2 - TS, dv2 = v2;
      }
    }
    // neighbourhoods of the next tile (in flight during this tile's histogram)
    i0 += (int)s0;
    int carry = i0 >= n0;
    i0 -= carry ? n0 : 0;
    i1 += (int)s1 + carry;
    carry = i1 >= n1;
    i1 -= carry ? n1 : 0;
    i2 += (int)s2 + carry;
    v += ts;
    if constexpr (TWO) {
      j0 += (int)s0;
      carry = j0 >= n0;
      j0 -= carry ? n0 : 0;
      j1 += (int)s1 + carry;
      carry = j1 >= n1;
      j1 -= carry ? n1 : 0;
      j2 += (int)s2 + carry;
      v2 += ts;
    }
    fetch();
    // the next tile's counter: its last readers read it before the barrier
    // that ended the previous tile, and the barrier below (which waits for the
    // wavefront's LDS writes) orders the clearing before the next tile's
    // additions
    if (tid == 0) counter[par ^ 1] = 0;
    __syncthreads();
    const int ne = uniform(counter[par]);
    histogram(min(ne, TS));
    if constexpr (TWO) {
      if (ne > TS) {  // the same for every thread: the stage overflowed
        stage_free();
        // the deferred vertices: their records again (from cache), their
        // grid positions by division
        auto refetch = [&](int ds, uint32_t u) {
          uint32_t a0, a1;
          const uint32_t r = divmod_u32(u, (uint32_t)n0, inv0, a0);
          const uint32_t a2 = divmod_u32(r, (uint32_t)n1, inv1, a1);
          CubRec<N> g;
          g.load(rec, ax0, ax1, ax2, n0, n1, n2, (int)a0, (int)a1, (int)a2, u, true);
          int32_t gw[L::NO];
          uint32_t gp[L::NO / 2];
          if constexpr (L::PACKED) g.packed(gp);
          else g.weights(gw);
          put(ds, g.cx, g.cy, g.cz, (int)a1, (int)a2, gp, gw);
        };
        if (dslot >= 0) refetch(dslot, dv);
        if (dslot2 >= 0) refetch(dslot2, dv2);
        __syncthreads();
        histogram(ne - TS);
      }
    }
    stage_free();
  }
  __syncthreads();  // every addition has landed before the caller reads the histogram
}

template <int N, int WM, int DPL, bool PRE>
__global__ __launch_bounds__(1024) void k_cub_fwd(Params p) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int T = p.T;
  uint32_t* hist = (uint32_t*)smem;
  size_t off = (size_t)(T + 1) * W * DPL * 4;
  float* P = (float*)(smem + off);
  off += align_up((size_t)(T + 1) * 4, 16);
  int* counter = (int*)(smem + off);
  off += 16;
  float* stage = (float*)(smem + off);
  Thr th;
  setup_thresholds(p.thr, T, P, th);
  for (int i = threadIdx.x; i < (T + 1) * W * DPL; i += blockDim.x) hist[i] = 0u;
  __syncthreads();

  const int k = blockIdx.x;
  int64_t pos, end;
  int b;
  if (!block_range<uint32_t>(p, hist, k, 0, pos, end, b)) return;
  const int gpc = p.ntiles;
  const int lane = threadIdx.x & (W - 1);
  while (pos < end) {
    const int64_t cb = cum_elems(p, b);
    const int64_t nb = cum_elems(p, b + 1) - cb;
    if (nb == 0) { ++b; continue; }
    const int64_t base = (int64_t)gpc * cb;
    const int t = (int)((pos - base) / nb);
    const int64_t e0 = (pos - base) - (int64_t)t * nb;
    const int64_t e1 = mn64(nb, e0 + (end - pos));
    float sx[DPL], sy[DPL], sz[DPL];
    int orth[DPL];
#pragma unroll
    for (int j = 0; j < DPL; ++j) {
      load_dir(p, t * W * DPL + j * W + lane, sx[j], sy[j], sz[j]);
      orth[j] = (sx[j] < 0.0f ? 1 : 0) | (sy[j] < 0.0f ? 2 : 0) | (sz[j] < 0.0f ? 4 : 0);
    }
    if (PRE && p.stage_vox > p.stage) {
      if (th.fast) cub_fwd_range<N, WM, true, DPL, PRE, PRE>(p, b, e0, e1, sx, sy, sz, orth, hist, stage, counter, th);
      else cub_fwd_range<N, WM, false, DPL, PRE, PRE>(p, b, e0, e1, sx, sy, sz, orth, hist, stage, counter, th);
    } else {
      if (th.fast) cub_fwd_range<N, WM, true, DPL, PRE, false>(p, b, e0, e1, sx, sy, sz, orth, hist, stage, counter, th);
      else cub_fwd_range<N, WM, false, DPL, PRE, false>(p, b, e0, e1, sx, sy, sz, orth, hist, stage, counter, th);
    }
    end_group<uint32_t>(p, hist, k, b, t, e0 == 0 && e1 == nb, 0);
    pos += e1 - e0;
    if (e1 == nb && t == gpc - 1) ++b;
  }
}

// ---------------------------------------------------------------------------

}  // namespace

template <int N, int WM, int DPL>
static hipError_t launch_cub_fwd_t(const Params& p, int block, size_t lds, hipStream_t s) {
  if (p.cub_rec) {
    if (hipError_t e = set_lds_limit(k_cub_fwd<N, WM, DPL, true>, lds); e != hipSuccess) return e;
    hipLaunchKernelGGL((k_cub_fwd<N, WM, DPL, true>), dim3(p.G), dim3(block), lds, s, p);
  } else {
    if (hipError_t e = set_lds_limit(k_cub_fwd<N, WM, DPL, false>, lds); e != hipSuccess) return e;
    hipLaunchKernelGGL((k_cub_fwd<N, WM, DPL, false>), dim3(p.G), dim3(block), lds, s, p);
  }
  return hipGetLastError();
}

template <int DPL>
static hipError_t launch_cub_fwd_d(const Params& p, int block, size_t lds, hipStream_t s) {
  if (p.n == 2) return p.wmode == WM_ONES ? launch_cub_fwd_t<2, WM_ONES, DPL>(p, block, lds, s)
                                          : launch_cub_fwd_t<2, WM_VMAX, DPL>(p, block, lds, s);
  return p.wmode == WM_ONES ? launch_cub_fwd_t<3, WM_ONES, DPL>(p, block, lds, s)
                            : launch_cub_fwd_t<3, WM_VMAX, DPL>(p, block, lds, s);
}

hipError_t launch_cub_records(const Params& p, hipStream_t s) {
  if (p.total_voxels <= 0 || p.B <= 0) return hipSuccess;
  // blocks per complex for one voxel per thread in a complex of average size
  const int64_t per = std::max<int64_t>(1, (p.total_voxels / p.B + 255) / 256);
  const dim3 grid((unsigned)std::min<int64_t>(per, 65535), (unsigned)std::min(p.B, 65535));
  if (p.n == 2) {
    if (p.wmode == WM_ONES) hipLaunchKernelGGL((k_cub_records<2, WM_ONES>), grid, dim3(256), 0, s, p);
    else hipLaunchKernelGGL((k_cub_records<2, WM_VMAX>), grid, dim3(256), 0, s, p);
  } else {
    if (p.wmode == WM_ONES) hipLaunchKernelGGL((k_cub_records<3, WM_ONES>), grid, dim3(256), 0, s, p);
    else hipLaunchKernelGGL((k_cub_records<3, WM_VMAX>), grid, dim3(256), 0, s, p);
  }
  return hipGetLastError();
}

hipError_t launch_forward_cub(const Params& p, int block, size_t lds, hipStream_t s) {
  return p.dpl == 2 ? launch_cub_fwd_d<2>(p, block, lds, s) : launch_cub_fwd_d<1>(p, block, lds, s);
}

}  // namespace wect
