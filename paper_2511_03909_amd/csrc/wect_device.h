// Device-side helpers shared by the HIP kernels of the library (gfx950).
// Included by every kernel translation unit; everything is in an anonymous
// namespace, so each unit keeps its own copy.
//
//
// Work layout shared by the forward and backward kernels
// ------------------------------------------------------
// One lane of a 64-wide wavefront owns one direction of a 64-direction tile.
// A wavefront walks a list of cells (simplices, or voxels of an image) whose
// data are identical for all of its lanes, so every per-cell load is a
// broadcast and each lane only evaluates its own direction: heights, the
// maximum over the cell's vertices, the threshold index.  The forward adds the
// signed weight to an LDS histogram laid out [threshold index][lane]: the 64
// lanes of one atomic always hit 64 different words in 64 consecutive banks,
// whatever their threshold indices are, so LDS atomics never conflict.
//
// The cells of all complexes of a batch and all direction tiles form one
// stream ordered (complex, direction tile, cell).  A "group" is one
// (complex, direction tile) pair.  Block k of G processes the contiguous
// stream range [k*S/G, (k+1)*S/G) and writes one partial histogram per group
// it touches into slot k + group; a second kernel sums a group's slots and
// scans along the thresholds (the cumulative sum of Algorithm 1).
//
// Numerics: heights are float32 with contraction off, ((x*sx) + (y*sy)) + (z*sz);
// a cell's threshold index is the first stored threshold at or above its
// maximum height (identical to the maximum of its vertices' indices because
// the index is monotone, as in the correctness proof of Algorithm 1).

#pragma once

#include "wect_internal.h"

#include <math.h>

#include <algorithm>

#include <atomic>

#pragma clang fp contract(off)

namespace wect {
namespace {

constexpr int W = kWave;

enum : int { WM_ONES = 0, WM_EXPLICIT = 1, WM_VMAX = 2 };

template <typename A, typename B>
__device__ __forceinline__ A bitcast(B x) {
  static_assert(sizeof(A) == sizeof(B), "size");
  A r;
  __builtin_memcpy(&r, &x, sizeof(A));
  return r;
}

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t mn64(int64_t a, int64_t b) { return a < b ? a : b; }
__device__ __forceinline__ int64_t mx64(int64_t a, int64_t b) { return a > b ? a : b; }

// ---------------------------------------------------------------------------
// heights
// ---------------------------------------------------------------------------

template <int N>
__device__ __forceinline__ float height(const float* c, float sx, float sy, float sz) {
  float h = c[0] * sx;
  if constexpr (N >= 2) h = h + c[1] * sy;
  if constexpr (N >= 3) h = h + c[2] * sz;
  return h;
}

// ---------------------------------------------------------------------------
// threshold index: b = min{ q : thr[q] >= h }, in [0, T]
// ---------------------------------------------------------------------------

struct Thr {
  const float* P;   // LDS [T+1]: P[q] = thr[q-1], P[0] = -inf
  float c, k;       // guess: t = fma(h, c, k) puts thr[q] near q + 1.5
  float ka;         // arithmetic index: t = fma(h, c, ka) puts thr[q] just above q + 1
  float tmax;       // T + 0.5
  float theta;      // arithmetic index exact when frac(t) > theta (see thr_arith)
  int T, p2, fast, arith;
};

// Monotone first guess of the index: an affine map of the height (one fused
// multiply-add), shifted by half a step so that it never falls below the true
// index, clamped to [0, T].
__device__ __forceinline__ int guess(float h, float c, float k, int T) {
  float t = __builtin_fmaf(h, c, k);
  t = __builtin_amdgcn_fmed3f(t, 0.0f, (float)T);
  return (int)t;
}

// Near-threshold fix of the arithmetic index and of the guess: b is the
// candidate m (in [0, T]); P[m] = thr[m-1] decides between m-1 and m.
__device__ __forceinline__ int thr_near(float h, int b, const Thr& th) { return b - (h <= th.P[b] ? 1 : 0); }

__device__ __forceinline__ float next_up(float x) {
  if (!(x == x) || x == INFINITY) return x;
  if (x == 0.0f) return __int_as_float(1);
  int i = __float_as_int(x);
  return __int_as_float(x > 0.0f ? i + 1 : i - 1);
}

// Exact index L(h) = #{q : thr[q] < h}.  Fast path: the guess g is L or L+1
// for every float (checked against the stored thresholds when the block
// starts), and g == L+1 exactly when h <= thr[g-1], so one comparison settles
// it.  Otherwise a branch-free binary search over the stored thresholds.
template <bool FAST>
__device__ __forceinline__ int thr_index(float h, const Thr& th) {
  if constexpr (FAST) {
    return thr_near(h, guess(h, th.c, th.k, th.T), th);
  }
  int lo = 0;
  for (int s = th.p2; s > 0; s >>= 1) {
    int cand = lo + s;
    if (cand <= th.T && th.P[cand] < h) lo = cand;  // P[cand] == thr[cand-1]
  }
  return lo;
}

// Index from the affine map alone.  With x(h) = h c + ka (exact, strictly
// increasing) and tau_q = x(thr[q]), L(h) = #{q : tau_q < x(h)}.  The block
// prologue picks ka so that every tau_q lies in [q+1+rmin, q+1+rmax] with
// rmin >= eps, where eps = 2^-24 (T+2) bounds the rounding of t = fl(x(h)).
// Write t = m + u (m = floor t, 0 <= u < 1).  Every tau_q with q+1 >= m+1 is
// then >= m+1+eps > x(h), and when u > theta = rmax + eps every tau_q with
// q+1 <= m is <= m+rmax < x(h): L = clamp(m, 0, T), one truncation.  Otherwise
// x(h) is within rmax+2 eps of m and only tau_{m-1} can be on either side:
// L = m - [h <= thr[m-1]] (thr_near).  Clamping t to [-0.5, T+0.5] keeps both
// ends exact: u = 0.5 there and the truncation gives 0 and T.
__device__ __forceinline__ bool thr_arith(float h, const Thr& th, int& b) {
  float t = __builtin_fmaf(h, th.c, th.ka);
  t = __builtin_amdgcn_fmed3f(t, -0.5f, th.tmax);
  b = (int)t;
  return __builtin_amdgcn_fractf(t) > th.theta;
}

// Minimum over the block (every thread gets it); red holds 16 doubles.
__device__ __forceinline__ double block_min(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  v = INFINITY;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v = fmin(v, red[w]);
  return v;
}

// Block prologue: stage P in LDS and decide whether the fast path is exact
// for this threshold array.  g is monotone in h and L is constant on
// (thr[q], thr[q+1]], so g(thr[q]) in {q, q+1} and g(next float above thr[q])
// in {q+1, q+2} (clamped to T) for every q give g in {L, L+1} everywhere
// (strictly increasing thresholds required).
__device__ __forceinline__ void setup_thresholds(const float* thr, int T, float* P, Thr& th) {
  for (int q = threadIdx.x; q <= T; q += blockDim.x) P[q] = q > 0 ? thr[q - 1] : -INFINITY;
  int p2 = 1;
  while (p2 * 2 <= T) p2 *= 2;
  float c = 0.0f, k = 0.0f;
  int ok = 0;
  if (T >= 2) {
    const float t0 = thr[0], t1 = thr[T - 1];
    const float delta = (t1 - t0) / (float)(T - 1);
    c = 1.0f / delta;
    k = 1.5f - t0 * c;  // t(thr[q]) ~ q + 1.5
    ok = (delta > 0.0f) && isfinite(c) && isfinite(k) && (c > 0.0f);
  }
  int bad = 0;
  if (ok) {
    for (int q = threadIdx.x; q < T; q += blockDim.x) {
      const float x = thr[q];
      if (q + 1 < T && !(x < thr[q + 1])) bad = 1;
      const int g0 = guess(x, c, k, T);
      const int g1 = guess(next_up(x), c, k, T);
      if (g0 < q || g0 > q + 1 || g1 < min(q + 1, T) || g1 > q + 2) bad = 1;
    }
  }
  bad = __syncthreads_or(bad);
  // arithmetic index: place every tau_q = thr[q] c + ka at or above q + 1 + eps
  // (exact products in double, one rounding of about 2^-53 (T+2))
  __shared__ double s_red[2][16];
  const double eps = ldexp(1.0, -24) * (T + 2) + 1e-9;
  float ka = 0.0f;
  double rmin = 0.0, rmax = 0.0;
  int arith = 0;
  if (ok && !bad) {
    const float ka0 = 1.0f - thr[0] * c;
    double lo = INFINITY;
    for (int q = threadIdx.x; q < T; q += blockDim.x)
      lo = fmin(lo, (double)thr[q] * (double)c + (double)ka0 - (double)(q + 1));
    lo = block_min(lo, s_red[0]);
    // the smallest float ka >= ka0 + (eps - lo) (exact in double, rounded up)
    const double want = (double)ka0 + (eps - lo) + 1e-9;
    ka = (float)want;
    if ((double)ka < want) ka = next_up(ka);
    double a = INFINITY, z = -INFINITY;
    for (int q = threadIdx.x; q < T; q += blockDim.x) {
      const double r = (double)thr[q] * (double)c + (double)ka - (double)(q + 1);
      a = fmin(a, r);
      z = fmax(z, r);
    }
    rmin = block_min(a, s_red[0]);
    rmax = -block_min(-z, s_red[1]);
    arith = rmin >= eps && rmax + eps < 0.25;
  }
  th.P = P;
  th.c = c;
  th.k = k;
  th.ka = ka;
  th.tmax = (float)T + 0.5f;
  th.theta = (float)(rmax + eps) + 0x1p-24f;  // rounded up past rmax + eps
  th.T = T;
  th.p2 = p2;
  th.fast = uniform(ok && !bad);
  th.arith = uniform(th.fast && arith);
  __syncthreads();
}

// ---------------------------------------------------------------------------
// LDS accumulation
// ---------------------------------------------------------------------------

__device__ __forceinline__ void lds_add(uint32_t* a, uint32_t v) {
  __hip_atomic_fetch_add(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add(uint64_t* a, uint64_t v) {
  __hip_atomic_fetch_add(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Adds staged entries to the lane's histogram column col ([T+1] rows of W
// lanes): the pairs (e, e+1) for e = first, first + step, ... below ne, then a
// last single entry.  entry(e, h, w) gives the lane's height and the signed
// weight of entry e.
//
// Per-wavefront choice between the arithmetic index (no LDS read unless a lane
// sits on a threshold) and the one-read guess: images whose pixel lattice is
// commensurate with the threshold grid put many heights exactly on thresholds
// for some directions; a wavefront that needs the near-threshold fix in more
// than a quarter of a run of up to 32 pairs switches to the guess for the rest
// of its range.  The mode lives in *arith (wavefront-uniform).
template <bool FAST, typename ACC, typename Entry>
__device__ __forceinline__ void hist_entries(ACC* col, int first, int step, int ne, const Thr& th, int* arith,
                                             Entry entry) {
  int e = first;
  if constexpr (FAST) {
    while (*arith && e + 1 < ne) {
      const int stop = min(ne - 1, e + 32 * step);
      int fixes = 0, pairs = 0;
      for (; e < stop; e += step) {
        float h0, h1;
        ACC w0, w1;
        entry(e, h0, w0);
        entry(e + 1, h1, w1);
        int b0, b1;
        const bool ok0 = thr_arith(h0, th, b0);
        const bool ok1 = thr_arith(h1, th, b1);
        if (__builtin_amdgcn_ballot_w64(!(ok0 && ok1)) != 0) {
          ++fixes;
          if (!ok0) b0 = thr_near(h0, b0, th);
          if (!ok1) b1 = thr_near(h1, b1, th);
        }
        ++pairs;
        lds_add(&col[b0 * W], w0);
        lds_add(&col[b1 * W], w1);
      }
      if (4 * fixes > pairs) *arith = 0;
    }
  }
  for (; e + 1 < ne; e += step) {
    float h0, h1;
    ACC w0, w1;
    entry(e, h0, w0);
    entry(e + 1, h1, w1);
    const int b0 = thr_index<FAST>(h0, th);
    const int b1 = thr_index<FAST>(h1, th);
    lds_add(&col[b0 * W], w0);
    lds_add(&col[b1 * W], w1);
  }
  if (e < ne) {
    float h0;
    ACC w0;
    entry(e, h0, w0);
    lds_add(&col[thr_index<FAST>(h0, th) * W], w0);
  }
}

// As hist_entries for entries that serve two directions per lane (a tile of
// 128 directions: column `lane` for the first, `lane + 64` for the second,
// rows 128 wide).  entry(e, j, k, h, w) gives the height and weight of entry
// e for the lane's k-th direction; it is called for k = 0 and then k = 1 of one
// entry before the next entry, with j = 0 for the first entry of a pair and
// j = 1 for the second (j = 0 for a lone last entry).  The index mode switch is per wavefront as in
// hist_entries, counted over both directions.
template <bool FAST, typename ACC, typename Entry>
__device__ __forceinline__ void hist_entries2(ACC* col, int first, int step, int ne, const Thr& th, int* arith,
                                              Entry entry) {
  constexpr int RW = 2 * W;
  int e = first;
  if constexpr (FAST) {
    while (*arith && e + 1 < ne) {
      const int stop = min(ne - 1, e + 32 * step);
      int fixes = 0, pairs = 0;
      for (; e < stop; e += step) {
        float h[2][2];
        ACC w[2][2];
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int k = 0; k < 2; ++k) entry(e + j, j, k, h[j][k], w[j][k]);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          int b0, b1;
          const bool ok0 = thr_arith(h[0][k], th, b0);
          const bool ok1 = thr_arith(h[1][k], th, b1);
          if (__builtin_amdgcn_ballot_w64(!(ok0 && ok1)) != 0) {
            ++fixes;
            if (!ok0) b0 = thr_near(h[0][k], b0, th);
            if (!ok1) b1 = thr_near(h[1][k], b1, th);
          }
          ++pairs;
          lds_add(&col[b0 * RW + k * W], w[0][k]);
          lds_add(&col[b1 * RW + k * W], w[1][k]);
        }
      }
      if (4 * fixes > pairs) *arith = 0;
    }
  }
  for (; e + 1 < ne; e += step) {
    float h[2][2];
    ACC w[2][2];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int k = 0; k < 2; ++k) entry(e + j, j, k, h[j][k], w[j][k]);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      lds_add(&col[thr_index<FAST>(h[0][k], th) * RW + k * W], w[0][k]);
      lds_add(&col[thr_index<FAST>(h[1][k], th) * RW + k * W], w[1][k]);
    }
  }
  if (e < ne) {
    float h[2];
    ACC w[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) entry(e, 0, k, h[k], w[k]);
#pragma unroll
    for (int k = 0; k < 2; ++k) lds_add(&col[thr_index<FAST>(h[k], th) * RW + k * W], w[k]);
  }
}

// Logistic sigmoid 1 / (1 + 2^-x) of x = lam (thr - h) log2(e); also returns
// e = 2^-x, from which sig (1 - sig) = e sig^2 follows without cancellation.
__device__ __forceinline__ float sigmoid2(float x, float& e) {
  e = __builtin_amdgcn_exp2f(-x);
  return __builtin_amdgcn_rcpf(1.0f + e);
}

// floor(x + 1/2) as an int32 in one instruction (|x| < 2^31): rounding to
// the nearest integer, halves upwards.
__device__ __forceinline__ int round_half_up(float x) {
  int r;
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

// Relaxation: the entry's signed fixed-point weight C is spread over the
// thresholds.  Inside its window [lo, hi) = {q : |thr[q] - h| <= R} the entry
// contributes F_q = round(C sig(lam (thr[q] - h))) at threshold q (nearest
// integer, halves upwards), and from hi
// on all of C.  The histogram holds differences (F_lo at lo, F_q - F_{q-1} at
// q, C - F_{hi-1} at hi), so the threshold scan that follows returns exactly
// these values.  |C| < 2^30, so every F_q and difference fits in int32.
template <bool FAST>
__device__ __forceinline__ void smooth_add(uint64_t* col, float h, uint64_t C, const Thr& th, float R, float kap) {
  const int lo = thr_index<FAST>(h - R, th);
  const int hi = thr_index<FAST>(next_up(h + R), th);
  const float cf = (float)(int32_t)(uint32_t)C;
  auto term = [&](int q) {
    float ex;
    return round_half_up(cf * sigmoid2((th.P[q + 1] - h) * kap, ex));
  };
  // two terms per iteration: half the loop control, and no register copy
  int prev = 0, q = lo;
  for (; q + 1 < hi; q += 2) {
    const int F0 = term(q), F1 = term(q + 1);
    lds_add(&col[q * W], (uint64_t)(int64_t)(F0 - prev));
    lds_add(&col[(q + 1) * W], (uint64_t)(int64_t)(F1 - F0));
    prev = F1;
  }
  if (q < hi) {
    const int F = term(q);
    lds_add(&col[q * W], (uint64_t)(int64_t)(F - prev));
    prev = F;
  }
  lds_add(&col[hi * W], C - (uint64_t)(int64_t)prev);
}

template <bool FAST, typename Entry>
__device__ __forceinline__ void smooth_entries(uint64_t* col, int first, int step, int ne, const Thr& th, float R,
                                               float kap, Entry entry) {
  for (int e = first; e < ne; e += step) {
    float h;
    uint64_t C;
    entry(e, h, C);
    smooth_add<FAST>(col, h, C, th, R, kap);
  }
}

// Sum over the 64 lanes of a wavefront: rotate-and-add inside each row of 16
// lanes (DPP row_ror), then add the four row sums.
__device__ __forceinline__ float wave_sum(float v) {
  v += bitcast<float>(__builtin_amdgcn_update_dpp(0, bitcast<int>(v), 0x128, 0xf, 0xf, false));
  v += bitcast<float>(__builtin_amdgcn_update_dpp(0, bitcast<int>(v), 0x124, 0xf, 0xf, false));
  v += bitcast<float>(__builtin_amdgcn_update_dpp(0, bitcast<int>(v), 0x122, 0xf, 0xf, false));
  v += bitcast<float>(__builtin_amdgcn_update_dpp(0, bitcast<int>(v), 0x121, 0xf, 0xf, false));
  float r0 = bitcast<float>(__builtin_amdgcn_readlane(bitcast<int>(v), 0));
  float r1 = bitcast<float>(__builtin_amdgcn_readlane(bitcast<int>(v), 16));
  float r2 = bitcast<float>(__builtin_amdgcn_readlane(bitcast<int>(v), 32));
  float r3 = bitcast<float>(__builtin_amdgcn_readlane(bitcast<int>(v), 48));
  return (r0 + r1) + (r2 + r3);
}

// Sums over the 64 lanes of 8 values at once: on return, every lane l holds
// the total of v[l & 7] over all 64 lanes.  Within each group of 8 lanes a
// butterfly halves the values per lane at each step (partners: half mirror
// 7 - l, then the quad swaps l ^ 2 and l ^ 1, which split on lane bits 2, 1,
// 0), so lane l ends with its group's sum of v[l & 7]; exchanges at lane
// distances 8, 16 and 32 add the eight group sums.  About 4 instructions per
// value, against about 11 for a wave_sum of each.
__device__ __forceinline__ float sum_scatter8(const float (&v)[8]) {
  const int lane = threadIdx.x & (W - 1);
  const bool b2 = lane & 4, b1 = lane & 2, b0 = lane & 1;
  auto hmirror = [](float x) {  // row_half_mirror
    return bitcast<float>(__builtin_amdgcn_update_dpp(0, bitcast<int>(x), 0x141, 0xf, 0xf, false));
  };
  auto swap2 = [](float x) {  // quad_perm [2,3,0,1]
    return bitcast<float>(__builtin_amdgcn_update_dpp(0, bitcast<int>(x), 0x4e, 0xf, 0xf, false));
  };
  auto swap1 = [](float x) {  // quad_perm [1,0,3,2]
    return bitcast<float>(__builtin_amdgcn_update_dpp(0, bitcast<int>(x), 0xb1, 0xf, 0xf, false));
  };
  auto ror8 = [](float x) {  // row_ror:8, partner l ^ 8 within a row of 16
    return bitcast<float>(__builtin_amdgcn_update_dpp(0, bitcast<int>(x), 0x128, 0xf, 0xf, false));
  };
  float c[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float keep = b2 ? v[k + 4] : v[k], send = b2 ? v[k] : v[k + 4];
    c[k] = keep + hmirror(send);
  }
  float d[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const float keep = b1 ? c[k + 2] : c[k], send = b1 ? c[k] : c[k + 2];
    d[k] = keep + swap2(send);
  }
  const float keep = b0 ? d[1] : d[0], send = b0 ? d[0] : d[1];
  float r = keep + swap1(send);
  r += ror8(r);
  r += __shfl_xor(r, 16);
  r += __shfl_xor(r, 32);
  return r;
}

// ---------------------------------------------------------------------------
// stream bookkeeping
// ---------------------------------------------------------------------------

// Number of stream elements (cells handled one by one) of the complexes
// before complex b: all simplices of all dimensions, or all voxels.
__device__ __forceinline__ int64_t cum_elems(const Params& p, int b) {
  if (p.ls) {  // vertex-centric kernels: one stream element per vertex
    if (!p.vert_off) return b == 0 ? 0 : p.count[0];
    return p.vert_off[b];
  }
  if (p.kind == 1) {
    if (p.grid_off) return p.grid_off[b];
    return b == 0 ? 0 : p.total_voxels;
  }
  if (p.B == 1 && !p.vert_off) {
    if (b == 0) return 0;
    int64_t s = 0;
    for (int i = 0; i <= p.top_dim; ++i) s += p.count[i];
    return s;
  }
  int64_t s = p.vert_off[b];
  for (int i = 1; i <= p.top_dim; ++i) s += p.simp_off[i][b];
  return s;
}

__device__ __forceinline__ int64_t off_or(const int64_t* off, int b, int64_t dflt) {
  return off ? off[b] : (b == 0 ? 0 : dflt);
}

// Largest b in [0, B) with groups_per_complex * cum_elems(b) <= pos.
__device__ __forceinline__ int find_complex(const Params& p, int64_t pos, int gpc) {
  int lo = 0, hi = p.B - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if ((int64_t)gpc * cum_elems(p, mid) <= pos) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int64_t block_start(int64_t k, int64_t S, int64_t G) { return (k * S) / G; }

// ---------------------------------------------------------------------------
// simplicial staging: one thread gathers one simplex into registers
// ---------------------------------------------------------------------------

// Forward accumulator: unit and int32 weights accumulate in uint32 (two's
// complement, wraps exactly like int32); float32 weights are converted to
// signed 64-bit fixed point (see fixed_exp) and accumulate in uint64.  Integer
// LDS atomics run one lane per bank per pass, float ones do not, and integer
// sums do not depend on the order of the additions.
template <typename WT>
struct AccOf {
  using T = uint32_t;
};
template <>
struct AccOf<float> {
  using T = uint64_t;
};

// N = 0 is the WECF of a general vertex filter: a staged vertex is then its
// global row in fvals (one word) instead of its N coordinates.
template <int N, int DIM, typename ACC>
struct SimpLayout {
  static constexpr int NV = DIM + 1;
  static constexpr int NC = N == 0 ? 1 : N;                   // words per staged vertex
  static constexpr int WW = sizeof(ACC) / 4;                 // words of the staged weight
  static constexpr int WOFF = ((NV * NC + WW - 1) / WW) * WW;  // weight slot, aligned to its size
  static constexpr int OOFF = WOFF + WW;                     // owner slot (vertex-max backward)
  static constexpr int STRIDE = ((OOFF + 1 + 3) / 4) * 4;
  static_assert(STRIDE <= kMaxStride, "entry too large");
};

// Exponent e of the fixed-point scale 2^e for float32 weights: with M the
// largest |w| and C the number of cells, every sum of rounded weights stays
// below C * (M 2^e + 1/2) < 2^63.  Computed identically by every block from
// the per-block maxima written by k_absmax.
//
// The sigmoid relaxation also rounds every term w sig to this scale in int32
// arithmetic, so there the scale is capped further to keep M 2^e < 2^30 (unit
// weights: M = 1).
__device__ __forceinline__ int fixed_exp(const Params& p) {
  float M = 0.0f;
  if (p.smooth && p.wmode == WM_ONES) M = 1.0f;
  for (int i = 0; i < p.nabsmax; ++i) M = fmaxf(M, p.absmax[i]);
  const double X = (double)M * p.cells_total;
  if (!(X > 0.0) || !isfinite(X)) return 0;
  int ex = 0;
  (void)frexp(X, &ex);  // X = f 2^ex, f in [0.5, 1): floor(log2 X) = ex - 1
  int e = 61 - (ex - 1);
  if (p.smooth) {
    // vertex-centric kernels combine a vertex's weight with those of its
    // cofaces: at most (1 + largest degree) M
    const double Mc = p.ls ? (double)M * (double)(1 + p.ls_hdr[1]) : (double)M;
    int em = 0;
    (void)frexp(Mc, &em);  // Mc < 2^em
    e = min(e, 30 - em);
  }
  return e;
}

__device__ __forceinline__ uint64_t to_fixed(float w, int e) {
  return (uint64_t)(int64_t)rint(ldexp((double)w, e));
}

template <int N, int DIM, int WM, typename WT, bool FWD>
struct SimpStager {
  using ACC = typename AccOf<WT>::T;
  using L = SimpLayout<N, DIM, ACC>;
  float e[L::OOFF + 1];
  int idx[L::NV];

  // vertex ids (local to the complex) of simplex `row` (global row index)
  __device__ __forceinline__ void load_idx(const Params& p, int64_t row, int64_t lrow) {
    if constexpr (DIM == 0) {
      idx[0] = (int)lrow;
    } else {
      const int32_t* s = p.simp[DIM] + row * L::NV;
#pragma unroll
      for (int j = 0; j < L::NV; ++j) idx[j] = s[j];
    }
  }
  __device__ __forceinline__ void put_weight(ACC a) {
    if constexpr (DIM & 1) a = ACC(0) - a;  // (-1)^dim: the forward stages signed weights
    if constexpr (sizeof(ACC) == 4) {
      e[L::WOFF] = bitcast<float>(a);
    } else {
      e[L::WOFF] = bitcast<float>((uint32_t)a);
      e[L::WOFF + 1] = bitcast<float>((uint32_t)(a >> 32));
    }
  }
  // coordinates (or filter rows), signed weight and owner vertex of the simplex whose ids are in idx
  __device__ __forceinline__ void gather(const Params& p, int64_t row, int64_t voff, int fexp) {
#pragma unroll
    for (int j = 0; j < L::NV; ++j) {
      if constexpr (N == 0) {
        e[j] = bitcast<float>((int32_t)(voff + idx[j]));  // global vertex row (< 2^31)
      } else {
        const float* c = p.coords + (voff + idx[j]) * N;
#pragma unroll
        for (int k = 0; k < N; ++k) e[j * N + k] = c[k];
      }
    }
#pragma unroll
    for (int k = L::NV * L::NC; k < L::WOFF; ++k) e[k] = 0.0f;
    e[L::OOFF] = 0.0f;
    if constexpr (WM == WM_ONES) {
      if constexpr (FWD) {
        if constexpr (sizeof(ACC) == 8) put_weight(to_fixed(1.0f, fexp));  // relaxation: fixed point
        else put_weight(ACC(1));
      }
    } else if constexpr (WM == WM_EXPLICIT) {
      if constexpr (FWD) {
        const WT w = ((const WT*)p.weights[DIM])[row];
        if constexpr (sizeof(ACC) == 4) put_weight(bitcast<ACC>(w));
        else put_weight(to_fixed(w, fexp));
      }
    } else {
      const float* w = (const float*)p.weights[0];
      float best = w[voff + idx[0]];
      int own = idx[0];
#pragma unroll
      for (int j = 1; j < L::NV; ++j) {
        float x = w[voff + idx[j]];
        if (x > best || (x == best && idx[j] < own)) { best = x; own = idx[j]; }
      }
      if constexpr (FWD) put_weight(to_fixed(best, fexp));
      e[L::OOFF] = bitcast<float>(own);
    }
  }
  __device__ __forceinline__ void store(float* dst) const {
#pragma unroll
    for (int k = 0; k <= L::OOFF; ++k) dst[k] = e[k];
  }
};

template <typename ACC>
__device__ __forceinline__ ACC load_weight(const float* E) {
  if constexpr (sizeof(ACC) == 4) return bitcast<ACC>(E[0]);
  else return *(const uint64_t*)E;
}

// Maximum height of a staged simplex for the lane's direction.
template <int N, int DIM>
__device__ __forceinline__ float max_height(const float* E, float sx, float sy, float sz) {
  float h = height<N>(E, sx, sy, sz);
#pragma unroll
  for (int j = 1; j <= DIM; ++j) h = fmaxf(h, height<N>(E + j * N, sx, sy, sz));
  return h;
}

// Histogram rows are W * p.dpl columns wide (p.dpl directions per lane).
template <typename ACC>
__device__ void flush_hist(const Params& p, ACC* hist, int64_t slot) {
  __syncthreads();
  const int T = p.T, RW = W * p.dpl;
  ACC* dst = (ACC*)p.partial + slot * (int64_t)T * RW;
  for (int i = threadIdx.x; i < T * RW; i += blockDim.x) dst[i] = hist[i];
  __syncthreads();
  for (int i = threadIdx.x; i < (T + 1) * RW; i += blockDim.x) hist[i] = ACC(0);
  __syncthreads();
}

template <typename ACC>
struct OutOf;
template <>
struct OutOf<uint32_t> {
  using T = uint32_t;  // int32 bit pattern
  __device__ static uint32_t conv(uint32_t x, int) { return x; }
};
template <>
struct OutOf<uint64_t> {
  using T = float;
  __device__ static float conv(uint64_t x, int fexp) { return (float)ldexp((double)(int64_t)x, -fexp); }
};

// A block that covered a whole group (complex b, direction tile t) writes its
// output itself: out[b][t*64 + lane][q] = sum_{j <= q} hist[j][lane] (row
// stride p.ldo, so that a launch over one tile of the thresholds writes its
// columns of the full output) (the
// cumulative sum of Algorithm 1), then clears hist.  The scan runs in place:
// wavefront r takes rows [r c, (r+1) c) and turns them into a running sum, so
// the last row of each chunk holds the chunk total that later chunks add.
template <typename ACC>
__device__ void finish_group(const Params& p, ACC* hist, int b, int t, int fexp) {
  using O = OutOf<ACC>;
  using OT = typename O::T;
  __syncthreads();
  const int T = p.T, RW = W * p.dpl;
  const int lane = threadIdx.x & (W - 1), r = threadIdx.x >> 6, R = blockDim.x >> 6;
  const int chunk = ((T + R - 1) / R + 3) & ~3;  // a multiple of 4 rows
  const int q0 = min(T, r * chunk), q1 = min(T, q0 + chunk);
  for (int c = lane; c < RW; c += W) {
    ACC run = 0;
    for (int q = q0; q < q1; ++q) {
      run += hist[q * RW + c];
      hist[q * RW + c] = run;
    }
  }
  __syncthreads();
  for (int c = lane; c < RW; c += W) {
    ACC off = 0;
    for (int rr = 0; rr < r; ++rr) {
      const int e = min(T, (rr + 1) * chunk);
      if (e > rr * chunk) off += hist[(e - 1) * RW + c];
    }
    const int dir = t * RW + c;
    if (dir < p.d && q0 < q1) {
      OT* o = (OT*)p.out + ((int64_t)b * p.d + dir) * p.ldo;
      if ((T & 3) == 0 && (p.ldo & 3) == 0 && (reinterpret_cast<uintptr_t>(p.out) & 15) == 0) {
        // rows start 16-byte aligned and q0 is a multiple of 4
        for (int q = q0; q < q1; q += 4) {
          OT v[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) v[j] = O::conv(hist[(q + j) * RW + c] + off, fexp);
          *(uint4*)(o + q) = *(const uint4*)v;
        }
      } else {
        for (int q = q0; q < q1; ++q) o[q] = O::conv(hist[q * RW + c] + off, fexp);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < (T + 1) * RW; i += blockDim.x) hist[i] = ACC(0);
  __syncthreads();
}

// End of a block's share of group (b, t): the whole group gives the output
// directly, part of it a partial histogram in slot k + group.
template <typename ACC>
__device__ __forceinline__ void end_group(const Params& p, ACC* hist, int k, int b, int t, bool whole, int fexp) {
  if (whole) finish_group<ACC>(p, hist, b, t, fexp);
  else flush_hist<ACC>(p, hist, (int64_t)k + (int64_t)b * p.ntiles + t);
}

// Stream range [pos, end) of block k and the complex it starts in.  Group
// mode: exactly group k (an empty group writes its zero output here).
template <typename ACC>
__device__ __forceinline__ bool block_range(const Params& p, ACC* hist, int k, int fexp, int64_t& pos, int64_t& end,
                                            int& b) {
  const int gpc = p.ntiles;
  if (p.group_mode) {
    b = k / gpc;
    const int t = k - b * gpc;
    const int64_t cb = cum_elems(p, b);
    const int64_t nb = cum_elems(p, b + 1) - cb;
    pos = (int64_t)gpc * cb + (int64_t)t * nb;
    end = pos + nb;
    if (nb == 0) {
      finish_group<ACC>(p, hist, b, t, fexp);
      return false;
    }
    return true;
  }
  pos = block_start(k, p.S, p.G);
  end = block_start(k + 1, p.S, p.G);
  if (pos >= end) return false;
  b = find_complex(p, pos, gpc);
  return true;
}

// The lane's direction.  The empty asm statement reads the three components,
// so the compiler waits for their loads here, once per group: otherwise it may
// place that wait inside the histogram loop, where it would also wait for the
// loads of the next staging tile that are meant to be in flight.
__device__ __forceinline__ void load_dir(const Params& p, int gp, float& sx, float& sy, float& sz) {
  sx = sy = sz = 0.0f;
  if (gp < p.d) {
    const float* s = p.dirs + (int64_t)gp * p.n;
    sx = s[0];
    if (p.n >= 2) sy = s[1];
    if (p.n >= 3) sz = s[2];
  }
  asm volatile("" ::"v"(sx), "v"(sy), "v"(sz));
}

__device__ __forceinline__ size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }



// Opt each kernel in to the full LDS of a workgroup once per process (the
// attribute is per function); later launches, including captured ones, only
// enqueue.
template <typename K>
hipError_t set_lds_limit(K kernel, size_t bytes) {
  static std::atomic<size_t> granted{64 * 1024};
  if (bytes <= granted.load(std::memory_order_acquire)) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) granted.store(bytes, std::memory_order_release);
  return e;
}


}  // namespace
}  // namespace wect
