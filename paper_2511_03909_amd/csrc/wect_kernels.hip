// HIP kernels (gfx950) for the weighted Euler characteristic transform.
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

// Histogram of staged simplices for a general vertex filter (n = 0).  The
// threshold index of every filter value was computed by k_vertex_buckets
// (Algorithm 1 indexes the vertex filter values first); since the index is
// monotone, a simplex's index is the largest of its vertices' indices.  The
// 64 lanes read 64 consecutive indices of a vertex row.  Global-memory latency
// dominates, so a wavefront gathers the indices of K pairs of entries before
// it adds any of them (out-of-range pairs re-read a valid one: always in bounds).
template <int DIM, typename VB, typename ACC, typename L>
__device__ __forceinline__ void filter_hist(ACC* col, const float* stage, int first, int step, int ne,
                                            const VB* vb, int m, int fcol) {
  constexpr int NV = DIM + 1;
  constexpr int K = 8;
  auto rowb = [&](const float* E, int j) { return (int)vb[(int64_t)bitcast<int32_t>(E[j]) * m + fcol]; };
  int e = first;
  for (; e + 1 < ne; e += K * step) {
    int x[K][2][NV];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int ek = e + k * step;
      const float* E = stage + (ek + 1 < ne ? ek : e) * L::STRIDE;
#pragma unroll
      for (int j = 0; j < NV; ++j) {
        x[k][0][j] = rowb(E, j);
        x[k][1][j] = rowb(E + L::STRIDE, j);
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int ek = e + k * step;
      if (ek + 1 < ne) {
        int b0 = x[k][0][0], b1 = x[k][1][0];
#pragma unroll
        for (int j = 1; j < NV; ++j) {
          b0 = max(b0, x[k][0][j]);
          b1 = max(b1, x[k][1][j]);
        }
        const float* E = stage + ek * L::STRIDE;
        lds_add(&col[b0 * W], load_weight<ACC>(E + L::WOFF));
        lds_add(&col[b1 * W], load_weight<ACC>(E + L::STRIDE + L::WOFF));
      }
    }
  }
  // pair starts are first + k step with first + k step + 1 < ne; the next start
  // after them holds a last single entry when it is below ne
  const int npairs = first + 1 < ne ? (ne - 2 - first) / step + 1 : 0;
  e = first + npairs * step;
  if (e < ne) {
    const float* E0 = stage + e * L::STRIDE;
    int c0 = 0;
#pragma unroll
    for (int j = 0; j < NV; ++j) c0 = max(c0, rowb(E0, j));
    lds_add(&col[c0 * W], load_weight<ACC>(E0 + L::WOFF));
  }
}

// Forward over the simplices [lo, hi) (local numbering) of dimension DIM of
// one complex: stage TS simplices at a time, then every wavefront adds its
// share of them to the LDS histogram.  Indices are prefetched one tile ahead
// of the coordinate gather, which runs one tile ahead of the histogram.
template <int N, int DIM, int WM, typename WT, bool FAST, bool SM>
__device__ void simp_fwd_range(const Params& p, int64_t lo, int64_t hi, int64_t voff, int64_t soff,
                               float sx, float sy, float sz, int fcol, typename AccOf<WT>::T* hist, float* stage,
                               const Thr& th, int fexp) {
  using ACC = typename AccOf<WT>::T;
  using L = SimpLayout<N, DIM, ACC>;
  using ST = SimpStager<N, DIM, WM, WT, true>;
  const int tid = threadIdx.x, lane = tid & (W - 1);
  const int wave = uniform(tid >> 6), nw = blockDim.x >> 6;
  const int TS = p.stage;
  const int64_t ntile = (hi - lo + TS - 1) / TS;
  ST st;
  auto tile_row = [&](int64_t t) { return lo + t * TS + tid; };
  // prologue: ids of tile 0, gather tile 0, ids of tile 1
  if (tid < TS && tile_row(0) < hi) {
    st.load_idx(p, soff + tile_row(0), tile_row(0));
    st.gather(p, soff + tile_row(0), voff, fexp);
  }
  int nidx[L::NV];
  int arith = th.arith;
  bool have_next = ntile > 1 && tid < TS && tile_row(1) < hi;
  if (have_next) {
    ST tmp;
    tmp.load_idx(p, soff + tile_row(1), tile_row(1));
#pragma unroll
    for (int j = 0; j < L::NV; ++j) nidx[j] = tmp.idx[j];
  }
  for (int64_t t = 0; t < ntile; ++t) {
    const int cnt = (int)mn64(TS, hi - (lo + t * TS));
    __syncthreads();
    if (tid < cnt) st.store(stage + tid * L::STRIDE);
    __syncthreads();
    // gather tile t+1 (ids loaded last iteration), load ids of tile t+2
    if (have_next) {
#pragma unroll
      for (int j = 0; j < L::NV; ++j) st.idx[j] = nidx[j];
      st.gather(p, soff + tile_row(t + 1), voff, fexp);
    }
    have_next = (t + 2 < ntile) && tid < TS && tile_row(t + 2) < hi;
    if (have_next) {
      ST tmp;
      tmp.load_idx(p, soff + tile_row(t + 2), tile_row(t + 2));
#pragma unroll
      for (int j = 0; j < L::NV; ++j) nidx[j] = tmp.idx[j];
    }
    // histogram of tile t: each wavefront takes adjacent pairs of entries
    // (relaxation: every nw-th entry, each spread over its window)
    if constexpr (SM) {
      static_assert(sizeof(ACC) == 8 && N > 0, "relaxation: fixed-point weights and coordinates");
      smooth_entries<FAST>(hist + lane, wave, nw, cnt, th, p.sm_r, p.sm_k, [&](int e, float& h, uint64_t& C) {
        const float* E = stage + e * L::STRIDE;
        h = max_height<N, DIM>(E, sx, sy, sz);
        C = load_weight<ACC>(E + L::WOFF);
      });
    } else if constexpr (N == 0) {
      if (p.vb_bytes == 1)
        filter_hist<DIM, uint8_t, ACC, L>(hist + lane, stage, 2 * wave, 2 * nw, cnt, (const uint8_t*)p.vbuckets, p.d,
                                          fcol);
      else
        filter_hist<DIM, uint16_t, ACC, L>(hist + lane, stage, 2 * wave, 2 * nw, cnt, (const uint16_t*)p.vbuckets,
                                           p.d, fcol);
    } else {
      hist_entries<FAST, ACC>(hist + lane, 2 * wave, 2 * nw, cnt, th, &arith,
                              [&](int e, float& h, ACC& w) {
                                const float* E = stage + e * L::STRIDE;
                                h = max_height<N, DIM>(E, sx, sy, sz);
                                w = load_weight<ACC>(E + L::WOFF);
                              });
    }
  }
  __syncthreads();
}

template <int N, int WM, typename WT, bool FAST, bool SM>
__device__ __forceinline__ void simp_fwd_dim(int dim, const Params& p, int64_t lo, int64_t hi, int64_t voff,
                                             int64_t soff, float sx, float sy, float sz, int fcol,
                                             typename AccOf<WT>::T* hist, float* stage, const Thr& th, int fexp) {
  switch (dim) {
    case 0: simp_fwd_range<N, 0, WM, WT, FAST, SM>(p, lo, hi, voff, soff, sx, sy, sz, fcol, hist, stage, th, fexp); break;
    case 1: simp_fwd_range<N, 1, WM, WT, FAST, SM>(p, lo, hi, voff, soff, sx, sy, sz, fcol, hist, stage, th, fexp); break;
    case 2: simp_fwd_range<N, 2, WM, WT, FAST, SM>(p, lo, hi, voff, soff, sx, sy, sz, fcol, hist, stage, th, fexp); break;
    default: simp_fwd_range<N, 3, WM, WT, FAST, SM>(p, lo, hi, voff, soff, sx, sy, sz, fcol, hist, stage, th, fexp); break;
  }
}

template <typename ACC>
__device__ void flush_hist(const Params& p, ACC* hist, int64_t slot) {
  __syncthreads();
  const int T = p.T;
  ACC* dst = (ACC*)p.partial + slot * (int64_t)T * W;
  for (int i = threadIdx.x; i < T * W; i += blockDim.x) dst[i] = hist[i];
  __syncthreads();
  for (int i = threadIdx.x; i < (T + 1) * W; i += blockDim.x) hist[i] = ACC(0);
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
// output itself: out[b][t*64 + lane][q] = sum_{j <= q} hist[j][lane] (the
// cumulative sum of Algorithm 1), then clears hist.  The scan runs in place:
// wavefront r takes rows [r c, (r+1) c) and turns them into a running sum, so
// the last row of each chunk holds the chunk total that later chunks add.
template <typename ACC>
__device__ void finish_group(const Params& p, ACC* hist, int b, int t, int fexp) {
  using O = OutOf<ACC>;
  using OT = typename O::T;
  __syncthreads();
  const int T = p.T;
  const int lane = threadIdx.x & (W - 1), r = threadIdx.x >> 6, R = blockDim.x >> 6;
  const int chunk = ((T + R - 1) / R + 3) & ~3;  // a multiple of 4 rows
  const int q0 = min(T, r * chunk), q1 = min(T, q0 + chunk);
  ACC run = 0;
  for (int q = q0; q < q1; ++q) {
    run += hist[q * W + lane];
    hist[q * W + lane] = run;
  }
  __syncthreads();
  ACC off = 0;
  for (int rr = 0; rr < r; ++rr) {
    const int e = min(T, (rr + 1) * chunk);
    if (e > rr * chunk) off += hist[(e - 1) * W + lane];
  }
  const int dir = t * W + lane;
  if (dir < p.d && q0 < q1) {
    OT* o = (OT*)p.out + ((int64_t)b * p.d + dir) * T;
    if ((T & 3) == 0 && (reinterpret_cast<uintptr_t>(p.out) & 15) == 0) {
      // rows start 16-byte aligned and q0 is a multiple of 4
      for (int q = q0; q < q1; q += 4) {
        OT v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = O::conv(hist[(q + j) * W + lane] + off, fexp);
        *(uint4*)(o + q) = *(const uint4*)v;
      }
    } else {
      for (int q = q0; q < q1; ++q) o[q] = O::conv(hist[q * W + lane] + off, fexp);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < (T + 1) * W; i += blockDim.x) hist[i] = ACC(0);
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

// ---------------------------------------------------------------------------
// forward, simplicial
// ---------------------------------------------------------------------------

template <int N, int WM, typename WT, bool SM>
__global__ __launch_bounds__(1024) void k_simp_fwd(Params p) {
  using ACC = typename AccOf<WT>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  const int T = p.T;
  ACC* hist = (ACC*)smem;
  float* P = (float*)(smem + (size_t)(T + 1) * W * sizeof(ACC));
  float* stage = (float*)(smem + (size_t)(T + 1) * W * sizeof(ACC) + align_up((size_t)(T + 1) * 4, 16));
  Thr th;
  setup_thresholds(p.thr, T, P, th);
  for (int i = threadIdx.x; i < (T + 1) * W; i += blockDim.x) hist[i] = ACC(0);
  int fexp = 0;
  if constexpr (sizeof(ACC) == 8) fexp = fixed_exp(p);
  __syncthreads();

  const int k = blockIdx.x;
  int64_t pos, end;
  int b;
  if (!block_range<ACC>(p, hist, k, fexp, pos, end, b)) return;
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
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
    // filter column of the lane (N = 0); lanes past the last column read the
    // last one and their histogram column is never written out
    const int fcol = min(t * W + lane, p.d - 1);
    if constexpr (N > 0) load_dir(p, t * W + lane, sx, sy, sz);
    const int64_t voff = off_or(p.vert_off, b, p.count[0]);
    // dimension ranges within the complex's element numbering
    int64_t dlo = 0;
    for (int dim = 0; dim <= p.top_dim; ++dim) {
      int64_t kd = (dim == 0) ? (off_or(p.vert_off, b + 1, p.count[0]) - voff)
                              : (off_or(p.simp_off[dim], b + 1, p.count[dim]) - off_or(p.simp_off[dim], b, p.count[dim]));
      const int64_t dhi = dlo + kd;
      const int64_t lo = mx64(e0, dlo), hi = mn64(e1, dhi);
      if (lo < hi) {
        const int64_t soff = dim == 0 ? voff : off_or(p.simp_off[dim], b, p.count[dim]);
        if (th.fast)
          simp_fwd_dim<N, WM, WT, true, SM>(dim, p, lo - dlo, hi - dlo, voff, soff, sx, sy, sz, fcol, hist, stage,
                                            th, fexp);
        else
          simp_fwd_dim<N, WM, WT, false, SM>(dim, p, lo - dlo, hi - dlo, voff, soff, sx, sy, sz, fcol, hist, stage,
                                             th, fexp);
      }
      dlo = dhi;
    }
    end_group<ACC>(p, hist, k, b, t, e0 == 0 && e1 == nb, fexp);
    pos += e1 - e0;
    if (e1 == nb && t == gpc - 1) ++b;
  }
}

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

template <int N>
struct CubLayout {
  static constexpr int NO = 1 << N;                 // orthants
  static constexpr int COFF = N == 2 ? 2 : 4;       // first combined weight
  static constexpr int STRIDE = N == 2 ? 8 : 12;
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

// Forward over the voxels [lo, hi) of complex b for one direction tile: the
// neighbourhoods of tile t+1 are loaded while the histogram of tile t runs.
template <int N, int WM, bool FAST>
__device__ void cub_fwd_range(const Params& p, int b, int64_t lo, int64_t hi, float sx, float sy, float sz,
                              int orth, uint32_t* hist, float* stage, int* counter, const Thr& th) {
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
  // grid position of the thread's voxel lo + tid, advanced by TS voxels per
  // tile without division (voxel counts of one complex are below 2^31)
  const uint32_t ts = (uint32_t)TS;
  const uint32_t s0 = ts % (uint32_t)n0, s1 = (ts / (uint32_t)n0) % (uint32_t)n1;
  const uint32_t s2 = ts / ((uint32_t)n0 * (uint32_t)n1);
  uint32_t v = (uint32_t)(lo + tid);
  int i0 = (int)(v % (uint32_t)n0), i1 = (int)((v / (uint32_t)n0) % (uint32_t)n1);
  int i2 = (int)(v / ((uint32_t)n0 * (uint32_t)n1));
  CubFetch<N> f;
  f.load(vol, ax0, ax1, ax2, n0, n1, n2, i0, i1, i2, v < (uint32_t)hi && tid < TS);
  for (int64_t t0 = lo; t0 < hi; t0 += TS) {
    if (tid == 0) *counter = 0;
    __syncthreads();
    bool keep = false;
    int32_t cw[L::NO];
    if (f.valid && f.nb[(CubFetch<N>::M - 1) / 2] > p.include_above) {
      cub_weights<N, WM>(f, p.include_above, cw);
      bool nz = false;
#pragma unroll
      for (int o = 0; o < L::NO; ++o) nz = nz || (cw[o] != 0);
      keep = nz;
    }
    // compact the contributing vertices
    const uint64_t bal = __ballot(keep);
    int base = 0;
    if (lane == 0 && bal) base = atomicAdd(counter, __popcll(bal));
    base = __shfl(base, 0);
    if (keep) {
      const int slot = base + __popcll(bal & ((1ull << lane) - 1ull));
      float* E = stage + slot * L::STRIDE;
      E[0] = f.cx;
      E[1] = f.cy;
      if constexpr (N == 3) { E[2] = f.cz; E[3] = 0.0f; }
#pragma unroll
      for (int o = 0; o < L::NO; ++o) E[L::COFF + o] = bitcast<float>(cw[o]);
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
    f.load(vol, ax0, ax1, ax2, n0, n1, n2, i0, i1, i2, v < (uint32_t)hi && tid < TS);
    __syncthreads();
    const int ne = uniform(*counter);
    const float* Wl = stage + L::COFF + orth;  // the lane's combined weight within an entry
    hist_entries<FAST, uint32_t>(hist + lane, 2 * wave, 2 * nw, ne, th, &arith,
                                 [&](int e, float& h, uint32_t& w) {
                                   h = height<N>(stage + e * L::STRIDE, sx, sy, sz);
                                   w = bitcast<uint32_t>(Wl[e * L::STRIDE]);
                                 });
    __syncthreads();
  }
}

template <int N, int WM>
__global__ __launch_bounds__(1024) void k_cub_fwd(Params p) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int T = p.T;
  uint32_t* hist = (uint32_t*)smem;
  size_t off = (size_t)(T + 1) * W * 4;
  float* P = (float*)(smem + off);
  off += align_up((size_t)(T + 1) * 4, 16);
  int* counter = (int*)(smem + off);
  off += 16;
  float* stage = (float*)(smem + off);
  Thr th;
  setup_thresholds(p.thr, T, P, th);
  for (int i = threadIdx.x; i < (T + 1) * W; i += blockDim.x) hist[i] = 0u;
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
    float sx, sy, sz;
    load_dir(p, t * W + lane, sx, sy, sz);
    const int orth = (sx < 0.0f ? 1 : 0) | (sy < 0.0f ? 2 : 0) | (sz < 0.0f ? 4 : 0);
    if (th.fast) cub_fwd_range<N, WM, true>(p, b, e0, e1, sx, sy, sz, orth, hist, stage, counter, th);
    else cub_fwd_range<N, WM, false>(p, b, e0, e1, sx, sy, sz, orth, hist, stage, counter, th);
    end_group<uint32_t>(p, hist, k, b, t, e0 == 0 && e1 == nb, 0);
    pos += e1 - e0;
    if (e1 == nb && t == gpc - 1) ++b;
  }
}

// ---------------------------------------------------------------------------
// reduce the partial histograms of a group and scan along the thresholds
// (cumulative sum of Algorithm 1): out[b][p][q] = sum_{j <= q} D[p][j]
// ---------------------------------------------------------------------------

// Slots of the partial buffer written for group g = (complex b, tile t): the
// blocks whose stream range meets the group's range [gs, ge) are kfirst..klast
// (block k covers [k S / G, (k+1) S / G)), and block k wrote slot k + g.
__device__ __forceinline__ void group_slots(const Params& p, int g, int64_t& kfirst, int64_t& klast) {
  const int gpc = p.ntiles;
  const int b = g / gpc, t = g % gpc;
  const int64_t cb = cum_elems(p, b);
  const int64_t nb = cum_elems(p, b + 1) - cb;
  kfirst = 0;
  klast = -1;
  if (nb > 0 && p.S > 0) {
    const int64_t gs = (int64_t)gpc * cb + (int64_t)t * nb;
    const int64_t ge = gs + nb;
    kfirst = ((gs + 1) * p.G - 1) / p.S;
    klast = (ge * p.G - 1) / p.S;
  }
}

// Groups with at most this many partial slots are summed inside the scan
// kernel; larger ones are summed first by k_slot_sum (fully parallel).
constexpr int kFusedSlots = 16;

// Sum of the partial histograms of every group with more than kFusedSlots
// slots into dsum[g][T][64]: one thread per (group, threshold, lane).
template <typename ACC>
__global__ __launch_bounds__(256) void k_slot_sum(Params p) {
  const int g = blockIdx.x;
  const int q = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & (W - 1);
  const int T = p.T;
  if (q >= T) return;
  int64_t kfirst, klast;
  group_slots(p, g, kfirst, klast);
  if (klast - kfirst + 1 <= kFusedSlots) return;
  const ACC* src = (const ACC*)p.partial + (int64_t)q * W + lane;
  const int64_t slot_stride = (int64_t)T * W;
  ACC v0 = 0, v1 = 0, v2 = 0, v3 = 0;
  int64_t kk = kfirst;
  for (; kk + 3 <= klast; kk += 4) {
    v0 += src[(kk + g) * slot_stride];
    v1 += src[(kk + 1 + g) * slot_stride];
    v2 += src[(kk + 2 + g) * slot_stride];
    v3 += src[(kk + 3 + g) * slot_stride];
  }
  for (; kk <= klast; ++kk) v0 += src[(kk + g) * slot_stride];
  ((ACC*)p.dsum)[((int64_t)g * T + q) * W + lane] = (v0 + v1) + (v2 + v3);
}

// Per group (complex, direction tile): sum its slots (or read its dsum row),
// scan along the thresholds (cumulative sum of Algorithm 1,
// out[b][p][q] = sum_{j <= q} D[p][j]) and write the 64 x T block of out.
// 16 row chunks x 64 lanes; each thread holds PC rows of its chunk in
// registers at a time.  A chunk of at most PC rows (T <= 16 PC) takes one
// pass; longer chunks first sum every row group (for the offsets) and then
// scan piece by piece.
constexpr int kReducePiece = 16;

template <typename ACC>
__global__ __launch_bounds__(1024) void k_reduce_scan(Params p) {
  constexpr int PC = kReducePiece;
  using O = OutOf<ACC>;
  using OT = typename O::T;
  extern __shared__ __align__(16) unsigned char smem[];
  const int T = p.T;
  const int LS = T + 1;  // padded row of the transposed result
  OT* L = (OT*)smem;     // [64][T+1]
  ACC* tot = (ACC*)(smem + align_up((size_t)W * LS * sizeof(OT), 16));  // [16][64]
  const int g = blockIdx.x;
  const int gpc = p.ntiles;
  const int b = g / gpc, t = g % gpc;
  const int lane = threadIdx.x & (W - 1), r = threadIdx.x >> 6;
  const int chunk = (T + 15) / 16;
  const int q0 = min(T, r * chunk), nq = min(T, q0 + chunk) - q0;
  int fexp = 0;
  if constexpr (sizeof(ACC) == 8) fexp = fixed_exp(p);
  const int64_t slot_stride = (int64_t)T * W;
  int64_t kfirst = 0, klast = -1;
  group_slots(p, g, kfirst, klast);
  if (kfirst == klast) return;  // one block covered the whole group and wrote its output
  const bool active = r < 16 && nq > 0;
  const bool from_dsum = p.split && klast - kfirst + 1 > kFusedSlots;
  // v[j] = D[q + j] for j < n (rows past n repeat the last row and are dropped);
  // loads use clamped rows so that all PC loads of a slot are independent
  auto rows = [&](int q, int n, ACC* v) {
#pragma unroll
    for (int j = 0; j < PC; ++j) v[j] = 0;
    if (from_dsum) {
      const ACC* src = (const ACC*)p.dsum + (int64_t)g * slot_stride + (int64_t)q * W + lane;
#pragma unroll
      for (int j = 0; j < PC; ++j) v[j] = src[min(j, n - 1) * W];
    } else {
      for (int64_t kk = kfirst; kk <= klast; ++kk) {
        const ACC* src = (const ACC*)p.partial + (kk + g) * slot_stride + (int64_t)q * W + lane;
        ACC x[PC];
#pragma unroll
        for (int j = 0; j < PC; ++j) x[j] = src[min(j, n - 1) * W];
#pragma unroll
        for (int j = 0; j < PC; ++j) v[j] += x[j];
      }
    }
#pragma unroll
    for (int j = 0; j < PC; ++j)
      if (j >= n) v[j] = 0;
  };
  ACC acc[PC];
  if (chunk <= PC) {
    // one pass: the whole chunk stays in registers
#pragma unroll
    for (int j = 0; j < PC; ++j) acc[j] = 0;
    if (active) rows(q0, nq, acc);
    ACC run = 0;
#pragma unroll
    for (int j = 0; j < PC; ++j) {
      run += acc[j];
      acc[j] = run;
    }
    if (r < 16) tot[r * W + lane] = run;
    __syncthreads();
    ACC off = 0;
    for (int rr = 0; rr < r && rr < 16; ++rr) off += tot[rr * W + lane];
    if (active) {
#pragma unroll
      for (int j = 0; j < PC; ++j)
        if (j < nq) L[lane * LS + q0 + j] = O::conv(acc[j] + off, fexp);
    }
  } else {
    // two passes: chunk totals, then the scan piece by piece
    ACC run = 0;
    if (active)
      for (int q = 0; q < nq; q += PC) {
        rows(q0 + q, min(PC, nq - q), acc);
#pragma unroll
        for (int j = 0; j < PC; ++j) run += acc[j];
      }
    if (r < 16) tot[r * W + lane] = run;
    __syncthreads();
    ACC carry = 0;
    for (int rr = 0; rr < r && rr < 16; ++rr) carry += tot[rr * W + lane];
    if (active)
      for (int q = 0; q < nq; q += PC) {
        const int n = min(PC, nq - q);
        rows(q0 + q, n, acc);
#pragma unroll
        for (int j = 0; j < PC; ++j) {
          carry += acc[j];
          if (j < n) L[lane * LS + q0 + q + j] = O::conv(carry, fexp);
        }
      }
  }
  __syncthreads();
  const int dv = min(W, p.d - t * W);
  OT* out = (OT*)p.out + ((int64_t)b * p.d + (int64_t)t * W) * T;
  for (int i = threadIdx.x; i < dv * T; i += blockDim.x) {
    const int pp = i / T, q = i - pp * T;
    out[i] = L[pp * LS + q];
  }
}

// Largest |w| over the float32 weights, per block: absmax[dim * 64 + block].
__global__ __launch_bounds__(256) void k_absmax(Params p) {
  __shared__ float red[256];
  const int dim = blockIdx.y;
  const float* w = nullptr;
  int64_t n = 0;
  if (p.wmode == WM_VMAX) {
    if (dim == 0) { w = (const float*)p.weights[0]; n = p.count[0]; }
  } else if (dim <= p.top_dim) {
    w = (const float*)p.weights[dim];
    n = p.count[dim];
  }
  float m = 0.0f;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) m = fmaxf(m, fabsf(w[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) p.absmax[dim * gridDim.x + blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------
// backward (adjoint), simplicial, float32 weights
// ---------------------------------------------------------------------------
//
// For L = <grad_out, out>, dL/dw(c) = (-1)^dim(c) sum_p G[p][b_p(c)] with
// G[p][j] = sum_{q >= j} grad_out[p][q] and G[p][T] = 0.  The block holds G for
// up to `dg` direction tiles in LDS ([tile][T+1][64], read conflict-free by
// lane), recomputes each staged simplex's index per direction and sums the
// 64 x dg values with a wavefront reduction.

constexpr int kMaxDG = 4;

template <int N, int DIM, int WM, bool FAST>
__device__ __forceinline__ void simp_bwd_range(const Params& p, int b, int64_t lo, int64_t hi, int64_t voff, int64_t soff,
                               const float* sx, const float* sy, const float* sz, int ntl, int tile0,
                               const float* Gt, float* stage, const Thr& th) {
  using L = SimpLayout<N, DIM, uint64_t>;
  const int tid = threadIdx.x, lane = tid & (W - 1);
  const int wave = uniform(tid >> 6);
  const int TS = p.stage;
  const int T1 = p.T + 1;
  SimpStager<N, DIM, WM, float, false> st;
  for (int64_t t0 = lo; t0 < hi; t0 += TS) {
    const int cnt = (int)mn64(TS, hi - t0);
    if (tid < cnt) {
      st.load_idx(p, soff + t0 + tid, t0 + tid);
      st.gather(p, soff + t0 + tid, voff, 0);
      st.store(stage + tid * L::STRIDE);
    }
    __syncthreads();
    // wavefront w takes the 64 consecutive entries [64 w, 64 w + 64); the
    // total of entry j is parked in lane j and all 64 are written at once
    const int e0 = wave * W;
    const int ne = max(0, min(W, cnt - e0));
    float mine = 0.0f;
    // eight entries at a time: per-lane partial sums over the direction tiles,
    // then one reduce-scatter across the lanes (entries past ne re-read the
    // last one and are zeroed)
    for (int j0 = 0; j0 < ne; j0 += 8) {
      float acc[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const float* E = stage + (e0 + min(j0 + k, ne - 1)) * L::STRIDE;
        float a = 0.0f;
#pragma unroll
        for (int jj = 0; jj < kMaxDG; ++jj) {
          if (jj < ntl) {
            int bi;
            if constexpr (N == 0) {
              // general vertex filter: the largest of the vertices' threshold indices
              const int col = min((tile0 + jj) * W + lane, p.d - 1);
              bi = 0;
#pragma unroll
              for (int j = 0; j <= DIM; ++j) {
                const int64_t r = (int64_t)bitcast<int32_t>(E[j]) * p.d + col;
                bi = max(bi, p.vb_bytes == 1 ? (int)((const uint8_t*)p.vbuckets)[r]
                                             : (int)((const uint16_t*)p.vbuckets)[r]);
              }
            } else {
              const float h = max_height<N, DIM>(E, sx[jj], sy[jj], sz[jj]);
              if (FAST && th.arith) {
                // arithmetic index; the one-read fix only where a lane sits on a threshold
                if (__builtin_amdgcn_ballot_w64(!thr_arith(h, th, bi) ? 1 : 0) != 0) bi = thr_index<FAST>(h, th);
              } else {
                bi = thr_index<FAST>(h, th);
              }
            }
            a += Gt[((size_t)jj * T1 + bi) * W + lane];
          }
        }
        acc[k] = j0 + k < ne ? a : 0.0f;
      }
      const float tot = sum_scatter8(acc);  // lane l: total of entry j0 + (l & 7)
      mine = (lane >> 3) == (j0 >> 3) ? tot : mine;
    }
    if constexpr (DIM & 1) mine = -mine;
    if (lane < ne) {
      const int64_t row = soff + t0 + e0 + lane;
      if constexpr (WM == WM_VMAX) {
        const int own = bitcast<int>(stage[(e0 + lane) * L::STRIDE + L::OOFF]);
        atomicAdd(p.grad_vertex + voff + own, mine);
      } else {
        float* gw = p.grad_w[DIM];
        if (gw) {
          if (p.bwd_atomic) atomicAdd(gw + row, mine);
          else gw[row] = mine;
        }
      }
    }
    __syncthreads();
  }
}

template <int N, int WM, bool FAST>
__device__ __forceinline__ void simp_bwd_dim(int dim, const Params& p, int b, int64_t lo, int64_t hi, int64_t voff,
                                             int64_t soff, const float* sx, const float* sy, const float* sz, int ntl,
                                             int tile0, const float* Gt, float* stage, const Thr& th) {
  switch (dim) {
    case 0: simp_bwd_range<N, 0, WM, FAST>(p, b, lo, hi, voff, soff, sx, sy, sz, ntl, tile0, Gt, stage, th); break;
    case 1: simp_bwd_range<N, 1, WM, FAST>(p, b, lo, hi, voff, soff, sx, sy, sz, ntl, tile0, Gt, stage, th); break;
    case 2: simp_bwd_range<N, 2, WM, FAST>(p, b, lo, hi, voff, soff, sx, sy, sz, ntl, tile0, Gt, stage, th); break;
    default: simp_bwd_range<N, 3, WM, FAST>(p, b, lo, hi, voff, soff, sx, sy, sz, ntl, tile0, Gt, stage, th); break;
  }
}

template <int N, int WM>
__global__ __launch_bounds__(1024) void k_simp_bwd(Params p) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int T = p.T, T1 = T + 1;
  const int dg = p.dg;
  float* Gt = (float*)smem;
  size_t off = (size_t)dg * T1 * W * 4;
  float* P = (float*)(smem + off);
  off += align_up((size_t)T1 * 4, 16);
  float* stage = (float*)(smem + off);
  Thr th;
  setup_thresholds(p.thr, T, P, th);
  __syncthreads();

  const int k = blockIdx.x;
  int64_t pos = block_start(k, p.S, p.G);
  const int64_t end = block_start(k + 1, p.S, p.G);
  if (pos >= end) return;
  const int gpc = p.ngroups_dir;
  int b = find_complex(p, pos, gpc);
  const int tid = threadIdx.x, lane = tid & (W - 1), wave = tid >> 6, nw = blockDim.x >> 6;
  while (pos < end) {
    const int64_t cb = cum_elems(p, b);
    const int64_t nb = cum_elems(p, b + 1) - cb;
    if (nb == 0) { ++b; continue; }
    const int64_t base = (int64_t)gpc * cb;
    const int jg = (int)((pos - base) / nb);  // direction group
    const int64_t e0 = (pos - base) - (int64_t)jg * nb;
    const int64_t e1 = mn64(nb, e0 + (end - pos));
    const int tile0 = jg * dg;
    const int ntl = min(dg, p.ntiles - tile0);
    float sx[kMaxDG], sy[kMaxDG], sz[kMaxDG];
#pragma unroll
    for (int j = 0; j < kMaxDG; ++j) {
      sx[j] = sy[j] = sz[j] = 0.0f;
      if constexpr (N > 0) load_dir(p, (tile0 + j) * W + lane, sx[j], sy[j], sz[j]);
    }
    // reverse scan of grad_out for the group's tiles: one wavefront per tile
    __syncthreads();
    for (int j = wave; j < dg; j += nw) {
      const int gp = (tile0 + j) * W + lane;
      float* G = Gt + (size_t)j * T1 * W;
      G[(size_t)T * W + lane] = 0.0f;
      if (j < ntl && gp < p.d) {
        const float* g = p.grad_out + ((int64_t)b * p.d + gp) * T;
        double acc = 0.0;
        for (int q = T - 1; q >= 0; --q) {
          acc += (double)g[q];
          G[(size_t)q * W + lane] = (float)acc;
        }
      } else {
        for (int q = 0; q < T; ++q) G[(size_t)q * W + lane] = 0.0f;
      }
    }
    __syncthreads();
    const int64_t voff = off_or(p.vert_off, b, p.count[0]);
    int64_t dlo = 0;
    for (int dim = 0; dim <= p.top_dim; ++dim) {
      int64_t kd = (dim == 0) ? (off_or(p.vert_off, b + 1, p.count[0]) - voff)
                              : (off_or(p.simp_off[dim], b + 1, p.count[dim]) - off_or(p.simp_off[dim], b, p.count[dim]));
      const int64_t dhi = dlo + kd;
      const int64_t lo = mx64(e0, dlo), hi = mn64(e1, dhi);
      if (lo < hi) {
        const int64_t soff = dim == 0 ? voff : off_or(p.simp_off[dim], b, p.count[dim]);
        if (th.fast)
          simp_bwd_dim<N, WM, true>(dim, p, b, lo - dlo, hi - dlo, voff, soff, sx, sy, sz, ntl, tile0, Gt, stage, th);
        else
          simp_bwd_dim<N, WM, false>(dim, p, b, lo - dlo, hi - dlo, voff, soff, sx, sy, sz, ntl, tile0, Gt, stage, th);
      }
      dlo = dhi;
    }
    pos += e1 - e0;
    if (e1 == nb && jg == gpc - 1) ++b;
  }
}

// ---------------------------------------------------------------------------
// adjoint of the sigmoid relaxation
// ---------------------------------------------------------------------------
//
// S[p][q] = sum_c s(c) sig(lam (thr[q] - h_p(c))), s(c) = (-1)^dim w(c), and
// h_p(c) = <l(a), s_p> for the vertex a of c attaining the maximum height
// (lowest vertex id among equal heights).  For L = <g, S>, per cell and
// direction:
//   u_p  = sum_q g[q] sig_q                      (dL/ds(c) from direction p)
//   dh_p = -s(c) lam sum_q g[q] sig_q (1 - sig_q) (dL/dh_p(c))
// Inside the window sig is evaluated; above it sig = 1, so the tail of u is
// G[hi] = sum_{q >= hi} g[q]; below it sig = 0.  Then
//   dL/dw(c) = (-1)^dim sum_p u_p, dL/dl(a) += sum_p dh_p s_p,
//   dL/ds_p += dh_p l(a) (summed over cells in registers, one lane per p).
// The block holds one direction tile: g and G as [T(+1)][64] columns in LDS
// and the staged cells ([coordinates, global vertex rows, signed weight,
// owner]).  The 1 + (dim+1) n per-cell sums over the 64 lanes (u, and dh_p s_p
// placed in the slot of the lane's argmax vertex) go through the eight-value
// reduce-scatter; lanes 0..7 then issue the atomic adds.

template <int N, int DIM>
struct SmLayout {
  static constexpr int NV = DIM + 1;
  static constexpr int IDOFF = NV * N;     // global vertex rows
  static constexpr int COFF = IDOFF + NV;  // signed weight (float)
  static constexpr int OOFF = COFF + 1;    // owner vertex (vertex-max weights, local id)
  static constexpr int STRIDE = OOFF + 1;
};
constexpr int kSmMaxStride = 18;  // 4 vertices x 3 coordinates + 4 ids + weight + owner

template <int N, int DIM, int WM>
__device__ __forceinline__ void sm_stage(const Params& p, int64_t row, int64_t lrow, int64_t voff, float* dst) {
  using L = SmLayout<N, DIM>;
  int idx[L::NV];
  if constexpr (DIM == 0) {
    idx[0] = (int)lrow;
  } else {
    const int32_t* sp = p.simp[DIM] + row * L::NV;
#pragma unroll
    for (int j = 0; j < L::NV; ++j) idx[j] = sp[j];
  }
#pragma unroll
  for (int j = 0; j < L::NV; ++j) {
    const int64_t gid = voff + idx[j];
    const float* c = p.coords + gid * N;
#pragma unroll
    for (int k = 0; k < N; ++k) dst[j * N + k] = c[k];
    dst[L::IDOFF + j] = bitcast<float>((int32_t)gid);
  }
  float w = 1.0f;
  int own = idx[0];
  if constexpr (WM == WM_EXPLICIT) {
    w = ((const float*)p.weights[DIM])[row];
  } else if constexpr (WM == WM_VMAX) {
    const float* vw = (const float*)p.weights[0];
    w = vw[voff + idx[0]];
#pragma unroll
    for (int j = 1; j < L::NV; ++j) {
      const float x = vw[voff + idx[j]];
      if (x > w || (x == w && idx[j] < own)) { w = x; own = idx[j]; }
    }
  }
  dst[L::COFF] = (DIM & 1) ? -w : w;
  dst[L::OOFF] = bitcast<float>(own);
}

template <int N, int DIM, int WM, bool FAST>
__device__ __forceinline__ void sm_bwd_range(const Params& p, int64_t lo, int64_t hi, int64_t voff, int64_t soff,
                                             float sx, float sy, float sz, const float* g, const float* Gs,
                                             float* stage, const Thr& th, float (&gd)[3]) {
  using L = SmLayout<N, DIM>;
  constexpr int NVAL = 1 + L::NV * N;
  constexpr int NCH = (NVAL + 7) / 8;
  const int tid = threadIdx.x, lane = tid & (W - 1);
  const int wave = uniform(tid >> 6), nw = blockDim.x >> 6;
  const int TS = p.stage;
  const float R = p.sm_r, kap = p.sm_k, lam = p.sm_lam;
  const float sdir[3] = {sx, sy, sz};
  for (int64_t t0 = lo; t0 < hi; t0 += TS) {
    const int cnt = (int)mn64(TS, hi - t0);
    if (tid < cnt) sm_stage<N, DIM, WM>(p, soff + t0 + tid, t0 + tid, voff, stage + tid * L::STRIDE);
    __syncthreads();
    for (int e = wave; e < cnt; e += nw) {
      const float* E = stage + e * L::STRIDE;
      // maximum height and the vertex slot attaining it (lowest id on ties)
      float h = height<N>(E, sx, sy, sz);
      int a = 0;
      int id = bitcast<int>(E[L::IDOFF]);
#pragma unroll
      for (int j = 1; j < L::NV; ++j) {
        const float hj = height<N>(E + j * N, sx, sy, sz);
        const int idj = bitcast<int>(E[L::IDOFF + j]);
        if (hj > h || (hj == h && idj < id)) { h = hj; a = j; id = idj; }
      }
      const float c = E[L::COFF];
      const int qlo = thr_index<FAST>(h - R, th);
      const int qhi = thr_index<FAST>(next_up(h + R), th);
      float u = Gs[qhi * W + lane], v = 0.0f, u1 = 0.0f, v1 = 0.0f;
      auto term = [&](int q, float& uu, float& vv) {
        float ex;
        const float sg = sigmoid2((th.P[q + 1] - h) * kap, ex);
        const float gq = g[q * W + lane];
        uu = __builtin_fmaf(gq, sg, uu);
        vv = __builtin_fmaf(gq, ex * sg * sg, vv);
      };
      // two terms per iteration into two pairs of sums
      int q = qlo;
      for (; q + 1 < qhi; q += 2) {
        term(q, u, v);
        term(q + 1, u1, v1);
      }
      if (q < qhi) term(q, u, v);
      u += u1;
      v += v1;
      const float dh = -c * lam * v;
#pragma unroll
      for (int k = 0; k < N; ++k) gd[k] = __builtin_fmaf(dh, E[a * N + k], gd[k]);
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
        float v8[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int ix = ch * 8 + i;
          if (ix == 0) v8[i] = u;
          else if (ix < NVAL) v8[i] = a == (ix - 1) / N ? dh * sdir[(ix - 1) % N] : 0.0f;
          else v8[i] = 0.0f;
        }
        const float tot = sum_scatter8(v8);
        const int ix = ch * 8 + lane;
        if (lane < 8 && ix < NVAL) {
          if (ix == 0) {
            const float gw = (DIM & 1) ? -tot : tot;
            const int64_t row = soff + t0 + e;
            if constexpr (WM == WM_VMAX) {
              if (p.grad_vertex) atomicAdd(p.grad_vertex + voff + bitcast<int>(E[L::OOFF]), gw);
            } else if constexpr (WM == WM_EXPLICIT) {
              float* gwp = p.grad_w[DIM];
              if (gwp) {
                if (p.bwd_atomic) atomicAdd(gwp + row, gw);
                else gwp[row] = gw;
              }
            }
          } else if (p.grad_coords) {
            const int j = (ix - 1) / N, k = (ix - 1) - j * N;
            atomicAdd(p.grad_coords + (int64_t)bitcast<int>(E[L::IDOFF + j]) * N + k, tot);
          }
        }
      }
    }
    __syncthreads();
  }
}

template <int N, int WM, bool FAST>
__device__ __forceinline__ void sm_bwd_dim(int dim, const Params& p, int64_t lo, int64_t hi, int64_t voff,
                                           int64_t soff, float sx, float sy, float sz, const float* g,
                                           const float* Gs, float* stage, const Thr& th, float (&gd)[3]) {
  switch (dim) {
    case 0: sm_bwd_range<N, 0, WM, FAST>(p, lo, hi, voff, soff, sx, sy, sz, g, Gs, stage, th, gd); break;
    case 1: sm_bwd_range<N, 1, WM, FAST>(p, lo, hi, voff, soff, sx, sy, sz, g, Gs, stage, th, gd); break;
    case 2: sm_bwd_range<N, 2, WM, FAST>(p, lo, hi, voff, soff, sx, sy, sz, g, Gs, stage, th, gd); break;
    default: sm_bwd_range<N, 3, WM, FAST>(p, lo, hi, voff, soff, sx, sy, sz, g, Gs, stage, th, gd); break;
  }
}

template <int N, int WM>
__global__ __launch_bounds__(1024) void k_smooth_bwd(Params p) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int T = p.T, T1 = T + 1;
  float* g = (float*)smem;                        // [T][64]
  float* Gs = g + (size_t)T * W;                  // [T+1][64]
  float* P = Gs + (size_t)T1 * W;                 // [T+1]
  float* stage = (float*)((unsigned char*)P + align_up((size_t)T1 * 4, 16));
  Thr th;
  setup_thresholds(p.thr, T, P, th);
  __syncthreads();

  const int k = blockIdx.x;
  int64_t pos = block_start(k, p.S, p.G);
  const int64_t end = block_start(k + 1, p.S, p.G);
  if (pos >= end) return;
  const int gpc = p.ntiles;
  int b = find_complex(p, pos, gpc);
  const int tid = threadIdx.x, lane = tid & (W - 1), wave = tid >> 6;
  while (pos < end) {
    const int64_t cb = cum_elems(p, b);
    const int64_t nb = cum_elems(p, b + 1) - cb;
    if (nb == 0) { ++b; continue; }
    const int64_t base = (int64_t)gpc * cb;
    const int t = (int)((pos - base) / nb);  // direction tile
    const int64_t e0 = (pos - base) - (int64_t)t * nb;
    const int64_t e1 = mn64(nb, e0 + (end - pos));
    const int gp = t * W + lane;
    float sx, sy, sz;
    load_dir(p, gp, sx, sy, sz);
    // the tile's rows of grad_out (read along q by the whole block), then the
    // reverse scan G[j] = sum_{q >= j} g[q] (G[T] = 0) by wavefront 0, in float64
    __syncthreads();
    for (int i = tid; i < W * T; i += blockDim.x) {
      const int r = i / T, q = i - r * T;
      const int dir = t * W + r;
      g[(size_t)q * W + r] = dir < p.d ? p.grad_out[((int64_t)b * p.d + dir) * T + q] : 0.0f;
    }
    __syncthreads();
    if (wave == 0) {
      Gs[(size_t)T * W + lane] = 0.0f;
      double acc = 0.0;
      for (int q = T - 1; q >= 0; --q) {
        acc += (double)g[(size_t)q * W + lane];
        Gs[(size_t)q * W + lane] = (float)acc;
      }
    }
    __syncthreads();
    float gd[3] = {0.0f, 0.0f, 0.0f};
    const int64_t voff = off_or(p.vert_off, b, p.count[0]);
    int64_t dlo = 0;
    for (int dim = 0; dim <= p.top_dim; ++dim) {
      int64_t kd = (dim == 0) ? (off_or(p.vert_off, b + 1, p.count[0]) - voff)
                              : (off_or(p.simp_off[dim], b + 1, p.count[dim]) - off_or(p.simp_off[dim], b, p.count[dim]));
      const int64_t dhi = dlo + kd;
      const int64_t lo = mx64(e0, dlo), hi = mn64(e1, dhi);
      if (lo < hi) {
        const int64_t soff = dim == 0 ? voff : off_or(p.simp_off[dim], b, p.count[dim]);
        if (th.fast) sm_bwd_dim<N, WM, true>(dim, p, lo - dlo, hi - dlo, voff, soff, sx, sy, sz, g, Gs, stage, th, gd);
        else sm_bwd_dim<N, WM, false>(dim, p, lo - dlo, hi - dlo, voff, soff, sx, sy, sz, g, Gs, stage, th, gd);
      }
      dlo = dhi;
    }
    if (p.grad_dirs && gp < p.d) {
#pragma unroll
      for (int kk = 0; kk < N; ++kk) atomicAdd(p.grad_dirs + (int64_t)gp * N + kk, gd[kk]);
    }
    pos += e1 - e0;
    if (e1 == nb && t == gpc - 1) ++b;
  }
}

// ---------------------------------------------------------------------------
// lower-star index and the vertex-centric relaxation
// ---------------------------------------------------------------------------
//
// Every cell c has one vertex a_p(c) attaining its maximum height for
// direction p (lowest id among equal heights), and its relaxed term is
// sig(lam (t - h_p(a))).  Grouping the cells by that vertex, the relaxation is
//   S[p][q] = sum over vertices v of W_p(v) sig(lam (thr[q] - h_p(v))),
//   W_p(v) = sum of the signed weights of the cells c with a_p(c) = v,
// so one sigmoid window per vertex and direction replaces one per cell and
// direction.  W_p(v) needs the cells that contain v (the lower star of v is
// the part of them that v tops): the index lists, for every vertex (global
// row), the simplices of dimension >= 1 that contain it, as {dim, the other
// vertices' global rows (-1 padded)} and the simplex's row.  It depends on the
// simplex lists only, so one build serves every call on the same topology.
// Build: one atomic count per incidence, an exclusive scan of the counts
// (per-chunk sums, one-block scan of the sums, per-chunk scan), and a fill
// through per-vertex cursors.  The order of a vertex's entries follows the
// atomics; no result depends on it.

// complex of simplex row r of dimension dim: largest b with simp_off[dim][b] <= r
__device__ __forceinline__ int complex_of_row(const Params& p, int dim, int64_t r) {
  const int64_t* so = p.simp_off[dim];
  if (!so) return 0;
  int lo = 0, hi = p.B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (so[mid] <= r) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Global rows of the dim+1 vertices of simplex (dim, r); entries past dim are 0.
__device__ __forceinline__ void simplex_rows(const Params& p, int dim, int64_t r, int32_t (&g)[4]) {
  const int b = complex_of_row(p, dim, r);
  const int32_t voff = (int32_t)off_or(p.vert_off, b, p.count[0]);
  const int32_t* sp = p.simp[dim] + r * (dim + 1);
#pragma unroll
  for (int j = 0; j < 4; ++j) g[j] = j <= dim ? voff + sp[j] : 0;
}

__global__ __launch_bounds__(256) void k_ls_count(Params p) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int dim = 1; dim <= p.top_dim; ++dim) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < p.count[dim]; r += stride) {
      int32_t g[4];
      simplex_rows(p, dim, r, g);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (j <= dim) atomicAdd((unsigned long long*)&p.ls_cur[g[j]], 1ull);
    }
  }
}

// Sum over a block of 256 threads (every thread gets it); red holds 256 values.
__device__ __forceinline__ int64_t block_sum256(int64_t v, int64_t* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const int64_t r = red[0];
  __syncthreads();
  return r;
}

// per chunk of kLsChunk vertices: the sum of the counts, and the largest count
__global__ __launch_bounds__(256) void k_ls_scan_parts(Params p) {
  __shared__ int64_t red[256];
  const int64_t V = p.count[0];
  const int64_t c0 = (int64_t)blockIdx.x * kLsChunk, c1 = mn64(V, c0 + kLsChunk);
  int64_t sum = 0, mx = 0;
  for (int64_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) {
    const int64_t c = p.ls_cur[i];
    sum += c;
    mx = mx64(mx, c);
  }
  sum = block_sum256(sum, red);
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = mx64(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    p.ls_part[blockIdx.x] = sum;
    atomicMax((unsigned long long*)&p.ls_hdr[1], (unsigned long long)red[0]);
  }
}

// exclusive scan of the nparts chunk sums, in place (one block)
__global__ __launch_bounds__(1024) void k_ls_scan_top(Params p, int64_t nparts) {
  __shared__ int64_t tot[1024];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t per = (nparts + nt - 1) / nt;
  const int64_t a = mn64(nparts, tid * per), z = mn64(nparts, a + per);
  int64_t s = 0;
  for (int64_t i = a; i < z; ++i) s += p.ls_part[i];
  tot[tid] = s;
  __syncthreads();
  for (int o = 1; o < nt; o <<= 1) {
    const int64_t add = tid >= o ? tot[tid - o] : 0;
    __syncthreads();
    tot[tid] += add;
    __syncthreads();
  }
  int64_t run = tot[tid] - s;
  for (int64_t i = a; i < z; ++i) {
    const int64_t c = p.ls_part[i];
    p.ls_part[i] = run;
    run += c;
  }
}

// offsets (off[v+1] = counts up to v) and fill cursors (cur[v] = off[v]) of one
// chunk: every thread scans kLsChunk / 256 consecutive counts
__global__ __launch_bounds__(256) void k_ls_scan_apply(Params p) {
  __shared__ int64_t tot[256];
  constexpr int PER = kLsChunk / 256;
  const int64_t V = p.count[0];
  const int tid = threadIdx.x;
  const int64_t a = (int64_t)blockIdx.x * kLsChunk + (int64_t)tid * PER;
  int64_t c[PER];
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    c[k] = a + k < V ? p.ls_cur[a + k] : 0;
    s += c[k];
  }
  tot[tid] = s;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const int64_t add = tid >= o ? tot[tid - o] : 0;
    __syncthreads();
    tot[tid] += add;
    __syncthreads();
  }
  int64_t run = p.ls_part[blockIdx.x] + tot[tid] - s;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    if (a + k < V) {
      p.ls_cur[a + k] = run;
      run += c[k];
      p.ls_off[a + k + 1] = run;
    }
  }
  if (blockIdx.x == 0 && tid == 0) p.ls_off[0] = 0;
}

// One launch per dimension, in increasing order, so that every vertex's
// entries list its edges first.  Each entry also gets its neighbour bits: an
// edge is bit k when it is the vertex's k-th edge; after the edges (and
// k_ls_edge_counts), a higher coface maps each other vertex to the bit of
// the vertex's edge to it.  Every coface of a face-closed complex maps this
// way; a vertex with more than 32 edges, or with a coface whose vertex pair
// has no edge, gets nbc = -1 and is handled by the per-row height test.
__global__ __launch_bounds__(256) void k_ls_fill(Params p, int dim) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int4* ent = (const int4*)p.ls_ent;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < p.count[dim]; r += stride) {
    int32_t g[4];
    simplex_rows(p, dim, r, g);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (j <= dim) {
        const int32_t v = g[j];
        const int64_t pos = (int64_t)atomicAdd((unsigned long long*)&p.ls_cur[v], 1ull);
        // the other vertices in their order within the simplex
        int32_t o[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const int src = k < j ? k : k + 1;  // skip slot j
          o[k] = src <= dim ? g[src] : -1;
        }
        uint32_t m = 0;
        if (dim == 1) {
          const int64_t k = pos - p.ls_off[v];
          m = k < 32 ? 1u << (uint32_t)k : 0u;
        } else {
          const int nbc = p.ls_nbc[v];  // may turn -1 concurrently: then the bits are not used
          const int64_t e0 = p.ls_off[v];
          bool ok = nbc >= 0;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            if (k < dim && ok) {
              int at = -1;
              for (int q = 0; q < nbc; ++q)
                if (ent[e0 + q].y == o[k]) at = q;
              if (at < 0) ok = false;
              else m |= 1u << (uint32_t)at;
            }
          }
          if (nbc >= 0 && !ok) p.ls_nbc[v] = -1;
        }
        int4 e;
        e.x = dim;
        e.y = o[0];
        e.z = o[1];
        e.w = o[2];
        ((int4*)p.ls_ent)[pos] = e;
        p.ls_row[pos] = r;
        p.ls_mask[pos] = m;
      }
    }
  }
}

// After the edges are filled: nbc = the vertex's edge count (its first
// entries), or -1 above 32.
__global__ __launch_bounds__(256) void k_ls_edge_counts(Params p) {
  const int64_t V = p.count[0];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < V; v += stride) {
    const int64_t ne1 = p.ls_cur[v] - p.ls_off[v];
    p.ls_nbc[v] = ne1 <= 32 ? (int32_t)ne1 : -1;
  }
}

// Cofaces are staged per wavefront.  A wavefront takes groups of kLsGroup
// consecutive vertices; their cofaces are consecutive in the index, so as
// many of the group's vertices as have at most R cofaces (R = kLsRows, or half
// of it when the LDS is short) together are
// staged at once: lane r loads coface row r (its entry, then the other
// vertices' coordinates and weights, all rows in flight at once), lane t < nv
// loads vertex t's coordinates and own weight, and every lane then reads the
// rows as broadcasts.  A vertex with more than R cofaces is staged in
// chunks on its own.  Coface row layout (floats):
//   [3k .. 3k+N-1]  coordinates of the k-th other vertex (k < dim)
//   [9 + k]         its global row (-1 past dim)
//   [12] dim, [13] signed weight (-1)^dim w, [14..15] simplex row (int64),
//   [16] owner: lowest-numbered vertex of largest vertex weight (vertex-max),
//   [17] neighbour bits (written by k_ls_fill)
// Vertex rows: [4t .. 4t+N-1] coordinates, [4t+3] own weight.
//
// When every coface of the vertex maps to bits over its edges (nbc >= 0; the
// edges are its first nbc rows), each lane first sets bit k for every edge
// neighbour that lies above the vertex (greater height, or equal height and
// a lower row), and the vertex tops a coface exactly when the coface's bits
// miss that set: one AND per row instead of the other vertices' heights.
constexpr int kLsStride = 18;
constexpr int kLsRows = 64;   // staged coface rows per wavefront (32 when 64 leave too little LDS)
constexpr int kLsGroup = 10;  // vertices per wavefront group

template <int N, int WM, bool BWD>
__device__ __forceinline__ void ls_stage(const Params& p, int64_t e, int32_t gv, float* dst) {
  const int4 en = ((const int4*)p.ls_ent)[e];
  const int dim = en.x;
  const int32_t o[3] = {en.y, en.z, en.w};
  const float* vw = (const float*)p.weights[0];
  float wm = 0.0f;
  int32_t own = gv;
  if constexpr (WM == WM_VMAX) wm = vw[gv];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k < dim) {
      const float* c = p.coords + (int64_t)o[k] * N;
#pragma unroll
      for (int cc = 0; cc < N; ++cc) dst[3 * k + cc] = c[cc];
      if constexpr (WM == WM_VMAX) {
        const float x = vw[o[k]];
        if (x > wm || (x == wm && o[k] < own)) { wm = x; own = o[k]; }
      }
    }
    dst[9 + k] = bitcast<float>(k < dim ? o[k] : -1);
  }
  float w = 1.0f;
  int64_t row = 0;
  if constexpr (WM == WM_EXPLICIT || BWD) row = p.ls_row[e];
  if constexpr (WM == WM_EXPLICIT) w = ((const float*)p.weights[dim])[row];
  else if constexpr (WM == WM_VMAX) w = wm;
  dst[12] = bitcast<float>(dim);
  dst[13] = (dim & 1) ? -w : w;
  dst[17] = bitcast<float>(p.ls_mask[e]);
  if constexpr (BWD) {
    dst[14] = bitcast<float>((uint32_t)row);
    dst[15] = bitcast<float>((uint32_t)((uint64_t)row >> 32));
    dst[16] = bitcast<float>(own);
  }
}

// LDS writes of a wavefront made visible to its other lanes (and reads
// finished before the rows are overwritten).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Does vertex gv (height hv for the lane) attain the maximum height of the
// staged coface E?  Ties go to the lowest global row.  The row's dimension is
// the same for every lane (a broadcast read), so the loop over the other
// vertices branches on a scalar; the common case is decided by the largest
// other height, and only a wavefront with a lane on a tie takes the exact
// per-vertex test.
template <int N>
__device__ __forceinline__ bool ls_top(const float* E, int32_t gv, float hv, float sx, float sy, float sz) {
  const int dim = uniform(bitcast<int>(E[12]));
  float ho[3];
  float hmax = -INFINITY;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k < dim) {
      ho[k] = height<N>(E + 3 * k, sx, sy, sz);
      hmax = fmaxf(hmax, ho[k]);
    }
  }
  bool top = hv > hmax;
  if (__builtin_amdgcn_ballot_w64(hv == hmax) != 0) {
    top = hv >= hmax;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (k < dim) top = top && (ho[k] < hv || bitcast<int32_t>(E[9 + k]) > gv);
    }
  }
  return top;
}

// Bits of the vertex's edge neighbours (rows E0 .. E0 + nbc - 1) that lie
// above it for the lane's direction.
template <int N>
__device__ __forceinline__ uint32_t ls_above(const float* E0, int nbc, int32_t gv, float hv, float sx, float sy,
                                             float sz) {
  uint32_t above = 0;
  for (int k = 0; k < nbc; ++k) {
    const float* E = E0 + k * kLsStride;
    const float ho = height<N>(E, sx, sy, sz);
    const int32_t id = bitcast<int32_t>(E[9]);
    above |= (ho > hv || (ho == hv && id < gv)) ? (1u << k) : 0u;
  }
  return above;
}

template <int WM>
__device__ __forceinline__ float ls_self_weight(const Params& p, int32_t gv) {
  if constexpr (WM == WM_ONES) return 1.0f;
  else return ((const float*)p.weights[0])[gv];  // explicit vertex weight, or the vertex weight itself
}

// Walks the vertices [lo, hi) (local numbering, global row voff + v) of the
// wavefront's groups: begin(gv, xv, wself, nbc), then rows(S, r0, r1) for the
// vertex's coface rows (possibly in several chunks), then end().  nbc is the
// vertex's edge count from the index (-1: no neighbour bits).
template <int N, int WM, bool BWD, typename Begin, typename Rows, typename End>
__device__ __forceinline__ void ls_walk(const Params& p, int64_t lo, int64_t hi, int64_t voff, int R, float* S,
                                        float* Vr, Begin begin, Rows rows, End end) {
  const int lane = threadIdx.x & (W - 1);
  const int wave = uniform(threadIdx.x >> 6), nw = blockDim.x >> 6;
  for (int64_t vg = lo + (int64_t)wave * kLsGroup; vg < hi; vg += (int64_t)nw * kLsGroup) {
    const int64_t vend = mn64(vg + kLsGroup, hi);
    // the group's kLsGroup + 1 offsets in one load: lane k holds off[vg + k]
    const int64_t offl = p.ls_off[voff + mn64(vg + min(lane, kLsGroup), vend)];
    // and their edge counts: lane k holds nbc[vg + k] (k < vend - vg)
    const int nbcl = p.ls_nbc[voff + mn64(vg + min(lane, kLsGroup - 1), vend - 1)];
    auto nbc_at = [&](int64_t v) { return __builtin_amdgcn_readlane(nbcl, (int)(v - vg)); };
    auto off_at = [&](int64_t v) {  // off[v] for vg <= v <= vend (scalar)
      return (int64_t)__builtin_amdgcn_readlane((int)(uint32_t)offl, (int)(v - vg)) |
             ((int64_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)offl >> 32), (int)(v - vg)) << 32);
    };
    int64_t i = vg;
    while (i < vend) {
      const int64_t rb = off_at(i);
      int64_t j = i + 1;
      while (j < vend && off_at(j + 1) - rb <= R) ++j;
      const int nv = (int)(j - i);
      const int64_t nrows = off_at(j) - rb;
      // vertex rows
      if (lane < nv) {
        const int32_t gv = (int32_t)(voff + i + lane);
        const float* c = p.coords + (int64_t)gv * N;
#pragma unroll
        for (int cc = 0; cc < N; ++cc) Vr[4 * lane + cc] = c[cc];
        Vr[4 * lane + 3] = ls_self_weight<WM>(p, gv);
      }
      if (nrows <= R) {
        // the vertex each row belongs to: rows of vertex t start at off[i + t] - rb
        const int64_t rel = offl - rb;  // lane k: start of vertex vg + k
        const int sh = (int)(i - vg);
        if (lane < nrows) {
          int t = 0;
#pragma unroll
          for (int k = 1; k < kLsGroup; ++k) {
            const int64_t st = __shfl(rel, min(sh + k, kLsGroup));
            if (k < nv && st <= lane) t = k;
          }
          ls_stage<N, WM, BWD>(p, rb + lane, (int32_t)(voff + i + t), S + lane * kLsStride);
        }
        wave_lds_sync();
        for (int t = 0; t < nv; ++t) {
          const int32_t gv = (int32_t)(voff + i + t);
          begin(gv, Vr + 4 * t, Vr[4 * t + 3], nbc_at(i + t));
          rows(S, (int)(off_at(i + t) - rb), (int)(off_at(i + t + 1) - rb));
          end();
        }
        wave_lds_sync();
      } else {  // one vertex with more than R cofaces, in chunks
        const int32_t gv = (int32_t)(voff + i);
        wave_lds_sync();
        begin(gv, Vr, Vr[3], nbc_at(i));
        for (int64_t c0 = 0; c0 < nrows; c0 += R) {
          const int m = (int)mn64(R, nrows - c0);
          if (lane < m) ls_stage<N, WM, BWD>(p, rb + c0 + lane, gv, S + lane * kLsStride);
          wave_lds_sync();
          rows(S, 0, m);
          wave_lds_sync();
        }
        end();
      }
      i = j;
    }
  }
}

// Forward over vertices [lo, hi) of one complex: each lane combines the
// vertex's own weight with its cofaces' signed weights where the vertex tops
// them (float64 sum, then the fixed-point grid), and adds one sigmoid window.
template <int N, int WM, bool FAST>
__device__ __forceinline__ void ls_fwd_range(const Params& p, int64_t lo, int64_t hi, int64_t voff, int R, float sx,
                                             float sy, float sz, uint64_t* hist, float* stage, const Thr& th,
                                             int fexp) {
  const int lane = threadIdx.x & (W - 1);
  const int wave = uniform(threadIdx.x >> 6);
  float* S = stage + (size_t)wave * (R * kLsStride + 4 * kLsGroup);
  float* Vr = S + R * kLsStride;
  int32_t gv = 0;
  float hv = 0.0f;
  double Wc = 0.0;
  int nbc = -1;
  bool have = false;
  uint32_t above = 0;
  ls_walk<N, WM, false>(
      p, lo, hi, voff, R, S, Vr,
      [&](int32_t g, const float* xv, float wself, int nb) {
        gv = g;
        hv = height<N>(xv, sx, sy, sz);
        Wc = wself;
        nbc = nb;
        have = false;
      },
      [&](const float* Sr, int r0, int r1) {
        if (nbc >= 0) {
          if (!have) {  // the edges lead the vertex's first rows
            above = ls_above<N>(Sr + r0 * kLsStride, nbc, gv, hv, sx, sy, sz);
            have = true;
          }
          for (int r = r0; r < r1; ++r) {
            const float* E = Sr + r * kLsStride;
            Wc += (bitcast<uint32_t>(E[17]) & above) == 0 ? (double)E[13] : 0.0;
          }
        } else {
          for (int r = r0; r < r1; ++r) {
            const float* E = Sr + r * kLsStride;
            Wc += ls_top<N>(E, gv, hv, sx, sy, sz) ? (double)E[13] : 0.0;
          }
        }
      },
      [&]() {
        const uint64_t C = (uint64_t)(int64_t)rint(ldexp(Wc, fexp));
        smooth_add<FAST>(hist + lane, hv, C, th, p.sm_r, p.sm_k);
      });
}

template <int N, int WM>
__global__ __launch_bounds__(1024) void k_smooth_ls_fwd(Params p, int rows) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int T = p.T;
  uint64_t* hist = (uint64_t*)smem;
  float* P = (float*)(smem + (size_t)(T + 1) * W * 8);
  float* stage = (float*)((unsigned char*)P + align_up((size_t)(T + 1) * 4, 16));
  Thr th;
  setup_thresholds(p.thr, T, P, th);
  for (int i = threadIdx.x; i < (T + 1) * W; i += blockDim.x) hist[i] = 0;
  const int fexp = fixed_exp(p);
  __syncthreads();
  const int k = blockIdx.x;
  int64_t pos, end;
  int b;
  if (!block_range<uint64_t>(p, hist, k, fexp, pos, end, b)) return;
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
    float sx, sy, sz;
    load_dir(p, t * W + lane, sx, sy, sz);
    const int64_t voff = off_or(p.vert_off, b, p.count[0]);
    if (th.fast) ls_fwd_range<N, WM, true>(p, e0, e1, voff, rows, sx, sy, sz, hist, stage, th, fexp);
    else ls_fwd_range<N, WM, false>(p, e0, e1, voff, rows, sx, sy, sz, hist, stage, th, fexp);
    end_group<uint64_t>(p, hist, k, b, t, e0 == 0 && e1 == nb, fexp);
    pos += e1 - e0;
    if (e1 == nb && t == gpc - 1) ++b;
  }
}

// Adjoint over vertices [lo, hi) of one complex.  Per vertex and lane: the
// window sums u = G[hi] + sum g sig and v = sum g sig (1 - sig) (they depend on
// the vertex's height only); then the staged cofaces, eight at a time: each
// adds its signed weight to W where the vertex tops it, and the sum over the
// lanes of u where it does is that cell's weight gradient (eight-value
// reduce-scatter; lanes 0..7 add it).  Finally dh = -lam W v: the vertex's
// coordinate gradient is the lane sum of dh s_p (reduced together with the
// vertex's own weight gradient, the lane sum of u), and the direction
// gradient accumulates dh l(v) per lane.
template <int N, int WM, bool FAST>
__device__ __forceinline__ void ls_bwd_range(const Params& p, int64_t lo, int64_t hi, int64_t voff, int rows,
                                             float sx, float sy, float sz, const float* g, const float* Gs,
                                             float* stage, const Thr& th, float (&gd)[3]) {
  const int lane = threadIdx.x & (W - 1);
  const int wave = uniform(threadIdx.x >> 6);
  const float R = p.sm_r, kap = p.sm_k, lam = p.sm_lam;
  float* S = stage + (size_t)wave * (rows * kLsStride + 4 * kLsGroup);
  float* Vr = S + rows * kLsStride;
  int32_t gv = 0;
  float hv = 0.0f, u = 0.0f, vs = 0.0f, Wc = 0.0f, x0 = 0.0f, x1 = 0.0f, x2 = 0.0f;
  int nbc = -1;
  bool have = false;
  uint32_t above = 0;
  ls_walk<N, WM, true>(
      p, lo, hi, voff, rows, S, Vr,
      [&](int32_t gvi, const float* xv, float wself, int nb) {
        gv = gvi;
        nbc = nb;
        have = false;
        x0 = xv[0];
        if (N >= 2) x1 = xv[1];
        if (N >= 3) x2 = xv[2];
        hv = height<N>(xv, sx, sy, sz);
        const int qlo = thr_index<FAST>(hv - R, th);
        const int qhi = thr_index<FAST>(next_up(hv + R), th);
        float ua = Gs[qhi * W + lane], va = 0.0f, ub = 0.0f, vb = 0.0f;
        auto term = [&](int q, float& uu, float& vv) {
          float ex;
          const float sg = sigmoid2((th.P[q + 1] - hv) * kap, ex);
          const float gq = g[q * W + lane];
          uu = __builtin_fmaf(gq, sg, uu);
          vv = __builtin_fmaf(gq, ex * sg * sg, vv);
        };
        int q = qlo;
        for (; q + 1 < qhi; q += 2) {
          term(q, ua, va);
          term(q + 1, ub, vb);
        }
        if (q < qhi) term(q, ua, va);
        u = ua + ub;
        vs = va + vb;
        Wc = wself;
      },
      [&](const float* Sr, int r0, int r1) {
        if (nbc >= 0 && !have) {  // the edges lead the vertex's first rows
          above = ls_above<N>(Sr + r0 * kLsStride, nbc, gv, hv, sx, sy, sz);
          have = true;
        }
        for (int j0 = r0; j0 < r1; j0 += 8) {
          float v8[8];
          if (nbc >= 0) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              const float* E = Sr + min(j0 + k, r1 - 1) * kLsStride;  // past r1: a valid row, weighed 0
              const bool top = j0 + k < r1 && (bitcast<uint32_t>(E[17]) & above) == 0;
              Wc += top ? E[13] : 0.0f;
              v8[k] = top ? u : 0.0f;
            }
          } else {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              const float* E = Sr + min(j0 + k, r1 - 1) * kLsStride;
              const bool top = j0 + k < r1 && ls_top<N>(E, gv, hv, sx, sy, sz);
              Wc += top ? E[13] : 0.0f;
              v8[k] = top ? u : 0.0f;
            }
          }
          if constexpr (WM != WM_ONES) {
            const float tot = sum_scatter8(v8);
            if (lane < 8 && j0 + lane < r1) {
              const float* E = Sr + (j0 + lane) * kLsStride;
              const int dim = bitcast<int>(E[12]);
              const float gw = (dim & 1) ? -tot : tot;
              if constexpr (WM == WM_VMAX) {
                if (p.grad_vertex) atomicAdd(p.grad_vertex + bitcast<int32_t>(E[16]), gw);
              } else {
                const int64_t row =
                    (int64_t)(((uint64_t)bitcast<uint32_t>(E[15]) << 32) | bitcast<uint32_t>(E[14]));
                float* gwp = p.grad_w[dim];
                if (gwp) atomicAdd(gwp + row, gw);
              }
            }
          }
        }
      },
      [&]() {
        const float dh = -Wc * lam * vs;
        float c8[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) c8[k] = 0.0f;
        c8[0] = dh * sx;
        if (N >= 2) c8[1] = dh * sy;
        if (N >= 3) c8[2] = dh * sz;
        c8[3] = u;  // the vertex's own weight gradient
        gd[0] = __builtin_fmaf(dh, x0, gd[0]);
        if (N >= 2) gd[1] = __builtin_fmaf(dh, x1, gd[1]);
        if (N >= 3) gd[2] = __builtin_fmaf(dh, x2, gd[2]);
        const float tot = sum_scatter8(c8);
        if (lane < N && p.grad_coords) atomicAdd(p.grad_coords + (int64_t)gv * N + lane, tot);
        if constexpr (WM != WM_ONES) {
          if (lane == 3) {
            float* gwp = WM == WM_VMAX ? p.grad_vertex : p.grad_w[0];
            if (gwp) atomicAdd(gwp + gv, tot);
          }
        }
      });
}

template <int N, int WM>
__global__ __launch_bounds__(1024) void k_smooth_ls_bwd(Params p, int rows) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int T = p.T, T1 = T + 1;
  float* g = (float*)smem;
  float* Gs = g + (size_t)T * W;
  float* P = Gs + (size_t)T1 * W;
  float* stage = (float*)((unsigned char*)P + align_up((size_t)T1 * 4, 16));
  Thr th;
  setup_thresholds(p.thr, T, P, th);
  __syncthreads();
  const int k = blockIdx.x;
  int64_t pos = block_start(k, p.S, p.G);
  const int64_t end = block_start(k + 1, p.S, p.G);
  if (pos >= end) return;
  const int gpc = p.ntiles;
  int b = find_complex(p, pos, gpc);
  const int tid = threadIdx.x, lane = tid & (W - 1), wave = tid >> 6;
  while (pos < end) {
    const int64_t cb = cum_elems(p, b);
    const int64_t nb = cum_elems(p, b + 1) - cb;
    if (nb == 0) { ++b; continue; }
    const int64_t base = (int64_t)gpc * cb;
    const int t = (int)((pos - base) / nb);
    const int64_t e0 = (pos - base) - (int64_t)t * nb;
    const int64_t e1 = mn64(nb, e0 + (end - pos));
    const int gp = t * W + lane;
    float sx, sy, sz;
    load_dir(p, gp, sx, sy, sz);
    __syncthreads();
    for (int i = tid; i < W * T; i += blockDim.x) {
      const int r = i / T, q = i - r * T;
      const int dir = t * W + r;
      g[(size_t)q * W + r] = dir < p.d ? p.grad_out[((int64_t)b * p.d + dir) * T + q] : 0.0f;
    }
    __syncthreads();
    if (wave == 0) {
      Gs[(size_t)T * W + lane] = 0.0f;
      double acc = 0.0;
      for (int q = T - 1; q >= 0; --q) {
        acc += (double)g[(size_t)q * W + lane];
        Gs[(size_t)q * W + lane] = (float)acc;
      }
    }
    __syncthreads();
    float gd[3] = {0.0f, 0.0f, 0.0f};
    const int64_t voff = off_or(p.vert_off, b, p.count[0]);
    if (th.fast) ls_bwd_range<N, WM, true>(p, e0, e1, voff, rows, sx, sy, sz, g, Gs, stage, th, gd);
    else ls_bwd_range<N, WM, false>(p, e0, e1, voff, rows, sx, sy, sz, g, Gs, stage, th, gd);
    if (p.grad_dirs && gp < p.d) {
#pragma unroll
      for (int kk = 0; kk < N; ++kk) atomicAdd(p.grad_dirs + (int64_t)gp * N + kk, gd[kk]);
    }
    pos += e1 - e0;
    if (e1 == nb && t == gpc - 1) ++b;
  }
}

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------

__global__ void k_fill_zero(float* x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0.0f;
}

// Data checks; blockIdx.y selects the check.
__global__ void k_validate(Params p, int* flags) {
  const int64_t gtid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
  int f = 0;
  switch (blockIdx.y) {
    case 0: {  // thresholds and directions
      for (int64_t i = gtid; i < p.T; i += gstride) {
        float x = p.thr[i];
        if (!isfinite(x)) f |= kFlagNonfinite;
        if (i + 1 < p.T && !(x <= p.thr[i + 1])) f |= kFlagThr;
      }
      for (int64_t i = gtid; i < (int64_t)p.d * p.n; i += gstride)
        if (!isfinite(p.dirs[i])) f |= kFlagNonfinite;
      break;
    }
    case 1: {  // simplicial coordinates and float weights
      if (p.kind != 0) break;
      for (int64_t i = gtid; i < p.count[0] * p.n; i += gstride)
        if (!isfinite(p.coords[i])) f |= kFlagNonfinite;
      if (p.dtype == 1) {
        for (int dim = 0; dim <= p.top_dim; ++dim) {
          if (p.wmode == 2 && dim > 0) break;
          const float* w = (const float*)p.weights[dim];
          if (!w) continue;
          for (int64_t i = gtid; i < p.count[dim]; i += gstride)
            if (!isfinite(w[i])) f |= kFlagNonfinite;
        }
      }
      break;
    }
    case 2: {  // simplicial offsets and vertex ids
      if (p.kind != 0) break;
      if (p.B > 1 || p.vert_off) {
        for (int64_t b = gtid; b <= p.B; b += gstride) {
          if (b == 0 && p.vert_off[0] != 0) f |= kFlagIndex;
          if (b == p.B && p.vert_off[b] != p.count[0]) f |= kFlagIndex;
          if (b < p.B && p.vert_off[b + 1] < p.vert_off[b]) f |= kFlagIndex;
          for (int dim = 1; dim <= p.top_dim; ++dim) {
            const int64_t* so = p.simp_off[dim];
            if (!so) { f |= kFlagIndex; continue; }
            if (b == 0 && so[0] != 0) f |= kFlagIndex;
            if (b == p.B && so[b] != p.count[dim]) f |= kFlagIndex;
            if (b < p.B && so[b + 1] < so[b]) f |= kFlagIndex;
          }
        }
      }
      for (int dim = 1; dim <= p.top_dim; ++dim) {
        const int64_t* so = p.simp_off[dim];
        for (int64_t r = gtid; r < p.count[dim]; r += gstride) {
          int64_t V = p.count[0];
          if (so && p.vert_off) {
            int lo = 0, hi = p.B - 1;  // complex owning row r
            while (lo < hi) {
              int mid = (lo + hi + 1) >> 1;
              if (so[mid] <= r) lo = mid; else hi = mid - 1;
            }
            V = p.vert_off[lo + 1] - p.vert_off[lo];
          }
          for (int j = 0; j <= dim; ++j) {
            int v = p.simp[dim][r * (dim + 1) + j];
            if (v < 0 || v >= V) f |= kFlagIndex;
          }
        }
      }
      break;
    }
    case 3: {  // cubical shapes, offsets and axes
      if (p.kind != 1) break;
      for (int64_t b = gtid; b < p.B; b += gstride) {
        const int n0 = p.shape[3 * b], n1 = p.shape[3 * b + 1], n2 = p.shape[3 * b + 2];
        if (n0 < 1 || n1 < 1 || n2 < 1 || (p.n == 2 && n2 != 1)) { f |= kFlagIndex; continue; }
        const int64_t nv = (int64_t)n0 * n1 * n2;
        if (nv >= ((int64_t)1 << 31)) f |= kFlagIndex;
        const int64_t g0 = off_or(p.grid_off, (int)b, p.total_voxels), g1 = off_or(p.grid_off, (int)b + 1, p.total_voxels);
        if (g1 - g0 != nv) f |= kFlagIndex;
        if (b == 0 && g0 != 0) f |= kFlagIndex;
        if (b == p.B - 1 && g1 != p.total_voxels) f |= kFlagIndex;
        const int64_t a0 = p.axis_off ? p.axis_off[b] : 0;
        const int64_t na = (int64_t)n0 + n1 + (p.n == 3 ? n2 : 0);
        if (p.axis_off && p.axis_off[b + 1] - a0 != na) f |= kFlagIndex;
        const float* ax = p.axis + a0;
        const int ext[3] = {n0, n1, n2};
        int64_t o = 0;
        for (int a = 0; a < p.n; ++a) {
          for (int i = 0; i < ext[a]; ++i) {
            if (!isfinite(ax[o + i])) f |= kFlagNonfinite;
            if (i + 1 < ext[a] && !(ax[o + i] < ax[o + i + 1])) f |= kFlagThr;
          }
          o += ext[a];
        }
      }
      break;
    }
  }
  if (f) atomicOr(flags, f);
}

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

// ---------------------------------------------------------------------------
// ECF of an image / volume: the intensity is the vertex filter
// ---------------------------------------------------------------------------
//
// Every included pixel/voxel is a vertex and every axis-aligned edge, square
// and cube whose corners are all vertices is a cell that enters the filtration
// at the largest corner intensity.  Give each cell to its largest corner in
// the order (intensity, linear index): that corner is unique, and the cell's
// value is that corner's intensity.  Voxel v then contributes, at its own
// intensity, the signed sum over the cells it owns: itself, the edges towards
// neighbours it beats, the squares and cubes all of whose other corners it
// beats.  All of them lie in its 3^N neighbourhood.  With uint8 intensities the
// histogram runs over the 256 intensity values, whatever the thresholds.

constexpr int kEcfBins = 256;

// Whether offset (d0, d1, d2) precedes the centre in linear order (axis 0 fastest).
__device__ __forceinline__ constexpr bool precedes(int d0, int d1, int d2) {
  return d2 < 0 || (d2 == 0 && (d1 < 0 || (d1 == 0 && d0 < 0)));
}

// The 3^N intensities around voxel (i0, i1, i2), neighbour (d0, d1, d2) at
// index (d0+1) + 3 (d1+1) + 9 (d2+1).  Coordinates are clamped into the grid,
// so every load is in bounds; the evaluation masks the clamped ones out.
template <int N>
struct EcfNbhd {
  static constexpr int M = N == 2 ? 9 : 27;
  int u[M];

  __device__ __forceinline__ void load(const uint8_t* vol, int n0, int n1, int n2, int i0, int i1, int i2) {
    const uint32_t col[3] = {(uint32_t)max(i0 - 1, 0), (uint32_t)i0, (uint32_t)min(i0 + 1, n0 - 1)};
    const int row[3] = {max(i1 - 1, 0), i1, min(i1 + 1, n1 - 1)};
    const int lay[3] = {max(i2 - 1, 0), i2, min(i2 + 1, n2 - 1)};
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int d0 = m % 3, d1 = (m / 3) % 3, d2 = N == 3 ? m / 9 : 1;
      u[m] = vol[(uint32_t)(lay[d2] * n1 + row[d1]) * (uint32_t)n0 + col[d0]];
    }
  }
};

// Signed sum over the cells that voxel (i0, i1, i2) owns (0 if it is not a
// vertex); the caller adds it at intensity x = its own intensity.
template <int N, int WM>
__device__ __forceinline__ int ecf_owned(const EcfNbhd<N>& nb, int n0, int n1, int n2, int i0, int i1, int i2,
                                         int inc, int& x) {
  // neighbour (d0, d1, d2) has bit (d0+1) + 3 (d1+1) + 9 (d2+1) (d2 = 0 in 2D)
  auto bit = [](int d0, int d1, int d2) { return (d0 + 1) + 3 * (d1 + 1) + (N == 3 ? 9 * (d2 + 1) : 0); };
  constexpr int M = EcfNbhd<N>::M;
  x = nb.u[(M - 1) / 2];
  // bit set: that neighbour is a vertex and v beats it in (intensity, linear index)
  const bool lo0 = i0 > 0, hi0 = i0 < n0 - 1, lo1 = i1 > 0, hi1 = i1 < n1 - 1, lo2 = i2 > 0, hi2 = i2 < n2 - 1;
  uint32_t ok = 0;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int d0 = m % 3 - 1, d1 = (m / 3) % 3 - 1, d2 = N == 3 ? m / 9 - 1 : 0;
    if (d0 == 0 && d1 == 0 && d2 == 0) continue;
    const bool in = (d0 < 0 ? lo0 : d0 > 0 ? hi0 : true) && (d1 < 0 ? lo1 : d1 > 0 ? hi1 : true) &&
                    (d2 < 0 ? lo2 : d2 > 0 ? hi2 : true);
    const int u = nb.u[m];
    const bool beats = precedes(d0, d1, d2) ? x >= u : x > u;
    ok |= (uint32_t)(in && u > inc && beats) << bit(d0, d1, d2);
  }
  auto has = [&](int d0, int d1, int d2) { return (int)((ok >> bit(d0, d1, d2)) & 1u); };
  int c = 1;  // the vertex itself
#pragma unroll
  for (int s = -1; s <= 1; s += 2) {
    c -= has(s, 0, 0) + has(0, s, 0);  // edges
    if constexpr (N == 3) c -= has(0, 0, s);
  }
#pragma unroll
  for (int sa = -1; sa <= 1; sa += 2)
#pragma unroll
    for (int sb = -1; sb <= 1; sb += 2) {
      c += has(sa, 0, 0) & has(0, sb, 0) & has(sa, sb, 0);  // squares, plane 0-1
      if constexpr (N == 3) {
        c += has(sa, 0, 0) & has(0, 0, sb) & has(sa, 0, sb);  // plane 0-2
        c += has(0, sa, 0) & has(0, 0, sb) & has(0, sa, sb);  // plane 1-2
      }
    }
  if constexpr (N == 3) {
#pragma unroll
    for (int s0 = -1; s0 <= 1; s0 += 2)
#pragma unroll
      for (int s1 = -1; s1 <= 1; s1 += 2)
#pragma unroll
        for (int s2 = -1; s2 <= 1; s2 += 2)
          c -= has(s0, 0, 0) & has(0, s1, 0) & has(0, 0, s2) & has(s0, s1, 0) & has(s0, 0, s2) & has(0, s1, s2) &
               has(s0, s1, s2);  // cubes
  }
  if (x <= inc) c = 0;  // not a vertex
  return WM == WM_VMAX ? c * x : c;
}

// Histogram of the owned signed sums over the intensity values, per image: the
// voxel stream of the batch is cut into G equal ranges (block k takes
// [kS/G, (k+1)S/G)); each wavefront adds into its own LDS histogram, and at the
// end of every image segment the block adds its 256 sums into the image's row
// of acc [B][256] (zeroed beforehand) with integer atomics, which commute.
template <int N, int WM>
__global__ __launch_bounds__(1024) void k_image_ecf(Params p) {
  __shared__ int32_t H[16][kEcfBins];
  const int nw = blockDim.x >> 6, wave = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < nw * kEcfBins; i += blockDim.x) H[i / kEcfBins][i % kEcfBins] = 0;
  __syncthreads();
  const int k = blockIdx.x;
  int64_t pos = block_start(k, p.S, p.G);
  const int64_t end = block_start(k + 1, p.S, p.G);
  if (pos >= end) return;
  int b = find_complex(p, pos, 1);
  while (pos < end) {
    const int64_t gb = cum_elems(p, b), ge = cum_elems(p, b + 1);
    if (ge <= pos) { ++b; continue; }
    const int n0 = p.shape[3 * b], n1 = p.shape[3 * b + 1], n2 = N == 3 ? p.shape[3 * b + 2] : 1;
    const uint8_t* vol = p.intensity + gb;
    const int64_t lo = pos - gb, hi = mn64(ge, end) - gb;
    // grid position of the thread's first voxel (voxel counts of one image are
    // below 2^31, checked by wect_validate), then advanced by blockDim voxels
    // per step without division
    const uint32_t bd = blockDim.x;
    const uint32_t s0 = bd % (uint32_t)n0, s1 = (bd / (uint32_t)n0) % (uint32_t)n1;
    const uint32_t s2 = bd / ((uint32_t)n0 * (uint32_t)n1);
    uint32_t v = (uint32_t)(lo + threadIdx.x);
    int i0 = (int)(v % (uint32_t)n0), i1 = (int)((v / (uint32_t)n0) % (uint32_t)n1);
    int i2 = (int)(v / ((uint32_t)n0 * (uint32_t)n1));
    // the neighbourhood of the next voxel is loaded before the current one is
    // evaluated (past the end of the range the current one is loaded again)
    EcfNbhd<N> cur, nxt;
    if (v < (uint32_t)hi) cur.load(vol, n0, n1, n2, i0, i1, i2);
    for (; v < (uint32_t)hi; v += bd) {
      int j0 = i0 + (int)s0;
      int carry = j0 >= n0;
      j0 -= carry ? n0 : 0;
      int j1 = i1 + (int)s1 + carry;
      carry = j1 >= n1;
      j1 -= carry ? n1 : 0;
      int j2 = i2 + (int)s2 + carry;
      const bool more = v + bd < (uint32_t)hi;
      nxt.load(vol, n0, n1, n2, more ? j0 : i0, more ? j1 : i1, more ? j2 : i2);
      int x;
      const int c = ecf_owned<N, WM>(cur, n0, n1, n2, i0, i1, i2, p.include_above, x);
      if (c != 0) atomicAdd(&H[wave][x], c);
      cur = nxt;
      i0 = j0;
      i1 = j1;
      i2 = j2;
    }
    __syncthreads();
    int32_t* acc = (int32_t*)p.partial + (int64_t)b * kEcfBins;
    for (int j = threadIdx.x; j < kEcfBins; j += blockDim.x) {
      int32_t sum = 0;
      for (int w = 0; w < nw; ++w) {
        sum += H[w][j];
        H[w][j] = 0;
      }
      if (sum != 0) atomicAdd(&acc[j], sum);
    }
    __syncthreads();
    pos = gb + hi;
    if (gb + hi == ge) ++b;
  }
}

// Per image: scan its 256 sums over the intensity values (CH[i] = sum of the
// contributions at intensities <= i) and read out every threshold: a cell of
// integer value x enters at thr[q] iff x <= floor(thr[q]).
__global__ __launch_bounds__(256) void k_image_ecf_finish(Params p) {
  __shared__ int32_t CH[kEcfBins];
  const int b = blockIdx.x, j = threadIdx.x;
  CH[j] = ((const int32_t*)p.partial)[(int64_t)b * kEcfBins + j];
  __syncthreads();
  for (int o = 1; o < kEcfBins; o <<= 1) {
    const int32_t add = j >= o ? CH[j - o] : 0;
    __syncthreads();
    CH[j] += add;
    __syncthreads();
  }
  int32_t* out = (int32_t*)p.out + (int64_t)b * p.T;
  for (int q = j; q < p.T; q += blockDim.x) {
    const float t = p.thr[q];
    out[q] = t >= 0.0f ? CH[t >= 255.0f ? 255 : (int)floorf(t)] : 0;  // NaN and negative: no cell
  }
}

// First pass of the general-filter WECF: the threshold index of every filter
// value (the index step that Algorithm 1 applies to the vertex filter values),
// stored as uint8 (T < 255) or uint16.  Grid-stride over the [V, m] array;
// every block sets up the threshold search once.
template <typename VB>
__global__ __launch_bounds__(256) void k_vertex_buckets(Params p, int64_t nvals) {
  extern __shared__ __align__(16) unsigned char smem[];
  float* P = (float*)smem;
  Thr th;
  setup_thresholds(p.thr, p.T, P, th);
  VB* out = (VB*)p.vbuckets;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvals; i += stride) {
    const float h = p.fvals[i];
    int b;
    if (th.arith) {
      if (!thr_arith(h, th, b)) b = thr_near(h, b, th);
    } else if (th.fast) {
      b = thr_index<true>(h, th);
    } else {
      b = thr_index<false>(h, th);
    }
    out[i] = (VB)b;
  }
}

// ---------------------------------------------------------------------------
// device builder: the weighted Freudenthal complex of an image
// ---------------------------------------------------------------------------
//
// Images become weighted simplicial complexes through the Freudenthal
// triangulation, with vertex weights from the pixel intensities (Section
// "Background", after the weighted simplicial complex definition).  Pixel
// (i0, i1) of an n0 x n1 image is vertex i1 n0 + i0 at (axis0[i0], axis1[i1]);
// edges are the (n0-1) n1 horizontal ones (row-major), the n0 (n1-1) vertical
// ones, then the (n0-1)(n1-1) diagonals (i0,i1)-(i0+1,i1+1); triangles are
// first every {(i0,i1), (i0+1,i1), (i0+1,i1+1)}, then every
// {(i0,i1), (i0,i1+1), (i0+1,i1+1)}.

// CSR offsets of the B complexes (one block; chunked scan over the images).
__global__ __launch_bounds__(1024) void k_freudenthal_offsets(Params p, int64_t* voff, int64_t* eoff, int64_t* toff) {
  __shared__ int64_t sv[1024], se[1024], st[1024];
  const int B = p.B, tid = threadIdx.x, nt = blockDim.x;
  const int per = (B + nt - 1) / nt;
  const int b0 = min(B, tid * per), b1 = min(B, b0 + per);
  auto sizes = [&](int b, int64_t& v, int64_t& e, int64_t& t) {
    const int64_t n0 = p.shape[3 * b], n1 = p.shape[3 * b + 1];
    v = n0 * n1;
    e = (n0 - 1) * n1 + n0 * (n1 - 1) + (n0 - 1) * (n1 - 1);
    t = 2 * (n0 - 1) * (n1 - 1);
  };
  int64_t cv = 0, ce = 0, ct = 0;
  for (int b = b0; b < b1; ++b) {
    int64_t v, e, t;
    sizes(b, v, e, t);
    cv += v;
    ce += e;
    ct += t;
  }
  sv[tid] = cv;
  se[tid] = ce;
  st[tid] = ct;
  __syncthreads();
  for (int o = 1; o < nt; o <<= 1) {  // inclusive scan of the chunk totals
    const int64_t av = tid >= o ? sv[tid - o] : 0, ae = tid >= o ? se[tid - o] : 0, at = tid >= o ? st[tid - o] : 0;
    __syncthreads();
    sv[tid] += av;
    se[tid] += ae;
    st[tid] += at;
    __syncthreads();
  }
  int64_t ov = sv[tid] - cv, oe = se[tid] - ce, ot = st[tid] - ct;
  for (int b = b0; b < b1; ++b) {
    voff[b] = ov;
    eoff[b] = oe;
    toff[b] = ot;
    int64_t v, e, t;
    sizes(b, v, e, t);
    ov += v;
    oe += e;
    ot += t;
  }
  if (tid == nt - 1) {
    voff[B] = sv[tid];
    eoff[B] = se[tid];
    toff[B] = st[tid];
  }
}

// One thread per pixel: its coordinates and weight, and the edges and
// triangles it starts (those of the square to its upper right).
__global__ __launch_bounds__(256) void k_freudenthal_build(Params p, const int64_t* eoff, const int64_t* toff,
                                                           float* coords, float* vw, int32_t* edges, int32_t* tris) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < p.total_voxels; g += stride) {
    const int b = find_complex(p, g, 1);  // cum_elems = grid_off (every pixel is a vertex)
    const int64_t gb = cum_elems(p, b);
    const int n0 = p.shape[3 * b], n1 = p.shape[3 * b + 1];
    const int v = (int)(g - gb);  // local vertex id (< 2^31)
    const int i1 = v / n0, i0 = v - i1 * n0;
    const float* ax0 = p.axis + (p.axis_off ? p.axis_off[b] : 0);
    coords[2 * g] = ax0[i0];
    coords[2 * g + 1] = ax0[n0 + i1];
    vw[g] = (float)p.intensity[g];
    const int64_t H = (int64_t)(n0 - 1) * n1, Vt = (int64_t)n0 * (n1 - 1), S = (int64_t)(n0 - 1) * (n1 - 1);
    int32_t* E = edges + 2 * eoff[b];
    int32_t* F = tris + 3 * toff[b];
    if (i0 < n0 - 1) {
      const int64_t k = (int64_t)i1 * (n0 - 1) + i0;
      E[2 * k] = v;
      E[2 * k + 1] = v + 1;
    }
    if (i1 < n1 - 1) {
      const int64_t k = H + (int64_t)i1 * n0 + i0;
      E[2 * k] = v;
      E[2 * k + 1] = v + n0;
    }
    if (i0 < n0 - 1 && i1 < n1 - 1) {
      const int64_t sq = (int64_t)i1 * (n0 - 1) + i0;
      const int64_t k = H + Vt + sq;
      E[2 * k] = v;
      E[2 * k + 1] = v + n0 + 1;
      F[3 * sq] = v;
      F[3 * sq + 1] = v + 1;
      F[3 * sq + 2] = v + n0 + 1;
      F[3 * (S + sq)] = v;
      F[3 * (S + sq) + 1] = v + n0;
      F[3 * (S + sq) + 2] = v + n0 + 1;
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

size_t forward_lds_fixed(int T, int kind, int acc_bytes) {
  size_t hist = (size_t)(T + 1) * W * acc_bytes;
  size_t pairs = ((size_t)(T + 1) * 4 + 15) / 16 * 16;
  (void)kind;
  return hist + pairs + 16;
}

size_t forward_entry_bytes(int kind, int n) { return (size_t)(kind == 1 ? (n == 2 ? 8 : 12) : kMaxStride) * 4; }

size_t backward_lds_bytes(int T, int stage, int dg) {
  size_t g = (size_t)dg * (T + 1) * W * 4;
  size_t pairs = ((size_t)(T + 1) * 4 + 15) / 16 * 16;
  return g + pairs + (size_t)stage * kMaxStride * 4;
}

size_t smooth_backward_lds_bytes(int T, int stage) {
  size_t cols = (size_t)(2 * T + 1) * W * 4;
  size_t pairs = ((size_t)(T + 1) * 4 + 15) / 16 * 16;
  return cols + pairs + (size_t)stage * kSmMaxStride * 4;
}

static size_t reduce_lds_bytes(int T) {
  size_t lsz = (size_t)W * (T + 1) * 4;
  lsz = (lsz + 15) / 16 * 16;
  return lsz + (size_t)16 * W * 8;
}

template <int N, int WM, typename WT, bool SM = false>
static hipError_t launch_simp_fwd_t(const Params& p, int block, size_t lds, hipStream_t s) {
  if (hipError_t e = set_lds_limit(k_simp_fwd<N, WM, WT, SM>, lds); e != hipSuccess) return e;
  hipLaunchKernelGGL((k_simp_fwd<N, WM, WT, SM>), dim3(p.G), dim3(block), lds, s, p);
  return hipGetLastError();
}

template <int N, int WM>
static hipError_t launch_cub_fwd_t(const Params& p, int block, size_t lds, hipStream_t s) {
  if (hipError_t e = set_lds_limit(k_cub_fwd<N, WM>, lds); e != hipSuccess) return e;
  hipLaunchKernelGGL((k_cub_fwd<N, WM>), dim3(p.G), dim3(block), lds, s, p);
  return hipGetLastError();
}

template <int N>
static hipError_t launch_simp_fwd_n(const Params& p, int block, size_t lds, hipStream_t s) {
  if constexpr (N > 0) {
    if (p.smooth) {
      if (p.wmode == WM_ONES) return launch_simp_fwd_t<N, WM_ONES, float, true>(p, block, lds, s);
      if (p.wmode == WM_EXPLICIT) return launch_simp_fwd_t<N, WM_EXPLICIT, float, true>(p, block, lds, s);
      return launch_simp_fwd_t<N, WM_VMAX, float, true>(p, block, lds, s);
    }
  }
  if (p.wmode == WM_ONES) return launch_simp_fwd_t<N, WM_ONES, uint32_t>(p, block, lds, s);
  if (p.wmode == WM_EXPLICIT) {
    if (p.dtype == 0) return launch_simp_fwd_t<N, WM_EXPLICIT, uint32_t>(p, block, lds, s);
    return launch_simp_fwd_t<N, WM_EXPLICIT, float>(p, block, lds, s);
  }
  return launch_simp_fwd_t<N, WM_VMAX, float>(p, block, lds, s);
}

hipError_t launch_forward_main(const Params& p, int block, size_t lds, hipStream_t s) {
  if (p.kind == 1) {
    if (p.n == 2) return p.wmode == WM_ONES ? launch_cub_fwd_t<2, WM_ONES>(p, block, lds, s)
                                            : launch_cub_fwd_t<2, WM_VMAX>(p, block, lds, s);
    return p.wmode == WM_ONES ? launch_cub_fwd_t<3, WM_ONES>(p, block, lds, s)
                              : launch_cub_fwd_t<3, WM_VMAX>(p, block, lds, s);
  }
  switch (p.n) {
    case 0: return launch_simp_fwd_n<0>(p, block, lds, s);  // general vertex filter
    case 1: return launch_simp_fwd_n<1>(p, block, lds, s);
    case 2: return launch_simp_fwd_n<2>(p, block, lds, s);
    default: return launch_simp_fwd_n<3>(p, block, lds, s);
  }
}

template <typename ACC>
static hipError_t launch_reduce_t(const Params& p, hipStream_t s) {
  const int groups = p.B * p.ntiles;
  if (p.split) {
    hipLaunchKernelGGL(k_slot_sum<ACC>, dim3(groups, (p.T + 3) / 4), dim3(256), 0, s, p);
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  }
  const size_t lds = reduce_lds_bytes(p.T);
  if (hipError_t e = set_lds_limit(k_reduce_scan<ACC>, lds); e != hipSuccess) return e;
  hipLaunchKernelGGL((k_reduce_scan<ACC>), dim3(groups), dim3(1024), lds, s, p);
  return hipGetLastError();
}

hipError_t launch_forward_reduce(const Params& p, hipStream_t s) {
  if (p.group_mode) return hipSuccess;  // every block wrote its group's output
  const bool wide = p.kind == 0 && p.dtype == 1;
  return wide ? launch_reduce_t<uint64_t>(p, s) : launch_reduce_t<uint32_t>(p, s);
}

hipError_t launch_absmax(const Params& p, hipStream_t s) {
  hipLaunchKernelGGL(k_absmax, dim3(p.nabsmax / 4, 4), dim3(256), 0, s, p);
  return hipGetLastError();
}

template <int N, int WM>
static hipError_t launch_bwd_t(const Params& p, int block, size_t lds, hipStream_t s) {
  if (hipError_t e = set_lds_limit(k_simp_bwd<N, WM>, lds); e != hipSuccess) return e;
  hipLaunchKernelGGL((k_simp_bwd<N, WM>), dim3(p.G), dim3(block), lds, s, p);
  return hipGetLastError();
}

hipError_t launch_backward_main(const Params& p, int block, size_t lds, hipStream_t s) {
  const bool vm = p.wmode == WM_VMAX;
  switch (p.n) {
    case 0: return vm ? launch_bwd_t<0, WM_VMAX>(p, block, lds, s) : launch_bwd_t<0, WM_EXPLICIT>(p, block, lds, s);
    case 1: return vm ? launch_bwd_t<1, WM_VMAX>(p, block, lds, s) : launch_bwd_t<1, WM_EXPLICIT>(p, block, lds, s);
    case 2: return vm ? launch_bwd_t<2, WM_VMAX>(p, block, lds, s) : launch_bwd_t<2, WM_EXPLICIT>(p, block, lds, s);
    default: return vm ? launch_bwd_t<3, WM_VMAX>(p, block, lds, s) : launch_bwd_t<3, WM_EXPLICIT>(p, block, lds, s);
  }
}

template <int N, int WM>
static hipError_t launch_sm_bwd_t(const Params& p, int block, size_t lds, hipStream_t s) {
  if (hipError_t e = set_lds_limit(k_smooth_bwd<N, WM>, lds); e != hipSuccess) return e;
  hipLaunchKernelGGL((k_smooth_bwd<N, WM>), dim3(p.G), dim3(block), lds, s, p);
  return hipGetLastError();
}

template <int N>
static hipError_t launch_sm_bwd_n(const Params& p, int block, size_t lds, hipStream_t s) {
  if (p.wmode == WM_ONES) return launch_sm_bwd_t<N, WM_ONES>(p, block, lds, s);
  if (p.wmode == WM_EXPLICIT) return launch_sm_bwd_t<N, WM_EXPLICIT>(p, block, lds, s);
  return launch_sm_bwd_t<N, WM_VMAX>(p, block, lds, s);
}

hipError_t launch_smooth_backward(const Params& p, int block, size_t lds, hipStream_t s) {
  switch (p.n) {
    case 1: return launch_sm_bwd_n<1>(p, block, lds, s);
    case 2: return launch_sm_bwd_n<2>(p, block, lds, s);
    default: return launch_sm_bwd_n<3>(p, block, lds, s);
  }
}

LsLayout ls_layout(int64_t V, const int64_t count[4], int top_dim) {
  LsLayout L;
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  L.nent = 0;
  for (int d = 1; d <= top_dim; ++d) L.nent += (int64_t)(d + 1) * count[d];
  L.nparts = V > 0 ? (V + kLsChunk - 1) / kLsChunk : 1;
  L.hdr = 0;
  L.off = L.hdr + al(4 * 8);
  L.cur = L.off + al((size_t)(V + 1) * 8);
  L.part = L.cur + al((size_t)V * 8);
  L.ent = L.part + al((size_t)L.nparts * 8);
  L.row = L.ent + al((size_t)L.nent * 16);
  L.mask = L.row + al((size_t)L.nent * 8);
  L.nbc = L.mask + al((size_t)L.nent * 4);
  L.total = L.nbc + al((size_t)V * 4);
  return L;
}

void ls_bind(Params& p, void* base, const LsLayout& L) {
  unsigned char* b = static_cast<unsigned char*>(base);
  p.ls_hdr = (int64_t*)(b + L.hdr);
  p.ls_off = (int64_t*)(b + L.off);
  p.ls_cur = (int64_t*)(b + L.cur);
  p.ls_part = (int64_t*)(b + L.part);
  p.ls_ent = (int32_t*)(b + L.ent);
  p.ls_row = (int64_t*)(b + L.row);
  p.ls_mask = (uint32_t*)(b + L.mask);
  p.ls_nbc = (int32_t*)(b + L.nbc);
}

hipError_t launch_lower_star_build(const Params& p, const LsLayout& L, hipStream_t s) {
  const int64_t V = p.count[0];
  // header and counts start at zero (fill kernels: capture-safe)
  if (hipError_t e = launch_fill_zero((float*)p.ls_hdr, 8, s); e != hipSuccess) return e;
  if (hipError_t e = launch_fill_zero((float*)p.ls_cur, 2 * V, s); e != hipSuccess) return e;
  if (V == 0) return launch_fill_zero((float*)p.ls_off, 2, s);
  int64_t kmax = 0;
  for (int d = 1; d <= p.top_dim; ++d) kmax = kmax > p.count[d] ? kmax : p.count[d];
  const unsigned gb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(8192, (kmax + 255) / 256));
  hipLaunchKernelGGL(k_ls_count, dim3(gb), dim3(256), 0, s, p);
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ls_scan_parts, dim3((unsigned)L.nparts), dim3(256), 0, s, p);
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ls_scan_top, dim3(1), dim3(1024), 0, s, p, L.nparts);
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ls_scan_apply, dim3((unsigned)L.nparts), dim3(256), 0, s, p);
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  const unsigned gv = (unsigned)std::max<int64_t>(1, std::min<int64_t>(8192, (V + 255) / 256));
  for (int d = 1; d <= p.top_dim; ++d) {
    hipLaunchKernelGGL(k_ls_fill, dim3(gb), dim3(256), 0, s, p, d);
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
    if (d == 1) {
      hipLaunchKernelGGL(k_ls_edge_counts, dim3(gv), dim3(256), 0, s, p);
      if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
    }
  }
  if (p.top_dim < 1) {  // no edges: every vertex has nbc = 0
    hipLaunchKernelGGL(k_ls_edge_counts, dim3(gv), dim3(256), 0, s, p);
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  }
  return hipSuccess;
}

// LDS of the vertex-centric kernels: the histogram (forward: uint64 [T+1][W];
// adjoint: float g and G columns), the thresholds, and per wavefront `rows`
// coface rows plus the vertex rows.  64 rows per wavefront, or 32 when 64
// would not fit (long threshold arrays): half the rows, twice the wavefronts.
static size_t ls_lds(int T, int block, int rows, bool bwd) {
  const size_t hist = bwd ? (size_t)(2 * T + 1) * W * 4 : (size_t)(T + 1) * W * 8;
  return hist + ((size_t)(T + 1) * 4 + 15) / 16 * 16 + (size_t)(block / W) * (rows * kLsStride + 4 * kLsGroup) * 4;
}
static int ls_rows(int T, int block, bool bwd) {
  return ls_lds(T, block, kLsRows, bwd) <= kLdsBudget ? kLsRows : kLsRows / 2;
}

size_t smooth_ls_forward_lds_bytes(int T, int block) { return ls_lds(T, block, ls_rows(T, block, false), false); }

size_t smooth_ls_backward_lds_bytes(int T, int block) { return ls_lds(T, block, ls_rows(T, block, true), true); }

template <int N, int WM>
static hipError_t launch_ls_fwd_t(const Params& p, int block, size_t lds, hipStream_t s) {
  if (hipError_t e = set_lds_limit(k_smooth_ls_fwd<N, WM>, lds); e != hipSuccess) return e;
  hipLaunchKernelGGL((k_smooth_ls_fwd<N, WM>), dim3(p.G), dim3(block), lds, s, p, ls_rows(p.T, block, false));
  return hipGetLastError();
}

template <int N, int WM>
static hipError_t launch_ls_bwd_t(const Params& p, int block, size_t lds, hipStream_t s) {
  if (hipError_t e = set_lds_limit(k_smooth_ls_bwd<N, WM>, lds); e != hipSuccess) return e;
  hipLaunchKernelGGL((k_smooth_ls_bwd<N, WM>), dim3(p.G), dim3(block), lds, s, p, ls_rows(p.T, block, true));
  return hipGetLastError();
}

template <int N>
static hipError_t launch_ls_n(const Params& p, int block, size_t lds, hipStream_t s, bool bwd) {
  if (p.wmode == WM_ONES) return bwd ? launch_ls_bwd_t<N, WM_ONES>(p, block, lds, s)
                                     : launch_ls_fwd_t<N, WM_ONES>(p, block, lds, s);
  if (p.wmode == WM_EXPLICIT) return bwd ? launch_ls_bwd_t<N, WM_EXPLICIT>(p, block, lds, s)
                                         : launch_ls_fwd_t<N, WM_EXPLICIT>(p, block, lds, s);
  return bwd ? launch_ls_bwd_t<N, WM_VMAX>(p, block, lds, s) : launch_ls_fwd_t<N, WM_VMAX>(p, block, lds, s);
}

hipError_t launch_smooth_ls_forward(const Params& p, int block, size_t lds, hipStream_t s) {
  switch (p.n) {
    case 1: return launch_ls_n<1>(p, block, lds, s, false);
    case 2: return launch_ls_n<2>(p, block, lds, s, false);
    default: return launch_ls_n<3>(p, block, lds, s, false);
  }
}

hipError_t launch_smooth_ls_backward(const Params& p, int block, size_t lds, hipStream_t s) {
  switch (p.n) {
    case 1: return launch_ls_n<1>(p, block, lds, s, true);
    case 2: return launch_ls_n<2>(p, block, lds, s, true);
    default: return launch_ls_n<3>(p, block, lds, s, true);
  }
}

hipError_t launch_fill_zero(float* ptr, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, ptr, n);
  return hipGetLastError();
}

hipError_t launch_image_ecf(const Params& p, int block, hipStream_t s) {
  // clear the [B][256] accumulator with a kernel (no memset node in a captured graph)
  if (hipError_t e = launch_fill_zero((float*)p.partial, (int64_t)p.B * kEcfBins, s); e != hipSuccess) return e;
  if (p.S > 0) {
    const bool vm = p.wmode == WM_VMAX;
    if (p.n == 2) {
      if (vm) hipLaunchKernelGGL((k_image_ecf<2, WM_VMAX>), dim3(p.G), dim3(block), 0, s, p);
      else hipLaunchKernelGGL((k_image_ecf<2, WM_ONES>), dim3(p.G), dim3(block), 0, s, p);
    } else {
      if (vm) hipLaunchKernelGGL((k_image_ecf<3, WM_VMAX>), dim3(p.G), dim3(block), 0, s, p);
      else hipLaunchKernelGGL((k_image_ecf<3, WM_ONES>), dim3(p.G), dim3(block), 0, s, p);
    }
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_image_ecf_finish, dim3(p.B), dim3(kEcfBins), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_vertex_buckets(const Params& p, int64_t nvals, hipStream_t s) {
  if (nvals <= 0) return hipSuccess;
  const size_t lds = ((size_t)(p.T + 1) * 4 + 15) / 16 * 16;
  int64_t blocks = (nvals + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (p.vb_bytes == 1) {
    if (hipError_t e = set_lds_limit(k_vertex_buckets<uint8_t>, lds); e != hipSuccess) return e;
    hipLaunchKernelGGL(k_vertex_buckets<uint8_t>, dim3((unsigned)blocks), dim3(256), lds, s, p, nvals);
  } else {
    if (hipError_t e = set_lds_limit(k_vertex_buckets<uint16_t>, lds); e != hipSuccess) return e;
    hipLaunchKernelGGL(k_vertex_buckets<uint16_t>, dim3((unsigned)blocks), dim3(256), lds, s, p, nvals);
  }
  return hipGetLastError();
}

hipError_t launch_freudenthal(const Params& p, int64_t* voff, int64_t* eoff, int64_t* toff, float* coords,
                              float* vw, int32_t* edges, int32_t* tris, hipStream_t s) {
  hipLaunchKernelGGL(k_freudenthal_offsets, dim3(1), dim3(1024), 0, s, p, voff, eoff, toff);
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  if (p.total_voxels <= 0) return hipSuccess;
  int64_t blocks = (p.total_voxels + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_freudenthal_build, dim3((unsigned)blocks), dim3(256), 0, s, p, eoff, toff, coords, vw, edges,
                     tris);
  return hipGetLastError();
}

hipError_t launch_validate(const Params& p, int* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_validate, dim3(256, 4), dim3(256), 0, s, p, flags);
  return hipGetLastError();
}

}  // namespace wect
