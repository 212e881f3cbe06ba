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
  float ka;         // arithmetic index: t = fma(h, c, ka) puts thr[q] near q + 1
  float tmax;       // T + 0.5
  float half_open;  // 0.5 - delta (see thr_arith)
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
    const int g = guess(h, th.c, th.k, th.T);
    return g - (h <= th.P[g] ? 1 : 0);
  }
  int lo = 0;
  for (int s = th.p2; s > 0; s >>= 1) {
    int cand = lo + s;
    if (cand <= th.T && th.P[cand] < h) lo = cand;  // P[cand] == thr[cand-1]
  }
  return lo;
}

// Index from the affine map alone.  With x(h) = h c + ka (exact, strictly
// increasing) and tau_q = x(thr[q]), L(h) = #{q : tau_q < x(h)}.  The stored
// thresholds satisfy |tau_q - (q+1)| <= dev and t = fl(x(h)) is within
// 2^-24 (T+2) <= delta/2 of x(h) (delta = 2 dev + 2^-23 (T+2) + 1e-7, measured
// when the block starts).  When frac(t) is further than delta from 0 and 1,
// every tau_q with q+1 <= floor(t) lies below x(h) and every other one above,
// so L = clamp(floor(t), 0, T).  Otherwise h is within 2 delta of one position
// m = round(t) and only thr[m-1] can be on either side: L = m - [h <= thr[m-1]].
__device__ __forceinline__ bool thr_arith(float h, const Thr& th, int& b, float& t) {
  t = __builtin_fmaf(h, th.c, th.ka);
  t = __builtin_amdgcn_fmed3f(t, -0.5f, th.tmax);
  const float fr = __builtin_amdgcn_fractf(t);
  b = max((int)(t - fr), 0);
  return fabsf(fr - 0.5f) < th.half_open;
}

__device__ __forceinline__ int thr_near(float h, float t, const Thr& th) {
  const int m = min((int)rintf(t), th.T);
  return m - (h <= th.P[m] ? 1 : 0);
}

// Per-wavefront choice between the arithmetic index (no LDS read unless a lane
// sits on a threshold) and the one-read guess: images whose pixel lattice is
// commensurate with the threshold grid put many heights exactly on thresholds
// for some directions; a wavefront that needs the near-threshold fix in more
// than 8 of 32 consecutive pairs switches to the guess for the rest of its range.
struct IndexMode {
  int arith, pairs, fallbacks;
};

template <bool FAST>
__device__ __forceinline__ void thr_index2(float h0, float h1, const Thr& th, int& b0, int& b1, IndexMode& md) {
  if constexpr (FAST) {
    if (md.arith) {
      float t0, t1;
      const bool ok0 = thr_arith(h0, th, b0, t0);
      const bool ok1 = thr_arith(h1, th, b1, t1);
      if (__builtin_amdgcn_ballot_w64(!(ok0 && ok1)) != 0) {
        ++md.fallbacks;
        if (!ok0) b0 = thr_near(h0, t0, th);
        if (!ok1) b1 = thr_near(h1, t1, th);
      }
      if (++md.pairs == 32) {
        if (md.fallbacks > 8) md.arith = 0;
        md.pairs = 0;
        md.fallbacks = 0;
      }
      return;
    }
  }
  b0 = thr_index<FAST>(h0, th);
  b1 = thr_index<FAST>(h1, th);
}

// Block prologue: stage P in LDS and decide whether the fast path is exact
// for this threshold array.  g is monotone in h and L is constant on
// (thr[q], thr[q+1]], so g(thr[q]) in {q, q+1} and g(next float above thr[q])
// in {q+1, q+2} (clamped to T) for every q give g in {L, L+1} everywhere
// (strictly increasing thresholds required).
__device__ void setup_thresholds(const float* thr, int T, float* P, Thr& th) {
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
  // arithmetic index: distance of the stored thresholds from their positions
  __shared__ double s_dev[16];
  const float ka = ok ? 1.0f - thr[0] * c : 0.0f;
  double dev = 0.0;
  if (ok && !bad) {
    for (int q = threadIdx.x; q < T; q += blockDim.x) {
      const double tau = (double)thr[q] * (double)c + (double)ka;  // exact product, one rounding
      dev = fmax(dev, fabs(tau - (double)(q + 1)));
    }
  }
  for (int o = 32; o > 0; o >>= 1) dev = fmax(dev, __shfl_xor(dev, o));
  if ((threadIdx.x & 63) == 0) s_dev[threadIdx.x >> 6] = dev;
  __syncthreads();
  dev = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) dev = fmax(dev, s_dev[w]);
  const double delta = 2.0 * dev + ldexp(1.0, -23) * (T + 2) + 1e-7;
  th.P = P;
  th.c = c;
  th.k = k;
  th.ka = ka;
  th.tmax = (float)T + 0.5f;
  th.half_open = (float)(0.5 - delta);
  th.T = T;
  th.p2 = p2;
  th.fast = ok && !bad;
  th.arith = th.fast && delta < 0.25;
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

// ---------------------------------------------------------------------------
// stream bookkeeping
// ---------------------------------------------------------------------------

// Number of stream elements (cells handled one by one) of the complexes
// before complex b: all simplices of all dimensions, or all voxels.
__device__ __forceinline__ int64_t cum_elems(const Params& p, int b) {
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
__device__ int find_complex(const Params& p, int64_t pos, int gpc) {
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

template <int N, int DIM, typename ACC>
struct SimpLayout {
  static constexpr int NV = DIM + 1;
  static constexpr int WW = sizeof(ACC) / 4;                 // words of the staged weight
  static constexpr int WOFF = ((NV * N + WW - 1) / WW) * WW;  // weight slot, aligned to its size
  static constexpr int OOFF = WOFF + WW;                     // owner slot (vertex-max backward)
  static constexpr int STRIDE = ((OOFF + 1 + 3) / 4) * 4;
  static_assert(STRIDE <= kMaxStride, "entry too large");
};

// Exponent e of the fixed-point scale 2^e for float32 weights: with M the
// largest |w| and C the number of cells, every sum of rounded weights stays
// below C * (M 2^e + 1/2) < 2^63.  Computed identically by every block from
// the per-block maxima written by k_absmax.
__device__ __forceinline__ int fixed_exp(const Params& p) {
  float M = 0.0f;
  for (int i = 0; i < p.nabsmax; ++i) M = fmaxf(M, p.absmax[i]);
  const double X = (double)M * p.cells_total;
  if (!(X > 0.0) || !isfinite(X)) return 0;
  int ex = 0;
  (void)frexp(X, &ex);  // X = f 2^ex, f in [0.5, 1): floor(log2 X) = ex - 1
  return 61 - (ex - 1);
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
  // coordinates, signed weight and owner vertex of the simplex whose ids are in idx
  __device__ __forceinline__ void gather(const Params& p, int64_t row, int64_t voff, int fexp) {
#pragma unroll
    for (int j = 0; j < L::NV; ++j) {
      const float* c = p.coords + (voff + idx[j]) * N;
#pragma unroll
      for (int k = 0; k < N; ++k) e[j * N + k] = c[k];
    }
#pragma unroll
    for (int k = L::NV * N; k < L::WOFF; ++k) e[k] = 0.0f;
    e[L::OOFF] = 0.0f;
    if constexpr (WM == WM_ONES) {
      if constexpr (FWD) put_weight(ACC(1));
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

// Forward over the simplices [lo, hi) (local numbering) of dimension DIM of
// one complex: stage TS simplices at a time, then every wavefront adds its
// share of them to the LDS histogram.  Indices are prefetched one tile ahead
// of the coordinate gather, which runs one tile ahead of the histogram.
template <int N, int DIM, int WM, typename WT, bool FAST>
__device__ void simp_fwd_range(const Params& p, int64_t lo, int64_t hi, int64_t voff, int64_t soff,
                               float sx, float sy, float sz, typename AccOf<WT>::T* hist, float* stage,
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
  IndexMode md = {th.arith, 0, 0};
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
    int e = 2 * wave;
    for (; e + 1 < cnt; e += 2 * nw) {
      const float* E0 = stage + e * L::STRIDE;
      const float* E1 = E0 + L::STRIDE;
      float h0 = max_height<N, DIM>(E0, sx, sy, sz);
      float h1 = max_height<N, DIM>(E1, sx, sy, sz);
      ACC w0 = load_weight<ACC>(E0 + L::WOFF);
      ACC w1 = load_weight<ACC>(E1 + L::WOFF);
      int b0, b1;
      thr_index2<FAST>(h0, h1, th, b0, b1, md);
      lds_add(&hist[b0 * W + lane], w0);
      lds_add(&hist[b1 * W + lane], w1);
    }
    if (e < cnt) {
      const float* E0 = stage + e * L::STRIDE;
      float h0 = max_height<N, DIM>(E0, sx, sy, sz);
      ACC w0 = load_weight<ACC>(E0 + L::WOFF);
      int b0 = thr_index<FAST>(h0, th);
      lds_add(&hist[b0 * W + lane], w0);
    }
  }
  __syncthreads();
}

template <int N, int WM, typename WT, bool FAST>
__device__ __forceinline__ void simp_fwd_dim(int dim, const Params& p, int64_t lo, int64_t hi, int64_t voff,
                                             int64_t soff, float sx, float sy, float sz,
                                             typename AccOf<WT>::T* hist, float* stage, const Thr& th, int fexp) {
  switch (dim) {
    case 0: simp_fwd_range<N, 0, WM, WT, FAST>(p, lo, hi, voff, soff, sx, sy, sz, hist, stage, th, fexp); break;
    case 1: simp_fwd_range<N, 1, WM, WT, FAST>(p, lo, hi, voff, soff, sx, sy, sz, hist, stage, th, fexp); break;
    case 2: simp_fwd_range<N, 2, WM, WT, FAST>(p, lo, hi, voff, soff, sx, sy, sz, hist, stage, th, fexp); break;
    default: simp_fwd_range<N, 3, WM, WT, FAST>(p, lo, hi, voff, soff, sx, sy, sz, hist, stage, th, fexp); break;
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

__device__ __forceinline__ void load_dir(const Params& p, int gp, float& sx, float& sy, float& sz) {
  sx = sy = sz = 0.0f;
  if (gp < p.d) {
    const float* s = p.dirs + (int64_t)gp * p.n;
    sx = s[0];
    if (p.n >= 2) sy = s[1];
    if (p.n >= 3) sz = s[2];
  }
}

__device__ __forceinline__ size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------------------
// forward, simplicial
// ---------------------------------------------------------------------------

template <int N, int WM, typename WT>
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
  int64_t pos = block_start(k, p.S, p.G);
  const int64_t end = block_start(k + 1, p.S, p.G);
  if (pos >= end) return;
  const int gpc = p.ntiles;
  int b = find_complex(p, pos, gpc);
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
          simp_fwd_dim<N, WM, WT, true>(dim, p, lo - dlo, hi - dlo, voff, soff, sx, sy, sz, hist, stage, th, fexp);
        else
          simp_fwd_dim<N, WM, WT, false>(dim, p, lo - dlo, hi - dlo, voff, soff, sx, sy, sz, hist, stage, th, fexp);
      }
      dlo = dhi;
    }
    flush_hist<ACC>(p, hist, (int64_t)k + (int64_t)b * gpc + t);
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

// A cell around the staged vertex v: mx = largest corner intensity, mn =
// smallest corner value, where a corner that is not a vertex counts as -1; the
// cell exists iff mn >= 0.
struct CubCell {
  int mx, mn;
};

__device__ __forceinline__ CubCell cub_join(CubCell a, int x) { return {max(a.mx, x), min(a.mn, x)}; }
__device__ __forceinline__ CubCell cub_join(CubCell a, CubCell b) { return {max(a.mx, b.mx), min(a.mn, b.mn)}; }

template <int WM>
__device__ __forceinline__ int cub_val(CubCell c) {
  return c.mn >= 0 ? (WM == WM_ONES ? 1 : c.mx) : 0;
}

// Combined weights of vertex (i0,i1,i2) for the 2^N orthants.  Orthant bit k
// set means s_k < 0: the cells topped by v then extend towards +k, otherwise
// towards -k.  Each distinct cell containing v (2N edges, the squares of each
// axis pair, the 2^N cubes) is evaluated once.
template <int N, int WM>
__device__ __forceinline__ void cub_weights(const Params& p, const uint8_t* vol, int n0, int n1, int n2,
                                            int i0, int i1, int i2, int32_t* cw) {
  constexpr int M = N == 2 ? 9 : 27;
  int nb[M];
  const int thr = p.include_above;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int d0 = m % 3 - 1, d1 = (m / 3) % 3 - 1, d2 = N == 3 ? m / 9 - 1 : 0;
    const int j0 = i0 + d0, j1 = i1 + d1, j2 = i2 + d2;
    int v = -1;
    if (j0 >= 0 && j0 < n0 && j1 >= 0 && j1 < n1 && j2 >= 0 && j2 < n2) {
      int x = vol[((int64_t)j2 * n1 + j1) * n0 + j0];
      v = x > thr ? x : -1;
    }
    nb[m] = v;
  }
  auto at = [&](int d0, int d1, int d2) { return nb[(d0 + 1) + 3 * (d1 + 1) + (N == 3 ? 9 * (d2 + 1) : 0)]; };
  const int v0 = at(0, 0, 0);
  const CubCell cv = {v0, v0};
  // edges E[axis][side], side 0: towards -axis, 1: towards +axis
  CubCell E[N][2];
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      const int s = sd ? 1 : -1;
      E[a][sd] = cub_join(cv, at(a == 0 ? s : 0, a == 1 ? s : 0, a == 2 ? s : 0));
    }
  if constexpr (N == 2) {
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      const int s0 = o & 1, s1 = (o >> 1) & 1;
      const CubCell sq = cub_join(cub_join(E[0][s0], E[1][s1]), at(s0 ? 1 : -1, s1 ? 1 : -1, 0));
      cw[o] = cub_val<WM>(cv) - cub_val<WM>(E[0][s0]) - cub_val<WM>(E[1][s1]) + cub_val<WM>(sq);
    }
  } else {
    // squares F01[s0][s1], F02[s0][s2], F12[s1][s2]
    CubCell F01[2][2], F02[2][2], F12[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int sa = a ? 1 : -1, sb = b ? 1 : -1;
        F01[a][b] = cub_join(cub_join(E[0][a], E[1][b]), at(sa, sb, 0));
        F02[a][b] = cub_join(cub_join(E[0][a], E[2][b]), at(sa, 0, sb));
        F12[a][b] = cub_join(cub_join(E[1][a], E[2][b]), at(0, sa, sb));
      }
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      const int s0 = o & 1, s1 = (o >> 1) & 1, s2 = (o >> 2) & 1;
      // the cube's 8 corners: F01 and F12 cover six of them; add the 0-2 diagonal and the far corner
      const CubCell cube = cub_join(cub_join(cub_join(F01[s0][s1], F12[s1][s2]), at(s0 ? 1 : -1, 0, s2 ? 1 : -1)),
                                    at(s0 ? 1 : -1, s1 ? 1 : -1, s2 ? 1 : -1));
      cw[o] = cub_val<WM>(cv) - cub_val<WM>(E[0][s0]) - cub_val<WM>(E[1][s1]) - cub_val<WM>(E[2][s2]) +
              cub_val<WM>(F01[s0][s1]) + cub_val<WM>(F02[s0][s2]) + cub_val<WM>(F12[s1][s2]) - cub_val<WM>(cube);
    }
  }
}

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
  IndexMode md = {th.arith, 0, 0};
  for (int64_t t0 = lo; t0 < hi; t0 += TS) {
    const int cnt = (int)mn64(TS, hi - t0);
    if (tid == 0) *counter = 0;
    __syncthreads();
    bool keep = false;
    float cx = 0.0f, cy = 0.0f, cz = 0.0f;
    int32_t cw[L::NO];
    if (tid < cnt) {
      // voxel counts of one complex are below 2^31 (checked by wect_validate)
      const uint32_t v = (uint32_t)(t0 + tid);
      const uint32_t r = v / (uint32_t)n0;
      const int i0 = (int)(v - r * (uint32_t)n0);
      const uint32_t i2u = r / (uint32_t)n1;
      const int i1 = (int)(r - i2u * (uint32_t)n1);
      const int i2 = (int)i2u;
      if ((int)vol[v] > p.include_above) {
        cub_weights<N, WM>(p, vol, n0, n1, n2, i0, i1, i2, cw);
        bool nz = false;
#pragma unroll
        for (int o = 0; o < L::NO; ++o) nz = nz || (cw[o] != 0);
        keep = nz;
        cx = ax0[i0];
        cy = ax1[i1];
        if constexpr (N == 3) cz = ax2[i2];
      }
    }
    // compact the contributing vertices
    const uint64_t bal = __ballot(keep);
    int base = 0;
    if (lane == 0 && bal) base = atomicAdd(counter, __popcll(bal));
    base = __shfl(base, 0);
    if (keep) {
      const int slot = base + __popcll(bal & ((1ull << lane) - 1ull));
      float* E = stage + slot * L::STRIDE;
      E[0] = cx;
      E[1] = cy;
      if constexpr (N == 3) { E[2] = cz; E[3] = 0.0f; }
#pragma unroll
      for (int o = 0; o < L::NO; ++o) E[L::COFF + o] = bitcast<float>(cw[o]);
    }
    __syncthreads();
    const int ne = uniform(*counter);
    const float* Wl = stage + L::COFF + orth;  // the lane's combined weight within an entry
    int e = 2 * wave;
    for (; e + 1 < ne; e += 2 * nw) {
      const float* E0 = stage + e * L::STRIDE;
      const float* E1 = E0 + L::STRIDE;
      float h0 = height<N>(E0, sx, sy, sz);
      float h1 = height<N>(E1, sx, sy, sz);
      uint32_t w0 = bitcast<uint32_t>(Wl[e * L::STRIDE]);
      uint32_t w1 = bitcast<uint32_t>(Wl[e * L::STRIDE + L::STRIDE]);
      int b0, b1;
      thr_index2<FAST>(h0, h1, th, b0, b1, md);
      lds_add(&hist[b0 * W + lane], w0);
      lds_add(&hist[b1 * W + lane], w1);
    }
    if (e < ne) {
      const float* E0 = stage + e * L::STRIDE;
      float h0 = height<N>(E0, sx, sy, sz);
      uint32_t w0 = bitcast<uint32_t>(Wl[e * L::STRIDE]);
      int b0 = thr_index<FAST>(h0, th);
      lds_add(&hist[b0 * W + lane], w0);
    }
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
  int64_t pos = block_start(k, p.S, p.G);
  const int64_t end = block_start(k + 1, p.S, p.G);
  if (pos >= end) return;
  const int gpc = p.ntiles;
  int b = find_complex(p, pos, gpc);
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
    flush_hist<uint32_t>(p, hist, (int64_t)k + (int64_t)b * gpc + t);
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

// Per group (complex, direction tile): sum its slots (or read its dsum row),
// scan along the thresholds (cumulative sum of Algorithm 1,
// out[b][p][q] = sum_{j <= q} D[p][j]) and write the 64 x T block of out.
// 16 row chunks x 64 lanes: each thread keeps its chunk in registers.
template <typename ACC, int CH>
__global__ __launch_bounds__(1024) void k_reduce_scan(Params p) {
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

  ACC acc[CH];
#pragma unroll
  for (int j = 0; j < CH; ++j) acc[j] = 0;
  if (r < 16 && nq > 0) {
    const int64_t slot_stride = (int64_t)T * W;
    int64_t kfirst, klast;
    group_slots(p, g, kfirst, klast);
    // rows q0 .. q0+nq-1 of this thread; loads use clamped (in-range) rows and
    // the surplus values are dropped, so all CH loads of a slot are independent
    int rowoff[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) rowoff[j] = min(j, nq - 1) * W;
    if (p.split && klast - kfirst + 1 > kFusedSlots) {
      const ACC* src = (const ACC*)p.dsum + (int64_t)g * slot_stride + (int64_t)q0 * W + lane;
#pragma unroll
      for (int j = 0; j < CH; ++j) acc[j] = src[rowoff[j]];
    } else {
      for (int64_t kk = kfirst; kk <= klast; ++kk) {
        const ACC* src = (const ACC*)p.partial + (kk + g) * slot_stride + (int64_t)q0 * W + lane;
        ACC v[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) v[j] = src[rowoff[j]];
#pragma unroll
        for (int j = 0; j < CH; ++j) acc[j] += v[j];
      }
    }
#pragma unroll
    for (int j = 0; j < CH; ++j)
      if (j >= nq) acc[j] = 0;
  }
  ACC run = 0;
#pragma unroll
  for (int j = 0; j < CH; ++j) {
    run += acc[j];
    acc[j] = run;
  }
  if (r < 16) tot[r * W + lane] = run;
  __syncthreads();
  ACC off = 0;
  for (int rr = 0; rr < r && rr < 16; ++rr) off += tot[rr * W + lane];
  if (r < 16) {
#pragma unroll
    for (int j = 0; j < CH; ++j)
      if (j < nq) L[lane * LS + q0 + j] = O::conv(acc[j] + off, fexp);
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
__device__ void simp_bwd_range(const Params& p, int b, int64_t lo, int64_t hi, int64_t voff, int64_t soff,
                               const float* sx, const float* sy, const float* sz, int ntl,
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
    for (int j = 0; j < ne; ++j) {
      const float* E = stage + (e0 + j) * L::STRIDE;
      float acc = 0.0f;
#pragma unroll
      for (int jj = 0; jj < kMaxDG; ++jj) {
        if (jj < ntl) {
          const float h = max_height<N, DIM>(E, sx[jj], sy[jj], sz[jj]);
          const int bi = thr_index<FAST>(h, th);
          acc += Gt[((size_t)jj * T1 + bi) * W + lane];
        }
      }
      const float tot = wave_sum(acc);
      mine = lane == j ? tot : mine;
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
                                             const float* Gt, float* stage, const Thr& th) {
  switch (dim) {
    case 0: simp_bwd_range<N, 0, WM, FAST>(p, b, lo, hi, voff, soff, sx, sy, sz, ntl, Gt, stage, th); break;
    case 1: simp_bwd_range<N, 1, WM, FAST>(p, b, lo, hi, voff, soff, sx, sy, sz, ntl, Gt, stage, th); break;
    case 2: simp_bwd_range<N, 2, WM, FAST>(p, b, lo, hi, voff, soff, sx, sy, sz, ntl, Gt, stage, th); break;
    default: simp_bwd_range<N, 3, WM, FAST>(p, b, lo, hi, voff, soff, sx, sy, sz, ntl, Gt, stage, th); break;
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
    for (int j = 0; j < kMaxDG; ++j) load_dir(p, (tile0 + j) * W + lane, sx[j], sy[j], sz[j]);
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
        if (th.fast) simp_bwd_dim<N, WM, true>(dim, p, b, lo - dlo, hi - dlo, voff, soff, sx, sy, sz, ntl, Gt, stage, th);
        else simp_bwd_dim<N, WM, false>(dim, p, b, lo - dlo, hi - dlo, voff, soff, sx, sy, sz, ntl, Gt, stage, th);
      }
      dlo = dhi;
    }
    pos += e1 - e0;
    if (e1 == nb && jg == gpc - 1) ++b;
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

static size_t reduce_lds_bytes(int T) {
  size_t lsz = (size_t)W * (T + 1) * 4;
  lsz = (lsz + 15) / 16 * 16;
  return lsz + (size_t)16 * W * 8;
}

template <int N, int WM, typename WT>
static hipError_t launch_simp_fwd_t(const Params& p, int block, size_t lds, hipStream_t s) {
  if (hipError_t e = set_lds_limit(k_simp_fwd<N, WM, WT>, lds); e != hipSuccess) return e;
  hipLaunchKernelGGL((k_simp_fwd<N, WM, WT>), dim3(p.G), dim3(block), lds, s, p);
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
    case 1: return launch_simp_fwd_n<1>(p, block, lds, s);
    case 2: return launch_simp_fwd_n<2>(p, block, lds, s);
    default: return launch_simp_fwd_n<3>(p, block, lds, s);
  }
}

template <typename ACC, int CH>
static hipError_t launch_reduce_t(const Params& p, hipStream_t s) {
  const int groups = p.B * p.ntiles;
  if (p.split) {
    hipLaunchKernelGGL(k_slot_sum<ACC>, dim3(groups, (p.T + 3) / 4), dim3(256), 0, s, p);
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  }
  const size_t lds = reduce_lds_bytes(p.T);
  if (hipError_t e = set_lds_limit(k_reduce_scan<ACC, CH>, lds); e != hipSuccess) return e;
  hipLaunchKernelGGL((k_reduce_scan<ACC, CH>), dim3(groups), dim3(1024), lds, s, p);
  return hipGetLastError();
}

hipError_t launch_forward_reduce(const Params& p, hipStream_t s) {
  const bool wide = p.kind == 0 && p.dtype == 1;
  if (p.T <= 256) return wide ? launch_reduce_t<uint64_t, 16>(p, s) : launch_reduce_t<uint32_t, 16>(p, s);
  return wide ? launch_reduce_t<uint64_t, 48>(p, s) : launch_reduce_t<uint32_t, 48>(p, s);
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
    case 1: return vm ? launch_bwd_t<1, WM_VMAX>(p, block, lds, s) : launch_bwd_t<1, WM_EXPLICIT>(p, block, lds, s);
    case 2: return vm ? launch_bwd_t<2, WM_VMAX>(p, block, lds, s) : launch_bwd_t<2, WM_EXPLICIT>(p, block, lds, s);
    default: return vm ? launch_bwd_t<3, WM_VMAX>(p, block, lds, s) : launch_bwd_t<3, WM_EXPLICIT>(p, block, lds, s);
  }
}

hipError_t launch_fill_zero(float* ptr, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, ptr, n);
  return hipGetLastError();
}

hipError_t launch_validate(const Params& p, int* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_validate, dim3(256, 4), dim3(256), 0, s, p, flags);
  return hipGetLastError();
}

}  // namespace wect
