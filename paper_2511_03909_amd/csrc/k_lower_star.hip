// Lower-star index and the vertex-centric relaxation kernels.

#include "wect_device.h"

namespace wect {
namespace {

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
      g[(size_t)q * W + r] = dir < p.d ? p.grad_out[((int64_t)b * p.d + dir) * p.ldo + q] : 0.0f;
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


}  // namespace

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

size_t smooth_ls_backward_lds_bytes(int T, int block) { return ls_lds(T, block, ls_rows(T, block, true), true); }

}  // namespace wect
