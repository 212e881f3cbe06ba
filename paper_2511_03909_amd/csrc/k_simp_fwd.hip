// Simplicial forward (and the general-filter WECF index pass).

#include "wect_device.h"

namespace wect {
namespace {

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

// As hist_entries (arithmetic index with the per-wavefront switch to the
// guess), two pairs of entries per step: the four entries' staged words are
// read before any of their histogram adds, so the LDS reads of the second
// pair are in flight while the first pair's heights are formed.
template <bool FAST, typename ACC, typename Entry>
__device__ __forceinline__ void hist_entries_x2(ACC* col, int first, int step, int ne, const Thr& th, int* arith,
                                                Entry entry) {
  int e = first;
  if constexpr (FAST) {
    while (*arith && e + step + 1 < ne) {
      const int stop = min(ne - 1 - step, e + 32 * step);
      int fixes = 0, pairs = 0;
      for (; e < stop; e += 2 * step) {
        float h[4];
        ACC w[4];
        entry(e, h[0], w[0]);
        entry(e + 1, h[1], w[1]);
        entry(e + step, h[2], w[2]);
        entry(e + step + 1, h[3], w[3]);
#pragma unroll
        for (int q = 0; q < 4; q += 2) {
          int b0, b1;
          const bool ok0 = thr_arith(h[q], th, b0);
          const bool ok1 = thr_arith(h[q + 1], th, b1);
          if (__builtin_amdgcn_ballot_w64(!(ok0 && ok1)) != 0) {
            ++fixes;
            if (!ok0) b0 = thr_near(h[q], b0, th);
            if (!ok1) b1 = thr_near(h[q + 1], b1, th);
          }
          ++pairs;
          lds_add(&col[b0 * W], w[q]);
          lds_add(&col[b1 * W], w[q + 1]);
        }
      }
      if (4 * fixes > pairs) *arith = 0;
    }
  }
  hist_entries<FAST, ACC>(col, e, step, ne, th, arith, entry);
}

// Packed tiles (at most 32 directions or filter columns, dt of them rounded up
// to a power of two): lane l serves column l % dt of the entries of lane group
// g = l / dt, so 64 / dt entries share each instruction.  The wavefront's
// groups take the pairs (e + 2g, e + 2g + 1) of its block of 2 * cpw entries;
// entries past ne re-read a valid one and add zero.  Each lane keeps its own
// histogram column; fold_columns adds the groups' copies together before the
// scan.  entry(e, b, w) gives entry e's threshold index and signed weight for
// the lane's column.
template <typename ACC, typename Entry>
__device__ __forceinline__ void packed_entries(ACC* col, int first, int step, int ne, int g, Entry entry) {
  for (int e = first; e < ne; e += step) {
    const int e0 = e + 2 * g, e1 = e0 + 1;
    int b0, b1;
    ACC w0, w1;
    entry(min(e0, ne - 1), b0, w0);
    entry(min(e1, ne - 1), b1, w1);
    if (e0 >= ne) w0 = ACC(0);
    if (e1 >= ne) w1 = ACC(0);
    lds_add(&col[b0 * W], w0);
    lds_add(&col[b1 * W], w1);
  }
}

// Column c < dt of every row gets the copies of the other lane groups
// (columns c + dt, c + 2 dt, ...); the threshold scan then reads columns < dt.
template <typename ACC>
__device__ void fold_columns(ACC* hist, int T, int dt) {
  __syncthreads();
  const int cpw = W / dt;
  for (int i = threadIdx.x; i < (T + 1) * dt; i += blockDim.x) {
    const int q = i / dt, c = i - q * dt;
    ACC s = ACC(0);
    for (int g = 1; g < cpw; ++g) s += hist[q * W + g * dt + c];
    hist[q * W + c] += s;
  }
  __syncthreads();
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
    } else if (p.cpw > 1) {  // packed tile
      const int g = lane / p.dt;
      const int first = 2 * p.cpw * wave, step = 2 * p.cpw * nw;
      if constexpr (N == 0) {
        auto filt = [&](auto vb) {
          packed_entries<ACC>(hist + lane, first, step, cnt, g, [&](int e, int& b, ACC& w) {
            const float* E = stage + e * L::STRIDE;
            b = 0;
#pragma unroll
            for (int j = 0; j < L::NV; ++j) b = max(b, (int)vb[(int64_t)bitcast<int32_t>(E[j]) * p.d + fcol]);
            w = load_weight<ACC>(E + L::WOFF);
          });
        };
        if (p.vb_bytes == 1) filt((const uint8_t*)p.vbuckets);
        else filt((const uint16_t*)p.vbuckets);
      } else {
        packed_entries<ACC>(hist + lane, first, step, cnt, g, [&](int e, int& b, ACC& w) {
          const float* E = stage + e * L::STRIDE;
          b = thr_index<FAST>(max_height<N, DIM>(E, sx, sy, sz), th);
          w = load_weight<ACC>(E + L::WOFF);
        });
      }
    } else if constexpr (N == 0) {
      if (p.vb_bytes == 1)
        filter_hist<DIM, uint8_t, ACC, L>(hist + lane, stage, 2 * wave, 2 * nw, cnt, (const uint8_t*)p.vbuckets, p.d,
                                          fcol);
      else
        filter_hist<DIM, uint16_t, ACC, L>(hist + lane, stage, 2 * wave, 2 * nw, cnt, (const uint16_t*)p.vbuckets,
                                           p.d, fcol);
    } else {
      hist_entries_x2<FAST, ACC>(hist + lane, 2 * wave, 2 * nw, cnt, th, &arith,
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
    // the lane's column within the tile (packed tiles: lane l serves column
    // l % dt); filter column of the lane (N = 0): lanes past the last column
    // read the last one and their histogram column is never written out
    const int cl = p.cpw > 1 ? (lane & (p.dt - 1)) : lane;
    const int fcol = min(t * W + cl, p.d - 1);
    if constexpr (N > 0) load_dir(p, t * W + cl, sx, sy, sz);
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
    if (p.cpw > 1) fold_columns<ACC>(hist, T, p.dt);
    end_group<ACC>(p, hist, k, b, t, e0 == 0 && e1 == nb, fexp);
    pos += e1 - e0;
    if (e1 == nb && t == gpc - 1) ++b;
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


}  // namespace

template <int N, int WM, typename WT, bool SM = false>
static hipError_t launch_simp_fwd_t(const Params& p, int block, size_t lds, hipStream_t s) {
  if (hipError_t e = set_lds_limit(k_simp_fwd<N, WM, WT, SM>, lds); e != hipSuccess) return e;
  hipLaunchKernelGGL((k_simp_fwd<N, WM, WT, SM>), dim3(p.G), dim3(block), lds, s, p);
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

hipError_t launch_forward_simp(const Params& p, int block, size_t lds, hipStream_t s) {
  switch (p.n) {
    case 0: return launch_simp_fwd_n<0>(p, block, lds, s);  // general vertex filter
    case 1: return launch_simp_fwd_n<1>(p, block, lds, s);
    case 2: return launch_simp_fwd_n<2>(p, block, lds, s);
    default: return launch_simp_fwd_n<3>(p, block, lds, s);
  }
}

}  // namespace wect
