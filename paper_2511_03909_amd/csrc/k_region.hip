// Region index and the simplicial forward through per-region tables of vertex
// threshold indices.
//
// A cell's threshold index is the largest of its vertices' indices: the index
// is monotone, the fact the correctness proof of Algorithm 1 rests on.  The
// per-cell forward (k_simp_fwd) recomputes a vertex's height and index for
// every cell that contains it (about 13 cells per vertex in a 2D
// triangulation, 25 in a 3D one).  Here the cells are grouped by region:
// region k of complex b owns the vertices [kR, (k+1)R) (local ids) and holds
// every cell whose lowest vertex it owns; the other vertices those cells use
// form its halo.  For each region and direction tile the forward computes the
// index of every owned and halo vertex once into an LDS table laid out
// [vertex][lane] (one byte per entry), then each cell costs one table read per
// vertex, a maximum and the histogram add.  The histogram sums are integer or
// fixed point, so the output has the same bits as the per-cell forward's.
//
// The index depends on the simplex lists only; one build serves every call on
// the same topology.  Build: count the cells of every region (atomics), scan
// the counts, fill the cells into region order (atomics: the order inside a
// region is not fixed and no result depends on it), then one block per region
// collects, sorts and deduplicates its halo and writes the cells' local ids.

#include <type_traits>

#include "wect_device.h"

namespace wect {
namespace {

__device__ __forceinline__ int64_t* rg_cnt_row(const Params& p, int i) { return p.rg_cnt + (int64_t)i * (p.rg_nrmax + 1); }

// region of simplex (dim, r) (global row r) and its vertices (local ids)
__device__ __forceinline__ int64_t rg_region_of(const Params& p, int dim, int64_t r, int32_t (&v)[4]) {
  const int b = complex_of_row(p, dim, r);
  const int32_t* sp = p.simp[dim] + r * (dim + 1);
  int32_t mn = INT32_MAX;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    v[j] = j <= dim ? sp[j] : 0;
    if (j <= dim) mn = min(mn, v[j]);
  }
  // clamped into the index (vertex ids are valid by contract; an invalid one
  // must not turn into a write outside the count rows)
  const int64_t g = p.rg_reg[b] + (mn < 0 ? 0 : mn) / p.rg_R;
  return g < p.rg_nrmax ? g : p.rg_nrmax - 1;
}

__global__ __launch_bounds__(256) void k_rg_zero(Params p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) p.rg_cnt[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x < 8) p.rg_hdr[threadIdx.x] = threadIdx.x == 0 ? p.rg_R : 0;
}

// Inclusive scan of tot[0 .. blockDim.x) in place (every thread holds one entry).
template <typename I>
__device__ __forceinline__ void block_scan_incl(I* tot) {
  const int tid = threadIdx.x;
  for (int o = 1; o < (int)blockDim.x; o <<= 1) {
    const I add = tid >= o ? tot[tid - o] : I(0);
    __syncthreads();
    tot[tid] += add;
    __syncthreads();
  }
}

// First region of every complex: reg[b] = sum over b' < b of ceil(V_b' / R)
// (one block); hdr[1] = the number of regions.
__global__ __launch_bounds__(1024) void k_rg_regions(Params p) {
  __shared__ int64_t tot[1024];
  const int tid = threadIdx.x, nt = blockDim.x, B = p.B, R = p.rg_R;
  auto nreg = [&](int b) -> int64_t {
    const int64_t V = off_or(p.vert_off, b + 1, p.count[0]) - off_or(p.vert_off, b, p.count[0]);
    return (V + R - 1) / R;
  };
  const int per = (B + nt - 1) / nt;
  const int a = min(B, tid * per), z = min(B, a + per);
  int64_t s = 0;
  for (int b = a; b < z; ++b) s += nreg(b);
  tot[tid] = s;
  __syncthreads();
  block_scan_incl(tot);
  int64_t run = tot[tid] - s;
  for (int b = a; b < z; ++b) {
    p.rg_reg[b] = run;
    run += nreg(b);
  }
  if (tid == nt - 1) {
    p.rg_reg[B] = tot[nt - 1];
    p.rg_hdr[1] = tot[nt - 1];
  }
}

// Cells per region and dimension, and the halo references per region (each
// cell's vertices other than its lowest: dim of them).
__global__ __launch_bounds__(256) void k_rg_count(Params p) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t* href = rg_cnt_row(p, 0);
  for (int dim = 1; dim <= p.top_dim; ++dim) {
    int64_t* cnt = rg_cnt_row(p, dim);
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < p.count[dim]; r += stride) {
      int32_t v[4];
      const int64_t g = rg_region_of(p, dim, r, v);
      atomicAdd((unsigned long long*)&cnt[g], 1ull);
      atomicAdd((unsigned long long*)&href[g], (unsigned long long)dim);
    }
  }
}

// Block i: exclusive scan of count row i into its offsets (row 0: the halo
// list starts, rows 1..3: each dimension's region offsets), leaving the
// offsets in the count row as fill cursors.
__global__ __launch_bounds__(1024) void k_rg_scan(Params p) {
  __shared__ int64_t tot[1024];
  const int i = blockIdx.x;
  if (i > p.top_dim) return;
  const int64_t n = p.rg_nrmax;
  int64_t* cnt = rg_cnt_row(p, i);
  int64_t* off = i == 0 ? p.rg_hoff : p.rg_coff[i];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t per = (n + nt - 1) / nt;
  const int64_t a = mn64(n, tid * per), z = mn64(n, a + per);
  int64_t s = 0;
  for (int64_t r = a; r < z; ++r) s += cnt[r];
  tot[tid] = s;
  __syncthreads();
  block_scan_incl(tot);
  int64_t run = tot[tid] - s;
  for (int64_t r = a; r < z; ++r) {
    const int64_t c = cnt[r];
    off[r] = run;
    cnt[r] = run;
    run += c;
  }
  if (tid == nt - 1) off[n] = tot[nt - 1];
}

// Every cell into its region's range (row within its dimension).
__global__ __launch_bounds__(256) void k_rg_fill(Params p) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int dim = 1; dim <= p.top_dim; ++dim) {
    int64_t* cur = rg_cnt_row(p, dim);
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < p.count[dim]; r += stride) {
      int32_t v[4];
      const int64_t g = rg_region_of(p, dim, r, v);
      const int64_t pos = (int64_t)atomicAdd((unsigned long long*)&cur[g], 1ull);
      p.rg_perm[dim][pos] = (int32_t)r;
    }
  }
}

// One block per region: its halo (the vertices of its cells above the region,
// sorted and deduplicated: halo vertex k gets local id nown + k) and the local
// ids of its cells.  Status bits: 1 = more halo references than kRgCand,
// 2 = more local vertices than uint16 ids address.
constexpr int kRgPer = kRgCand / 1024;  // sorted candidates per thread

__global__ __launch_bounds__(1024) void k_rg_local(Params p) {
  extern __shared__ __align__(16) unsigned char smem[];
  int32_t* cand = (int32_t*)smem;            // [kRgCand]
  int32_t* sums = cand + kRgCand;             // [1024]
  __shared__ int32_t s_n;
  const int64_t r = blockIdx.x;
  if (r >= p.rg_hdr[1]) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  int lo = 0, hi = p.B - 1;  // complex of region r: largest b with reg[b] <= r
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (p.rg_reg[mid] <= r) lo = mid;
    else hi = mid - 1;
  }
  const int b = lo;
  const int64_t voff = off_or(p.vert_off, b, p.count[0]);
  const int64_t Vb = off_or(p.vert_off, b + 1, p.count[0]) - voff;
  const int R = p.rg_R;
  const int64_t vlo = (r - p.rg_reg[b]) * R;
  const int64_t vhi = mn64(vlo + R, Vb);
  const int nown = (int)(vhi - vlo);
  if (tid == 0) s_n = 0;
  __syncthreads();
  for (int dim = 1; dim <= p.top_dim; ++dim) {
    const int64_t c0 = p.rg_coff[dim][r], c1 = p.rg_coff[dim][r + 1];
    for (int64_t pos = c0 + tid; pos < c1; pos += nt) {
      const int32_t* sp = p.simp[dim] + (int64_t)p.rg_perm[dim][pos] * (dim + 1);
      for (int j = 0; j <= dim; ++j) {
        const int32_t v = sp[j];
        if (v >= vhi) {
          const int k = atomicAdd(&s_n, 1);
          if (k < kRgCand) cand[k] = v;
        }
      }
    }
  }
  __syncthreads();
  const int n = s_n;
  if (n > kRgCand) {
    if (tid == 0) atomicOr((unsigned long long*)&p.rg_hdr[2], 1ull);
    return;
  }
  int n2 = 1;
  while (n2 < n) n2 <<= 1;
  for (int i = n + tid; i < n2; i += nt) cand[i] = INT32_MAX;
  __syncthreads();
  // bitonic sort of cand[0 .. n2)
  for (int k = 2; k <= n2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < n2; i += nt) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const int32_t x = cand[i], y = cand[ixj];
          if ((x > y) == ((i & k) == 0)) {
            cand[i] = y;
            cand[ixj] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  // first occurrences, counted over contiguous chunks of kRgPer entries
  const int a = tid * kRgPer;
  int32_t v16[kRgPer];
  bool f16[kRgPer];
  int cu = 0;
#pragma unroll
  for (int q = 0; q < kRgPer; ++q) {
    const int i = a + q;
    const bool in = i < n;
    v16[q] = in ? cand[i] : 0;
    f16[q] = in && (i == 0 || cand[i] != cand[i - 1]);
    cu += f16[q] ? 1 : 0;
  }
  sums[tid] = cu;
  __syncthreads();
  block_scan_incl(sums);
  const int H = sums[nt - 1];
  int run = sums[tid] - cu;
  const int64_t hb = p.rg_hoff[r];
#pragma unroll
  for (int q = 0; q < kRgPer; ++q) {
    if (f16[q]) {
      cand[run] = v16[q];
      p.rg_halo[hb + run] = (int32_t)(voff + v16[q]);
      ++run;
    }
  }
  if (tid == 0) {
    p.rg_hcnt[r] = H;
    atomicMax((unsigned long long*)&p.rg_hdr[3], (unsigned long long)H);
    if (nown + H > kRgMaxLocal + 1) atomicOr((unsigned long long*)&p.rg_hdr[2], 2ull);
  }
  __syncthreads();
  auto local_id = [&](int32_t v) -> uint32_t {
    if (v < vhi) return (uint32_t)(v - vlo);
    int l = 0, h = H;  // lower bound of v in cand[0 .. H)
    while (l < h) {
      const int m = (l + h) >> 1;
      if (cand[m] < v) l = m + 1;
      else h = m;
    }
    return (uint32_t)(nown + l) & 0xffffu;
  };
  for (int dim = 1; dim <= p.top_dim; ++dim) {
    const int64_t c0 = p.rg_coff[dim][r], c1 = p.rg_coff[dim][r + 1];
    for (int64_t pos = c0 + tid; pos < c1; pos += nt) {
      const int32_t* sp = p.simp[dim] + (int64_t)p.rg_perm[dim][pos] * (dim + 1);
      if (dim == 1) {
        ((uint32_t*)p.rg_rec[1])[pos] = local_id(sp[0]) | (local_id(sp[1]) << 16);
      } else {
        const uint32_t i2 = local_id(sp[2]);
        const uint32_t i3 = dim == 3 ? local_id(sp[3]) : i2;
        uint2 w;
        w.x = local_id(sp[0]) | (local_id(sp[1]) << 16);
        w.y = i2 | (i3 << 16);
        ((uint2*)p.rg_rec[dim])[pos] = w;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
//
// LDS: hist [T+1][64] | P [T+1] | tab [cap][64] uint8 | ovf [cap] uint64 |
//      Vc [cap] float4 (coordinates, vertex weight) | Wst [waves][wb] uint4
// tab[u][lane] = min(threshold index of local vertex u, 255); with T = 256 an
// index of 256 (above every threshold) also reads 255 and ovf[u] has the
// lane's bit set, which the rare cells whose largest entry is 255 look up.
// Every wavefront walks its own batches of wb cells: its lanes stage a batch
// (one cell each) into its part of Wst as {table offsets of vertices 0,1 | of
// vertices 2,3 (uint16 pairs: local id * 64), signed weight (one or two
// words)}, then every lane reads each staged cell as a broadcast.  A cell with
// a vertex at or above the table (a halo larger than the table) keeps its
// local ids instead, flagged in a per-batch mask, and takes those indices from
// global memory.  Loads run two batches ahead: the local ids (and the cell's
// row) first, then the explicit weight that the row selects.

template <int N, int WM, typename ACC>
__device__ __forceinline__ float4 rg_vertex(const Params& p, int64_t g) {
  float4 v;
  const float* c = p.coords + g * N;
  v.x = c[0];
  v.y = N >= 2 ? c[1] : 0.0f;
  v.z = N >= 3 ? c[2] : 0.0f;
  v.w = WM == WM_VMAX ? ((const float*)p.weights[0])[g] : 0.0f;
  return v;
}

template <int N, bool FAST>
__device__ __forceinline__ int rg_index(const float4& v, float sx, float sy, float sz, const Thr& th) {
  const float c[3] = {v.x, v.y, v.z};
  return thr_index<FAST>(height<N>(c, sx, sy, sz), th);
}

// LDS writes of a wavefront made visible to its other lanes, and its reads
// finished before the area is written again.
__device__ __forceinline__ void rg_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Histogram of one wavefront's staged batch S of cells of dimension D, cnt
// rounded up to even (the staging pads an odd batch with a zero-weight copy).
// LEAN: no cell of the batch has a vertex outside the table and no vertex of
// the region lies above the last threshold, so each cell is its table reads,
// their maximum and the add.
template <int D, bool LEAN, bool OV, typename ACC, typename Slow>
__device__ __forceinline__ void rg_batch(ACC* col, const uint4* S, int cnt, uint64_t slowm, const uint8_t* tab,
                                         const uint64_t* ovf, Slow slow) {
  const int lane = threadIdx.x & (W - 1);
  auto index = [&](const uint4& s, int j) -> int {
    if constexpr (!LEAN) {
      if ((slowm >> j) & 1) {
        const int id[4] = {(int)(s.x & 0xffff), (int)(s.x >> 16), (int)(s.y & 0xffff), (int)(s.y >> 16)};
        return slow(id, D);
      }
    }
    const int o[4] = {(int)(s.x & 0xffff), (int)(s.x >> 16), (int)(s.y & 0xffff), (int)(s.y >> 16)};
    int b = tab[o[0] + lane];
#pragma unroll
    for (int q = 1; q <= D; ++q) b = max(b, (int)tab[o[q] + lane]);
    if constexpr (OV && !LEAN) {
      if (__builtin_amdgcn_ballot_w64(b == 255) != 0) {
        uint64_t m = ovf[o[0] >> 6];
#pragma unroll
        for (int q = 1; q <= D; ++q) m |= ovf[o[q] >> 6];
        if (b == 255 && ((m >> lane) & 1)) b = 256;
      }
    }
    return b;
  };
  auto weight = [](const uint4& s) -> ACC {
    if constexpr (sizeof(ACC) == 4) return s.z;
    else return (uint64_t)s.z | ((uint64_t)s.w << 32);
  };
  int j = 0;
  if constexpr (LEAN) {  // four independent cells in flight
    for (; j + 3 < cnt; j += 4) {
      const uint4 a = S[j], c = S[j + 1], e = S[j + 2], f = S[j + 3];
      const int ba = index(a, j), bc = index(c, j + 1), be = index(e, j + 2), bf = index(f, j + 3);
      lds_add(&col[ba * W], weight(a));
      lds_add(&col[bc * W], weight(c));
      lds_add(&col[be * W], weight(e));
      lds_add(&col[bf * W], weight(f));
    }
  }
  for (; j < cnt; j += 2) {
    const uint4 a = S[j], c = S[j + 1];
    const int ba = index(a, j), bc = index(c, j + 1);
    lds_add(&col[ba * W], weight(a));
    lds_add(&col[bc * W], weight(c));
  }
}

template <int N, int WM, typename WT, bool FAST, bool OV>
__device__ __forceinline__ void rg_fwd_range(const Params& p, int b, int64_t e0, int64_t e1, int64_t voff, int64_t Vb,
                                             float sx, float sy, float sz, typename AccOf<WT>::T* hist, uint8_t* tab,
                                             uint64_t* ovf, float4* Vc, uint4* Wst, int* s_ov, const Thr& th,
                                             int fexp) {
  using ACC = typename AccOf<WT>::T;
  using WR = typename std::conditional<sizeof(ACC) == 8, float, int32_t>::type;  // a weight as stored
  const int R = p.rg_R, CAP = p.rg_cap, WB = p.rg_chunk;
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & (W - 1);
  const int wave = uniform(tid >> 6), nw = nt >> 6;
  uint4* myst = Wst + wave * WB;
  // the regions whose first vertex lies in [e0, e1)
  const int64_t k0 = (e0 + R - 1) / R, k1 = (e1 + R - 1) / R;
  struct Reg {
    int64_t r, vlo, hb;
    int nown, H, Ut;
  };
  auto meta = [&](int64_t k) -> Reg {
    Reg g;
    g.r = p.rg_reg[b] + k;
    g.vlo = k * R;
    g.nown = (int)mn64(R, Vb - g.vlo);
    g.H = p.rg_hcnt[g.r];
    g.hb = p.rg_hoff[g.r];
    g.Ut = min(g.nown + g.H, CAP);
    return g;
  };
  // global row of local vertex u (clamped into the region's lists, so that an
  // index built for another topology cannot read out of bounds)
  auto grow_of = [&](const Reg& g, int u) -> int64_t {
    if (u < g.nown || g.H == 0) return voff + g.vlo + min(u, g.nown - 1);
    return (int64_t)p.rg_halo[g.hb + min(u - g.nown, g.H - 1)];
  };
  float4 pre = make_float4(0.0f, 0.0f, 0.0f, 0.0f);  // this thread's vertex row of the next region
  if (k0 < k1) {
    const Reg g = meta(k0);
    if (tid < g.Ut) pre = rg_vertex<N, WM, ACC>(p, grow_of(g, tid));
  }
  for (int64_t k = k0; k < k1; ++k) {
    const Reg g = meta(k);
    const int64_t r = g.r;
    const int Ut = g.Ut;
    auto grow = [&](int u) { return grow_of(g, u); };
    __syncthreads();  // every wavefront is done with the previous region's table
    if (tid == 0) *s_ov = 0;
    if (tid < Ut) Vc[tid] = pre;
    for (int u = tid + nt; u < Ut; u += nt) Vc[u] = rg_vertex<N, WM, ACC>(p, grow(u));
    __syncthreads();
    auto trow = [&](int u, int bi) {
      tab[u * W + lane] = (uint8_t)min(bi, 255);
      if constexpr (OV) {
        const uint64_t m = __builtin_amdgcn_ballot_w64(bi > 255);
        if (lane == 0) {
          ovf[u] = m;
          if (m) *s_ov = 1;
        }
      }
    };
    int u = wave;
    for (; u + nw < Ut; u += 2 * nw) {  // two rows in flight
      const float4 va = Vc[u], vb = Vc[u + nw];
      const int ba = rg_index<N, FAST>(va, sx, sy, sz, th), bb = rg_index<N, FAST>(vb, sx, sy, sz, th);
      trow(u, ba);
      trow(u + nw, bb);
    }
    if (u < Ut) trow(u, rg_index<N, FAST>(Vc[u], sx, sy, sz, th));
    if (k + 1 < k1) {  // the next region's vertex rows, while this region runs
      const Reg gn = meta(k + 1);
      if (tid < gn.Ut) pre = rg_vertex<N, WM, ACC>(p, grow_of(gn, tid));
    }
    __syncthreads();
    const bool ovr = OV && uniform(*s_ov) != 0;  // some vertex of the region is above the last threshold

    // cells: the region's owned vertices (dimension 0), then each dimension's
    // cells, in batches of WB; wavefront w takes batches w, w + nw, ...
    int64_t nd[4];
    nd[0] = g.nown;
#pragma unroll
    for (int d = 1; d <= 3; ++d) nd[d] = d <= p.top_dim ? p.rg_coff[d][r + 1] - p.rg_coff[d][r] : 0;
    int bs1 = (int)((nd[0] + WB - 1) / WB);
    const int bs2 = bs1 + (int)((nd[1] + WB - 1) / WB);
    const int bs3 = bs2 + (int)((nd[2] + WB - 1) / WB);
    const int btot = bs3 + (int)((nd[3] + WB - 1) / WB);
    auto where = [&](int bi, int& d, int64_t& j0, int& cnt) {
      d = (bi >= bs1 ? 1 : 0) + (bi >= bs2 ? 1 : 0) + (bi >= bs3 ? 1 : 0);
      const int first = d == 0 ? 0 : d == 1 ? bs1 : d == 2 ? bs2 : bs3;
      const int64_t n = d == 0 ? nd[0] : d == 1 ? nd[1] : d == 2 ? nd[2] : nd[3];
      j0 = (int64_t)(bi - first) * WB;
      cnt = (int)mn64(WB, n - j0);
    };
    struct S1 {
      uint32_t lo, hi;
      int64_t row;
    };
    // stage 1: the cell's local ids and, for explicit weights, its row
    auto s1 = [&](int bi) -> S1 {
      S1 a{0u, 0u, 0};
      if (bi < btot) {
        int d, cnt;
        int64_t j0;
        where(bi, d, j0, cnt);
        if (lane < cnt) {
          const int64_t j = j0 + lane;
          if (d == 0) {
            a.lo = (uint32_t)j | ((uint32_t)j << 16);
            a.hi = a.lo;
            a.row = grow((int)j);
          } else {
            const int64_t pos = p.rg_coff[d][r] + j;
            if (d == 1) {
              a.lo = ((const uint32_t*)p.rg_rec[1])[pos];
              a.hi = a.lo;
            } else {
              const uint2 x = ((const uint2*)p.rg_rec[d])[pos];
              a.lo = x.x;
              a.hi = x.y;
            }
            if constexpr (WM == WM_EXPLICIT) a.row = p.rg_perm[d][pos];
          }
        }
      }
      return a;
    };
    // stage 2: the explicit weight of the row
    auto s2 = [&](int bi, const S1& a) -> WR {
      WR w = WR(0);
      if constexpr (WM == WM_EXPLICIT) {
        if (bi < btot) {
          int d, cnt;
          int64_t j0;
          where(bi, d, j0, cnt);
          if (lane < cnt) w = ((const WR*)p.weights[d])[a.row];
        }
      }
      return w;
    };
    // a local vertex's threshold index from global memory (ids at or above the table)
    auto slow = [&](const int (&id)[4], int D) -> int {
      int m = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q <= D) m = max(m, rg_index<N, FAST>(rg_vertex<N, WM, ACC>(p, grow(id[q])), sx, sy, sz, th));
      return m;
    };
    // the lanes' cells of batch bi into the wavefront's staging area; returns the slow-cell mask
    auto stage = [&](int bi, const S1& a, WR wr) -> uint64_t {
      int d, cnt;
      int64_t j0;
      where(bi, d, j0, cnt);
      bool slw = false;
      if (lane < cnt) {
        // ids of a triangle repeat its third vertex, of an edge both, of a vertex itself:
        // the maximum over the four is the cell's
        const int id[4] = {(int)(a.lo & 0xffff), (int)(a.lo >> 16), (int)(a.hi & 0xffff), (int)(a.hi >> 16)};
        const int top = max(max(id[0], id[1]), max(id[2], id[3]));
        slw = top >= Ut;
        uint4 s;
        s.x = slw ? a.lo : ((uint32_t)id[0] << 6) | ((uint32_t)id[1] << 22);
        s.y = slw ? a.hi : ((uint32_t)id[2] << 6) | ((uint32_t)id[3] << 22);
        ACC c;
        if constexpr (WM == WM_ONES) {
          c = ACC(1);
        } else if constexpr (WM == WM_VMAX) {
          auto vw = [&](int u) { return u < Ut ? Vc[u].w : ((const float*)p.weights[0])[grow(u)]; };
          const float w = fmaxf(fmaxf(vw(id[0]), vw(id[1])), fmaxf(vw(id[2]), vw(id[3])));
          c = to_fixed(w, fexp);
        } else {
          if constexpr (sizeof(ACC) == 8) c = to_fixed(wr, fexp);
          else c = (uint32_t)wr;
        }
        if (d & 1) c = ACC(0) - c;
        s.z = (uint32_t)c;
        s.w = sizeof(ACC) == 8 ? (uint32_t)((uint64_t)c >> 32) : 0u;
        myst[lane] = s;
        if ((cnt & 1) && lane == cnt - 1) {  // pad to an even count: a copy of weight 0
          s.z = 0u;
          s.w = 0u;
          myst[cnt] = s;
        }
      }
      const uint64_t m = __builtin_amdgcn_ballot_w64(slw);
      const uint64_t mm = (cnt & 1) ? m | ((m >> (cnt - 1)) & 1) << cnt : m;
      // the same in every lane: keep it in scalar registers
      return ((uint64_t)(uint32_t)uniform((int)(mm >> 32)) << 32) | (uint32_t)uniform((int)(uint32_t)mm);
    };
    int bi = wave;
    S1 a1 = s1(bi), a2 = s1(bi + nw);
    WR w1 = s2(bi, a1);
    while (bi < btot) {
      const uint64_t sm = stage(bi, a1, w1);
      rg_wave_sync();
      const WR w2 = s2(bi + nw, a2);
      const S1 a3 = s1(bi + 2 * nw);
      int d, cnt;
      int64_t j0;
      where(bi, d, j0, cnt);
      cnt += cnt & 1;
      if (sm == 0 && !ovr) {
        if (d == 0) rg_batch<0, true, OV>(hist + lane, myst, cnt, sm, tab, ovf, slow);
        else if (d == 1) rg_batch<1, true, OV>(hist + lane, myst, cnt, sm, tab, ovf, slow);
        else if (d == 2) rg_batch<2, true, OV>(hist + lane, myst, cnt, sm, tab, ovf, slow);
        else rg_batch<3, true, OV>(hist + lane, myst, cnt, sm, tab, ovf, slow);
      } else {
        if (d == 0) rg_batch<0, false, OV>(hist + lane, myst, cnt, sm, tab, ovf, slow);
        else if (d == 1) rg_batch<1, false, OV>(hist + lane, myst, cnt, sm, tab, ovf, slow);
        else if (d == 2) rg_batch<2, false, OV>(hist + lane, myst, cnt, sm, tab, ovf, slow);
        else rg_batch<3, false, OV>(hist + lane, myst, cnt, sm, tab, ovf, slow);
      }
      rg_wave_sync();
      a1 = a2;
      w1 = w2;
      a2 = a3;
      bi += nw;
    }
  }
  __syncthreads();
}

template <int N, int WM, typename WT>
__global__ __launch_bounds__(1024) void k_rg_fwd(Params p) {
  using ACC = typename AccOf<WT>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  const int T = p.T, CAP = p.rg_cap;
  ACC* hist = (ACC*)smem;
  float* P = (float*)(smem + (size_t)(T + 1) * W * sizeof(ACC));
  uint8_t* tab = (uint8_t*)P + align_up((size_t)(T + 1) * 4, 16);
  uint64_t* ovf = (uint64_t*)(tab + (size_t)CAP * W);
  float4* Vc = (float4*)(ovf + CAP);
  uint4* Wst = (uint4*)(Vc + CAP);
  __shared__ int s_ov;
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
    float sx, sy, sz;
    load_dir(p, t * W + lane, sx, sy, sz);
    const int64_t voff = off_or(p.vert_off, b, p.count[0]);
    if (T > 255) {
      if (th.fast) rg_fwd_range<N, WM, WT, true, true>(p, b, e0, e1, voff, nb, sx, sy, sz, hist, tab, ovf, Vc, Wst, &s_ov, th, fexp);
      else rg_fwd_range<N, WM, WT, false, true>(p, b, e0, e1, voff, nb, sx, sy, sz, hist, tab, ovf, Vc, Wst, &s_ov, th, fexp);
    } else {
      if (th.fast) rg_fwd_range<N, WM, WT, true, false>(p, b, e0, e1, voff, nb, sx, sy, sz, hist, tab, ovf, Vc, Wst, &s_ov, th, fexp);
      else rg_fwd_range<N, WM, WT, false, false>(p, b, e0, e1, voff, nb, sx, sy, sz, hist, tab, ovf, Vc, Wst, &s_ov, th, fexp);
    }
    end_group<ACC>(p, hist, k, b, t, e0 == 0 && e1 == nb, fexp);
    pos += e1 - e0;
    if (e1 == nb && t == gpc - 1) ++b;
  }
}

template <int N, int WM, typename WT>
hipError_t launch_rg_fwd_t(const Params& p, int block, size_t lds, hipStream_t s) {
  if (hipError_t e = set_lds_limit(k_rg_fwd<N, WM, WT>, lds); e != hipSuccess) return e;
  hipLaunchKernelGGL((k_rg_fwd<N, WM, WT>), dim3(p.G), dim3(block), lds, s, p);
  return hipGetLastError();
}

template <int N>
hipError_t launch_rg_fwd_n(const Params& p, int block, size_t lds, hipStream_t s) {
  if (p.wmode == WM_ONES) return launch_rg_fwd_t<N, WM_ONES, uint32_t>(p, block, lds, s);
  if (p.wmode == WM_EXPLICIT) {
    if (p.dtype == 0) return launch_rg_fwd_t<N, WM_EXPLICIT, uint32_t>(p, block, lds, s);
    return launch_rg_fwd_t<N, WM_EXPLICIT, float>(p, block, lds, s);
  }
  return launch_rg_fwd_t<N, WM_VMAX, float>(p, block, lds, s);
}

}  // namespace

int region_size(int top_dim) { return top_dim >= 3 ? 64 : 384; }

RgLayout rg_layout(int B, int64_t V, const int64_t count[4], int top_dim) {
  RgLayout L{};
  L.R = region_size(top_dim);
  L.nrmax = (V + L.R - 1) / L.R + B;
  L.nhalo = 0;
  for (int i = 1; i <= top_dim; ++i) L.nhalo += (int64_t)i * count[i];
  auto a256 = [](size_t x) { return (x + 255) / 256 * 256; };
  size_t o = 0;
  L.hdr = o;
  o += a256(8 * 8);
  L.reg = o;
  o += a256((size_t)(B + 1) * 8);
  L.cnt = o;
  o += a256((size_t)4 * (L.nrmax + 1) * 8);
  for (int i = 0; i < 4; ++i) {
    L.coff[i] = L.perm[i] = L.rec[i] = 0;
    if (i < 1 || i > top_dim) continue;
    L.coff[i] = o;
    o += a256((size_t)(L.nrmax + 1) * 8);
    L.perm[i] = o;
    o += a256((size_t)count[i] * 4);
    L.rec[i] = o;
    o += a256((size_t)count[i] * (i == 1 ? 4 : 8));
  }
  L.hoff = o;
  o += a256((size_t)(L.nrmax + 1) * 8);
  L.hcnt = o;
  o += a256((size_t)L.nrmax * 4);
  L.halo = o;
  o += a256((size_t)std::max<int64_t>(L.nhalo, 1) * 4);
  L.total = o;
  return L;
}

void rg_bind(Params& p, void* base, const RgLayout& L) {
  unsigned char* b8 = static_cast<unsigned char*>(base);
  p.rg = 1;
  p.rg_R = L.R;
  p.rg_nrmax = L.nrmax;
  p.rg_hdr = (int64_t*)(b8 + L.hdr);
  p.rg_reg = (int64_t*)(b8 + L.reg);
  p.rg_cnt = (int64_t*)(b8 + L.cnt);
  for (int i = 0; i < 4; ++i) {
    const bool on = i >= 1 && i <= p.top_dim;
    p.rg_coff[i] = on ? (int64_t*)(b8 + L.coff[i]) : nullptr;
    p.rg_perm[i] = on ? (int32_t*)(b8 + L.perm[i]) : nullptr;
    p.rg_rec[i] = on ? (void*)(b8 + L.rec[i]) : nullptr;
  }
  p.rg_hoff = (int64_t*)(b8 + L.hoff);
  p.rg_hcnt = (int32_t*)(b8 + L.hcnt);
  p.rg_halo = (int32_t*)(b8 + L.halo);
}

hipError_t launch_region_build(const Params& p, const RgLayout& L, hipStream_t s) {
  int64_t cells = 0;
  for (int i = 1; i <= p.top_dim; ++i) cells = std::max<int64_t>(cells, p.count[i]);
  const int64_t ncnt = 4 * (L.nrmax + 1);
  hipLaunchKernelGGL(k_rg_zero, dim3((unsigned)std::min<int64_t>(4096, (ncnt + 255) / 256)), dim3(256), 0, s, p,
                     ncnt);
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rg_regions, dim3(1), dim3(1024), 0, s, p);
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  const unsigned gc = (unsigned)std::max<int64_t>(1, std::min<int64_t>(8192, (cells + 255) / 256));
  hipLaunchKernelGGL(k_rg_count, dim3(gc), dim3(256), 0, s, p);
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rg_scan, dim3(4), dim3(1024), 0, s, p);
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rg_fill, dim3(gc), dim3(256), 0, s, p);
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  const size_t lds = (size_t)(kRgCand + 1024) * 4;
  if (hipError_t e = set_lds_limit(k_rg_local, lds); e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rg_local, dim3((unsigned)L.nrmax), dim3(1024), lds, s, p);
  return hipGetLastError();
}

// chunk: staged cells of the whole block (wavefronts x cells per batch)
size_t region_forward_lds_bytes(int T, int cap, int chunk, int acc_bytes) {
  return (size_t)(T + 1) * kWave * acc_bytes + ((size_t)(T + 1) * 4 + 15) / 16 * 16 + (size_t)cap * kWave +
         (size_t)cap * 8 + (size_t)cap * 16 + (size_t)chunk * 16;
}

hipError_t launch_region_forward(const Params& p, int block, size_t lds, hipStream_t s) {
  switch (p.n) {
    case 1: return launch_rg_fwd_n<1>(p, block, lds, s);
    case 2: return launch_rg_fwd_n<2>(p, block, lds, s);
    default: return launch_rg_fwd_n<3>(p, block, lds, s);
  }
}

}  // namespace wect
