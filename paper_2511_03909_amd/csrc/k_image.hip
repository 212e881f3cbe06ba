// ECF of images / volumes and the Freudenthal builder.

#include "wect_device.h"

namespace wect {
namespace {

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

}  // namespace wect
