// Reduction of partial histograms, threshold scan, small kernels.

#include "wect_device.h"

namespace wect {
namespace {

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
  const int T = p.T, RW = W * p.dpl;
  if (q >= T) return;
  int64_t kfirst, klast;
  group_slots(p, g, kfirst, klast);
  if (klast - kfirst + 1 <= kFusedSlots) return;
  const int64_t slot_stride = (int64_t)T * RW;
  for (int c = lane; c < RW; c += W) {
    const ACC* src = (const ACC*)p.partial + (int64_t)q * RW + c;
    ACC v0 = 0, v1 = 0, v2 = 0, v3 = 0;
    int64_t kk = kfirst;
    for (; kk + 3 <= klast; kk += 4) {
      v0 += src[(kk + g) * slot_stride];
      v1 += src[(kk + 1 + g) * slot_stride];
      v2 += src[(kk + 2 + g) * slot_stride];
      v3 += src[(kk + 3 + g) * slot_stride];
    }
    for (; kk <= klast; ++kk) v0 += src[(kk + g) * slot_stride];
    ((ACC*)p.dsum)[((int64_t)g * T + q) * RW + c] = (v0 + v1) + (v2 + v3);
  }
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
  // block = (group g, 64-column half h of its dpl * 64 columns)
  const int g = blockIdx.x / p.dpl, h = blockIdx.x - g * p.dpl;
  const int RW = W * p.dpl;
  const int gpc = p.ntiles;
  const int b = g / gpc, t = g % gpc;
  const int lane = threadIdx.x & (W - 1), r = threadIdx.x >> 6;
  const int chunk = (T + 15) / 16;
  const int q0 = min(T, r * chunk), nq = min(T, q0 + chunk) - q0;
  int fexp = 0;
  if constexpr (sizeof(ACC) == 8) fexp = fixed_exp(p);
  const int64_t slot_stride = (int64_t)T * RW;
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
      const ACC* src = (const ACC*)p.dsum + (int64_t)g * slot_stride + (int64_t)q * RW + h * W + lane;
#pragma unroll
      for (int j = 0; j < PC; ++j) v[j] = src[min(j, n - 1) * RW];
    } else {
      for (int64_t kk = kfirst; kk <= klast; ++kk) {
        const ACC* src = (const ACC*)p.partial + (kk + g) * slot_stride + (int64_t)q * RW + h * W + lane;
        ACC x[PC];
#pragma unroll
        for (int j = 0; j < PC; ++j) x[j] = src[min(j, n - 1) * RW];
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
  const int dir0 = t * RW + h * W;
  const int dv = min(W, p.d - dir0);
  OT* out = (OT*)p.out + ((int64_t)b * p.d + (int64_t)dir0) * p.ldo;
  for (int i = threadIdx.x; i < dv * T; i += blockDim.x) {
    const int pp = i / T, q = i - pp * T;
    out[(int64_t)pp * p.ldo + q] = L[pp * LS + q];
  }
}

// Largest |w| over the float32 weights, one partial per block.  The weight
// arrays that the request reads (every dimension's, or the vertex weights of
// vertex-max weights) form one sequence of S values; block k takes the
// contiguous range [kS/G, (k+1)S/G) and reads it four floats per load between
// a scalar head (up to the array's next 16-byte boundary) and a scalar tail.
// fmaxf skips NaN; an infinite weight gives an infinite maximum, for which
// fixed_exp falls back to e = 0.
__global__ __launch_bounds__(1024) void k_absmax(Params p) {
  __shared__ float red[16];
  const int ndim = p.wmode == WM_VMAX ? 1 : p.top_dim + 1;
  int64_t S = 0;
  for (int d = 0; d < ndim; ++d) S += p.count[d];
  const int64_t lo = S * blockIdx.x / gridDim.x, hi = S * (blockIdx.x + 1) / gridDim.x;
  const int tid = threadIdx.x, nt = blockDim.x;
  float m = 0.0f;
  int64_t base = 0;
  for (int d = 0; d < ndim; ++d) {
    const int64_t n = p.count[d];
    const int64_t a = mx64(lo, base) - base, b = mn64(hi, base + n) - base;
    base += n;
    if (a >= b) continue;
    const float* w = (const float*)p.weights[d];
    const int64_t head = (int64_t)(((16 - ((uintptr_t)(w + a) & 15)) & 15) >> 2);
    const int64_t a4 = mn64(a + head, b);
    const int64_t nv = (b - a4) >> 2;
    const int64_t b4 = a4 + 4 * nv;
    if (a + tid < a4) m = fmaxf(m, fabsf(w[a + tid]));
    if (b4 + tid < b) m = fmaxf(m, fabsf(w[b4 + tid]));
    const float4* v = (const float4*)(w + a4);
#pragma unroll 4
    for (int64_t j = tid; j < nv; j += nt) {
      const float4 x = v[j];
      m = fmaxf(m, fmaxf(fmaxf(fabsf(x.x), fabsf(x.y)), fmaxf(fabsf(x.z), fabsf(x.w))));
    }
  }
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((tid & 63) == 0) red[tid >> 6] = m;
  __syncthreads();
  if (tid == 0) {
    float r = 0.0f;
    for (int i = 0; i < (nt >> 6); ++i) r = fmaxf(r, red[i]);
    p.absmax[blockIdx.x] = r;
  }
}

// ---------------------------------------------------------------------------

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

}  // namespace


size_t forward_lds_fixed(int T, int kind, int acc_bytes, int dpl) {
  size_t hist = (size_t)(T + 1) * W * dpl * acc_bytes;
  size_t pairs = ((size_t)(T + 1) * 4 + 15) / 16 * 16;
  (void)kind;
  return hist + pairs + 16;
}

size_t forward_entry_bytes(int kind, int n) { return (size_t)(kind == 1 ? 8 : kMaxStride) * 4; }

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

hipError_t launch_forward_main(const Params& p, int block, size_t lds, hipStream_t s) {
  return p.kind == 1 ? launch_forward_cub(p, block, lds, s) : launch_forward_simp(p, block, lds, s);
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
  hipLaunchKernelGGL((k_reduce_scan<ACC>), dim3(groups * p.dpl), dim3(1024), lds, s, p);
  return hipGetLastError();
}

hipError_t launch_forward_reduce(const Params& p, hipStream_t s) {
  if (p.group_mode) return hipSuccess;  // every block wrote its group's output
  const bool wide = p.kind == 0 && p.dtype == 1;
  return wide ? launch_reduce_t<uint64_t>(p, s) : launch_reduce_t<uint32_t>(p, s);
}

hipError_t launch_absmax(const Params& p, hipStream_t s) {
  hipLaunchKernelGGL(k_absmax, dim3(p.nabsmax), dim3(1024), 0, s, p);
  return hipGetLastError();
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
