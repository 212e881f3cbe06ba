// Adjoint of the sigmoid relaxation (per-cell kernel).

#include "wect_device.h"

namespace wect {
namespace {

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

}  // namespace

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

size_t smooth_backward_lds_bytes(int T, int stage) {
  size_t cols = (size_t)(2 * T + 1) * W * 4;
  size_t pairs = ((size_t)(T + 1) * 4 + 15) / 16 * 16;
  return cols + pairs + (size_t)stage * kSmMaxStride * 4;
}

}  // namespace wect
