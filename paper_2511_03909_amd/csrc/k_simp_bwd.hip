// Adjoint of the simplicial forward with respect to the weights.

#include "wect_device.h"

namespace wect {
namespace {

// backward (adjoint), simplicial, float32 weights
// ---------------------------------------------------------------------------
//
// For L = <grad_out, out>, dL/dw(c) = (-1)^dim(c) sum_p G[p][b_p(c)] with
// G[p][j] = sum_{q >= j} grad_out[p][q] and G[p][T] = 0.  The block holds G for
// up to `dg` direction tiles in LDS ([tile][T+1][64], read conflict-free by
// lane), recomputes each staged simplex's index per direction and sums the
// 64 x dg values with a wavefront reduction.

constexpr int kMaxDG = 4;

// DG: direction tiles of the group (compile time, so that the per-tile loop
// needs no predicates).
template <int N, int DIM, int WM, bool FAST, int DG>
__device__ __forceinline__ void simp_bwd_range(const Params& p, int b, int64_t lo, int64_t hi, int64_t voff, int64_t soff,
                               const float* sx, const float* sy, const float* sz, int tile0,
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
        const float* E = stage + uniform(e0 + min(j0 + k, ne - 1)) * L::STRIDE;
        float a = 0.0f;
#pragma unroll
        for (int jj = 0; jj < DG; ++jj) {
          {
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
                // arithmetic index; the one-read fix only on the lanes that sit on a threshold
                const bool ok = thr_arith(h, th, bi);
                if (__builtin_amdgcn_ballot_w64(!ok) != 0 && !ok) bi = thr_near(h, bi, th);
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

template <int N, int WM, bool FAST, int DG>
__device__ __forceinline__ void simp_bwd_dim_g(int dim, const Params& p, int b, int64_t lo, int64_t hi, int64_t voff,
                                               int64_t soff, const float* sx, const float* sy, const float* sz,
                                               int tile0, const float* Gt, float* stage, const Thr& th) {
  switch (dim) {
    case 0: simp_bwd_range<N, 0, WM, FAST, DG>(p, b, lo, hi, voff, soff, sx, sy, sz, tile0, Gt, stage, th); break;
    case 1: simp_bwd_range<N, 1, WM, FAST, DG>(p, b, lo, hi, voff, soff, sx, sy, sz, tile0, Gt, stage, th); break;
    case 2: simp_bwd_range<N, 2, WM, FAST, DG>(p, b, lo, hi, voff, soff, sx, sy, sz, tile0, Gt, stage, th); break;
    default: simp_bwd_range<N, 3, WM, FAST, DG>(p, b, lo, hi, voff, soff, sx, sy, sz, tile0, Gt, stage, th); break;
  }
}

template <int N, int WM, bool FAST>
__device__ __forceinline__ void simp_bwd_dim(int dim, const Params& p, int b, int64_t lo, int64_t hi, int64_t voff,
                                             int64_t soff, const float* sx, const float* sy, const float* sz, int ntl,
                                             int tile0, const float* Gt, float* stage, const Thr& th) {
  switch (ntl) {
    case 1: simp_bwd_dim_g<N, WM, FAST, 1>(dim, p, b, lo, hi, voff, soff, sx, sy, sz, tile0, Gt, stage, th); break;
    case 2: simp_bwd_dim_g<N, WM, FAST, 2>(dim, p, b, lo, hi, voff, soff, sx, sy, sz, tile0, Gt, stage, th); break;
    case 3: simp_bwd_dim_g<N, WM, FAST, 3>(dim, p, b, lo, hi, voff, soff, sx, sy, sz, tile0, Gt, stage, th); break;
    default: simp_bwd_dim_g<N, WM, FAST, kMaxDG>(dim, p, b, lo, hi, voff, soff, sx, sy, sz, tile0, Gt, stage, th); break;
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
        const float* g = p.grad_out + ((int64_t)b * p.d + gp) * p.ldo;
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

}  // namespace

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

}  // namespace wect
