// nsplat_forward / the first half of nsplat_backward: per-tile alpha
// compositing (Sec. 3.4, Eq. 8-9) and its adjoint.
//
// One block per (scene, tile); 8x8 tiles use one wavefront, 16x16 and 32x32
// tiles 256 threads (one or four pixels per thread).  The tile's Gaussians
// are staged into LDS in batches in front-to-back order (the slice of idx
// read from its end); each lane walks the batch for its pixel(s).  Centres
// become exact tile-local FP32 coordinates at staging time (FP64 centre minus
// the tile origin, rounded once).  The forward stops a pixel once T < eps_T
// and the block once all its pixels have stopped.  The adjoint walks the same
// lists back to front from each pixel's stopping position, recovering the
// transmittance as T / (1 - alpha) (alpha <= alpha_max < 1), reduces each
// Gaussian's gradient across the wavefront and adds it with one atomic per
// value and wavefront.
#include "nsplat_internal.h"

namespace nsp {

namespace {

template <int TILE>
struct TileCfg {
  static constexpr int THREADS = TILE == 8 ? 64 : 256;
  static constexpr int PPT = TILE * TILE / THREADS;
};

// Next (scene, tile) work item: the block's own index, or the next entry of
// the device work queue for the persistent form.
__device__ inline int next_tile(int it, int persistent, int32_t* queue, int* s_item) {
  if (!persistent) return it == 0 ? (int)blockIdx.x : 0x7fffffff;
  __syncthreads();
  if (threadIdx.x == 0) *s_item = atomicAdd(queue, 1);
  __syncthreads();
  return *s_item;
}

template <int C, int TILE>
__global__ __launch_bounds__(TileCfg<TILE>::THREADS) void k_blend_fwd(
    nsplat_curves cv, nsplat_params pr, Work w, int n_scenes, int n_tiles, const Gauss* __restrict__ gs,
    const int32_t* __restrict__ ranges, const int32_t* __restrict__ idx, const float* __restrict__ bg,
    float* __restrict__ image, float* __restrict__ Tfin, int32_t* __restrict__ nlast, int persistent) {
  constexpr int THREADS = TileCfg<TILE>::THREADS, PPT = TileCfg<TILE>::PPT;
  __shared__ float s_cx[MAX_BATCH], s_cy[MAX_BATCH], s_a[MAX_BATCH], s_r2[MAX_BATCH], s_o[MAX_BATCH];
  __shared__ float s_col[C][MAX_BATCH];
  __shared__ int s_item;
  const int B = pr.batch;
  const float amax = pr.alpha_max, eps = pr.eps_T, ks = pr.k_sigma;
  const int tid = threadIdx.x;
  for (int it = 0;; ++it) {
    const int tile = next_tile(it, persistent, w.queue, &s_item);
    if (tile >= n_tiles) break;
    const int s = scene_of_tile(w.scenes, n_scenes, tile);
    const SceneTab st = w.scenes[s];
    const int lt = tile - st.tile_off;
    const int x0 = (lt % st.tiles_x) * TILE, y0 = (lt / st.tiles_x) * TILE;
    float px[PPT], py[PPT], T[PPT], acc[PPT][C];
    int stop[PPT];
    bool done[PPT];
    const int start = ranges[2 * tile], end = ranges[2 * tile + 1];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int p = tid + q * THREADS;
      const int lx = p % TILE, ly = p / TILE;
      px[q] = (float)lx;
      py[q] = (float)ly;
      T[q] = 1.0f;
#pragma unroll
      for (int c = 0; c < C; ++c) acc[q][c] = 0.0f;
      stop[q] = start;
      done[q] = !(x0 + lx < st.W && y0 + ly < st.H);
    }
    const double ox = (double)x0 + 0.5, oy = (double)y0 + 0.5;
    for (int hi = end; hi > start; hi -= B) {
      const int n = min(B, hi - start);
      __syncthreads();
      for (int k = tid; k < n; k += THREADS) {
        const Gauss r = gs[idx[hi - 1 - k]];
        const double sg = (double)r.sigma;
        s_cx[k] = (float)(r.mx - ox);
        s_cy[k] = (float)(r.my - oy);
        s_a[k] = (float)(-0.5 * LOG2E / (sg * sg));
        const float rr = ks * r.sigma;
        s_r2[k] = rr * rr;
        s_o[k] = r.opacity;
#pragma unroll
        for (int c = 0; c < C; ++c) s_col[c][k] = cv.color[(int64_t)r.curve * C + c];
      }
      __syncthreads();
      for (int k = 0; k < n; ++k) {
        const float cx = s_cx[k], cy = s_cy[k], a = s_a[k], r2 = s_r2[k], o = s_o[k];
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
          if (done[q]) continue;
          const float dx = px[q] - cx, dy = py[q] - cy;
          const float d2 = __builtin_fmaf(dx, dx, dy * dy);
          if (d2 > r2) continue;
          const float G = __builtin_amdgcn_exp2f(a * d2);
          const float alpha = fminf(amax, o * G);
          const float wgt = alpha * T[q];
#pragma unroll
          for (int c = 0; c < C; ++c) acc[q][c] = __builtin_fmaf(s_col[c][k], wgt, acc[q][c]);
          T[q] = T[q] * (1.0f - alpha);
          if (T[q] < eps) {
            done[q] = true;
            stop[q] = hi - 1 - k;
          }
        }
      }
      bool mine = true;
#pragma unroll
      for (int q = 0; q < PPT; ++q) mine = mine && done[q];
      if (__syncthreads_and(mine)) break;
    }
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int p = tid + q * THREADS;
      const int x = x0 + p % TILE, y = y0 + p / TILE;
      if (x < st.W && y < st.H) {
        const int64_t pix = (int64_t)st.pix_off + (int64_t)y * st.W + x;
        const int64_t plane = (int64_t)st.H * st.W;
#pragma unroll
        for (int c = 0; c < C; ++c)
          image[(int64_t)st.pix_off * C + c * plane + (int64_t)y * st.W + x] =
              __builtin_fmaf(T[q], bg[s * C + c], acc[q][c]);
        Tfin[pix] = T[q];
        nlast[pix] = stop[q];
      }
    }
  }
}

__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

template <int C, int TILE>
__global__ __launch_bounds__(TileCfg<TILE>::THREADS) void k_blend_bwd(
    nsplat_curves cv, nsplat_params pr, Work w, int n_scenes, int n_tiles, const Gauss* __restrict__ gs,
    const int32_t* __restrict__ ranges, const int32_t* __restrict__ idx, const float* __restrict__ bg,
    const float* __restrict__ dL, const float* __restrict__ Tfin, const int32_t* __restrict__ nlast,
    int persistent) {
  constexpr int THREADS = TileCfg<TILE>::THREADS, PPT = TileCfg<TILE>::PPT;
  constexpr int NV = 4 + C;  // d/dmx, d/dmy, d/dsigma, d/dopacity, d/dcolour
  __shared__ float s_cx[MAX_BATCH], s_cy[MAX_BATCH], s_a[MAX_BATCH], s_r2[MAX_BATCH], s_o[MAX_BATCH];
  __shared__ float s_sg[MAX_BATCH];
  __shared__ float s_col[C][MAX_BATCH];
  __shared__ int s_g[MAX_BATCH];
  __shared__ int s_item, s_lo;
  const int B = pr.batch;
  const float amax = pr.alpha_max, ks = pr.k_sigma;
  const float ln2 = (float)LN2;
  const int tid = threadIdx.x, lane = __lane_id();
  float* __restrict__ ggrad = w.ggrad;
  for (int it = 0;; ++it) {
    const int tile = next_tile(it, persistent, w.queue, &s_item);
    if (tile >= n_tiles) break;
    const int s = scene_of_tile(w.scenes, n_scenes, tile);
    const SceneTab st = w.scenes[s];
    const int lt = tile - st.tile_off;
    const int x0 = (lt % st.tiles_x) * TILE, y0 = (lt / st.tiles_x) * TILE;
    const int start = ranges[2 * tile], end = ranges[2 * tile + 1];
    const int64_t plane = (int64_t)st.H * st.W;
    float px[PPT], py[PPT], T[PPT], A[PPT][C], gI[PPT][C];
    int stop[PPT];
    bool valid[PPT];
    if (tid == 0) s_lo = end;
    __syncthreads();
    int my_lo = end;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int p = tid + q * THREADS;
      const int lx = p % TILE, ly = p / TILE;
      px[q] = (float)lx;
      py[q] = (float)ly;
      valid[q] = (x0 + lx < st.W && y0 + ly < st.H);
      T[q] = 1.0f;
      stop[q] = end;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        A[q][c] = bg[s * C + c];
        gI[q][c] = 0.0f;
      }
      if (valid[q]) {
        const int64_t pix = (int64_t)st.pix_off + (int64_t)(y0 + ly) * st.W + (x0 + lx);
        T[q] = Tfin[pix];
        stop[q] = nlast[pix];
#pragma unroll
        for (int c = 0; c < C; ++c)
          gI[q][c] = dL[(int64_t)st.pix_off * C + c * plane + (int64_t)(y0 + ly) * st.W + (x0 + lx)];
        my_lo = min(my_lo, stop[q]);
      }
    }
    atomicMin(&s_lo, my_lo);
    __syncthreads();
    const int lo = max(s_lo, start);
    const double ox = (double)x0 + 0.5, oy = (double)y0 + 0.5;
    for (int base = lo; base < end; base += B) {
      const int n = min(B, end - base);
      __syncthreads();
      for (int k = tid; k < n; k += THREADS) {
        const int g = idx[base + k];
        const Gauss r = gs[g];
        const double sg = (double)r.sigma;
        s_g[k] = g;
        s_cx[k] = (float)(r.mx - ox);
        s_cy[k] = (float)(r.my - oy);
        s_a[k] = (float)(-0.5 * LOG2E / (sg * sg));
        const float rr = ks * r.sigma;
        s_r2[k] = rr * rr;
        s_o[k] = r.opacity;
        s_sg[k] = r.sigma;
#pragma unroll
        for (int c = 0; c < C; ++c) s_col[c][k] = cv.color[(int64_t)r.curve * C + c];
      }
      __syncthreads();
      for (int k = 0; k < n; ++k) {
        const int pos = base + k;
        const float cx = s_cx[k], cy = s_cy[k], a = s_a[k], r2 = s_r2[k], o = s_o[k];
        float v[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] = 0.0f;
        bool act = false;
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
          if (!valid[q] || pos < stop[q]) continue;
          const float dx = px[q] - cx, dy = py[q] - cy;
          const float d2 = __builtin_fmaf(dx, dx, dy * dy);
          if (d2 > r2) continue;
          act = true;
          const float G = __builtin_amdgcn_exp2f(a * d2);
          const float oG = o * G;
          const float alpha = fminf(amax, oG);
          const float onem = 1.0f - alpha;
          T[q] = T[q] / onem;  // transmittance in front of this Gaussian
          float dLda = 0.0f;
#pragma unroll
          for (int c = 0; c < C; ++c) {
            const float col = s_col[c][k];
            dLda = __builtin_fmaf(gI[q][c], col - A[q][c], dLda);
            v[4 + c] = __builtin_fmaf(gI[q][c], alpha * T[q], v[4 + c]);
            A[q][c] = __builtin_fmaf(alpha, col, onem * A[q][c]);
          }
          dLda *= T[q];
          if (oG < amax) {
            const float dG = dLda * o;
            const float dd2 = dG * G * a * ln2;  // d exp2(a d2) / d d2 = G a ln 2
            v[0] = __builtin_fmaf(-2.0f * dx, dd2, v[0]);
            v[1] = __builtin_fmaf(-2.0f * dy, dd2, v[1]);
            const float sg = s_sg[k];
            v[2] = __builtin_fmaf(dG * G, d2 / (sg * sg * sg), v[2]);
            v[3] = __builtin_fmaf(dLda, G, v[3]);
          }
        }
        if (__ballot(act) == 0ull) continue;
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
        if (lane == 0) {
          float* dst = ggrad + (int64_t)s_g[k] * 8;
#pragma unroll
          for (int i = 0; i < NV; ++i)
            if (v[i] != 0.0f) unsafeAtomicAdd(dst + i, v[i]);
        }
      }
    }
    __syncthreads();
  }
}

__global__ void k_reset_queue(int32_t* q) {
  if (threadIdx.x < 4 && blockIdx.x == 0) q[threadIdx.x] = 0;
}

template <class K>
int resident_grid(K kernel, int threads, int n_items, int n_cu) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  const int g = per_cu * n_cu;
  return g < n_items ? g : n_items;
}

template <int C, int TILE>
hipError_t fwd_t(const Launch& L, float* image, float* T_final, int32_t* n_last, int persistent) {
  constexpr int THREADS = TileCfg<TILE>::THREADS;
  const int n_tiles = (int)L.n_tiles;
  if (n_tiles <= 0) return hipSuccess;
  int grid = n_tiles;
  if (persistent) {
    grid = resident_grid(k_blend_fwd<C, TILE>, THREADS, n_tiles, L.n_cu);
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, L.stream, L.w.queue);
  }
  hipLaunchKernelGGL((k_blend_fwd<C, TILE>), dim3(grid), dim3(THREADS), 0, L.stream, *L.cv, *L.pr, L.w,
                     L.sc->n_scenes, n_tiles, (const Gauss*)L.bf->gauss, L.bf->ranges, L.bf->idx, L.sc->bg, image,
                     T_final, n_last, persistent);
  return hipGetLastError();
}

template <int C, int TILE>
hipError_t bwd_t(const Launch& L, const float* dL, const float* T_final, const int32_t* n_last, int persistent) {
  constexpr int THREADS = TileCfg<TILE>::THREADS;
  const int n_tiles = (int)L.n_tiles;
  if (n_tiles <= 0) return hipSuccess;
  int grid = n_tiles;
  if (persistent) {
    grid = resident_grid(k_blend_bwd<C, TILE>, THREADS, n_tiles, L.n_cu);
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, L.stream, L.w.queue);
  }
  hipLaunchKernelGGL((k_blend_bwd<C, TILE>), dim3(grid), dim3(THREADS), 0, L.stream, *L.cv, *L.pr, L.w,
                     L.sc->n_scenes, n_tiles, (const Gauss*)L.bf->gauss, L.bf->ranges, L.bf->idx, L.sc->bg, dL,
                     T_final, n_last, persistent);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_blend_fwd(const Launch& L, float* image, float* T_final, int32_t* n_last, int persistent) {
  const int C = L.cv->channels, t = L.pr->tile;
  if (C == 1) {
    if (t == 8) return fwd_t<1, 8>(L, image, T_final, n_last, persistent);
    if (t == 16) return fwd_t<1, 16>(L, image, T_final, n_last, persistent);
    return fwd_t<1, 32>(L, image, T_final, n_last, persistent);
  }
  if (t == 8) return fwd_t<3, 8>(L, image, T_final, n_last, persistent);
  if (t == 16) return fwd_t<3, 16>(L, image, T_final, n_last, persistent);
  return fwd_t<3, 32>(L, image, T_final, n_last, persistent);
}

hipError_t launch_blend_bwd(const Launch& L, const float* dL, const float* T_final, const int32_t* n_last,
                            int persistent) {
  const int C = L.cv->channels, t = L.pr->tile;
  if (C == 1) {
    if (t == 8) return bwd_t<1, 8>(L, dL, T_final, n_last, persistent);
    if (t == 16) return bwd_t<1, 16>(L, dL, T_final, n_last, persistent);
    return bwd_t<1, 32>(L, dL, T_final, n_last, persistent);
  }
  if (t == 8) return bwd_t<3, 8>(L, dL, T_final, n_last, persistent);
  if (t == 16) return bwd_t<3, 16>(L, dL, T_final, n_last, persistent);
  return bwd_t<3, 32>(L, dL, T_final, n_last, persistent);
}

}  // namespace nsp
