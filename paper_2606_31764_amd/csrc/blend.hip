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

// Block layout: 8x8 tiles use one wavefront; 16x16 and 32x32 tiles four, each
// wavefront owning one quadrant (8x8 or 16x16 pixels), each lane a BLK x BLK
// block of pixels.  A wavefront skips every staged Gaussian whose support
// square misses its quadrant (a uniform branch; results are unchanged because
// every pixel of the quadrant would fail the support test).
template <int TILE>
struct TileCfg {
  static constexpr int WAVES = TILE == 8 ? 1 : 4;
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int SUB = TILE == 8 ? 8 : TILE / 2;
  static constexpr int BLK = SUB / 8;
  static constexpr int PPT = BLK * BLK;
};

template <int TILE>
__device__ inline void pixel_of(int tid, int q, int* lx, int* ly) {
  using Cfg = TileCfg<TILE>;
  const int w = tid >> 6, lane = tid & 63;
  const int qx0 = (w & 1) * Cfg::SUB, qy0 = (w >> 1) * Cfg::SUB;
  *lx = qx0 + (lane & 7) * Cfg::BLK + q % Cfg::BLK;
  *ly = qy0 + (lane >> 3) * Cfg::BLK + q / Cfg::BLK;
}

// Next (scene, tile) work item: the block's own index, or the next entry of
// the device work queue for the persistent form.
__device__ inline int next_tile(int it, int persistent, int32_t* queue, int* s_item) {
  if (!persistent) return it == 0 ? (int)blockIdx.x : 0x7fffffff;
  __syncthreads();
  if (threadIdx.x == 0) *s_item = atomicAdd(queue, 1);
  __syncthreads();
  return *s_item;
}

// Staged Gaussian: tile-local centre (relative to the first pixel centre),
// squared support radius, exp2 coefficient -log2(e) / (2 sigma^2); a
// conservative culling radius; opacity and colour.
__device__ inline void stage_entry(const Gauss& r, double ox, double oy, float ks, const float* color, int C,
                                   float4* geo, float4* pc, float* rc) {
  const double sg = (double)r.sigma;
  const float rr = ks * r.sigma;
  *geo = make_float4((float)(r.mx - ox), (float)(r.my - oy), rr * rr, (float)(-0.5 * LOG2E / (sg * sg)));
  float4 q = make_float4(r.opacity, 0.f, 0.f, 0.f);
  q.y = color[(int64_t)r.curve * C];
  if (C == 3) {
    q.z = color[(int64_t)r.curve * C + 1];
    q.w = color[(int64_t)r.curve * C + 2];
  }
  *pc = q;
  *rc = rr * 1.0001f + 1e-4f;
}

// Builds this wavefront's list of the staged entries whose support square
// meets its quadrant (in staged order); returns its length.  Every lane of the
// wavefront must call it.
template <int TILE>
__device__ inline int compact_wave(const float4* geo, const float* rc, int n, int* wl) {
  using Cfg = TileCfg<TILE>;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const float qx0 = (float)((w & 1) * Cfg::SUB), qy0 = (float)((w >> 1) * Cfg::SUB);
  const float qx1 = qx0 + (float)(Cfg::SUB - 1), qy1 = qy0 + (float)(Cfg::SUB - 1);
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  int cnt = 0;
  for (int k0 = 0; k0 < n; k0 += 64) {
    const int k = k0 + lane;
    bool keep = false;
    if (k < n) {
      const float4 g = geo[k];
      const float r = rc[k];
      keep = !((g.x + r < qx0) || (g.x - r > qx1) || (g.y + r < qy0) || (g.y - r > qy1));
    }
    const uint64_t m = __ballot(keep);
    if (keep) wl[cnt + __popcll(m & lt)] = k;
    cnt += __popcll(m);
  }
  return cnt;
}

template <int C, int TILE>
__global__ __launch_bounds__(TileCfg<TILE>::THREADS) void k_blend_fwd(
    nsplat_curves cv, nsplat_params pr, Work w, int n_scenes, int n_tiles, const Gauss* __restrict__ gs,
    const int32_t* __restrict__ ranges, const int32_t* __restrict__ idx, const float* __restrict__ bg,
    float* __restrict__ image, float* __restrict__ Tfin, int32_t* __restrict__ nlast, int persistent) {
  using Cfg = TileCfg<TILE>;
  constexpr int THREADS = Cfg::THREADS, PPT = Cfg::PPT;
  __shared__ float4 s_geo[MAX_BATCH], s_pc[MAX_BATCH];
  __shared__ float s_rc[MAX_BATCH];
  __shared__ int s_wl[Cfg::WAVES][MAX_BATCH + 4];
  __shared__ int s_item;
  const int B = pr.batch;
  const float amax = pr.alpha_max, eps = pr.eps_T, ks = pr.k_sigma;
  const int tid = threadIdx.x, wv = tid >> 6;
  int* wl = s_wl[wv];
  for (int it = 0;; ++it) {
    const int tile = next_tile(it, persistent, w.queue, &s_item);
    if (tile >= n_tiles) break;
    const int s = scene_of_tile(w.scenes, n_scenes, tile);
    const SceneTab st = w.scenes[s];
    const int lt = tile - st.tile_off;
    const int x0 = (lt % st.tiles_x) * TILE, y0 = (lt / st.tiles_x) * TILE;
    float px[PPT], py[PPT], T[PPT], acc[PPT][4];
    int stop[PPT];
    bool done[PPT];
    const int start = ranges[2 * tile], end = ranges[2 * tile + 1];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      int lx, ly;
      pixel_of<TILE>(tid, q, &lx, &ly);
      px[q] = (float)lx;
      py[q] = (float)ly;
      T[q] = 1.0f;
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[q][c] = 0.0f;
      stop[q] = start;
      done[q] = !(x0 + lx < st.W && y0 + ly < st.H);
    }
    const double ox = (double)x0 + 0.5, oy = (double)y0 + 0.5;
    for (int hi = end; hi > start; hi -= B) {
      const int n = min(B, hi - start);
      __syncthreads();
      for (int k = tid; k < n; k += THREADS)
        stage_entry(gs[idx[hi - 1 - k]], ox, oy, ks, cv.color, C, &s_geo[k], &s_pc[k], &s_rc[k]);
      __syncthreads();
      const int cnt = compact_wave<TILE>(s_geo, s_rc, n, wl);
      __syncthreads();
      int jstop[PPT];
#pragma unroll
      for (int q = 0; q < PPT; ++q) jstop[q] = -1;
      for (int j = 0; j < cnt; ++j) {
        const int k = wl[j];
        const float4 gm = s_geo[k];
        const float4 pc = s_pc[k];
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
          const float dx = px[q] - gm.x, dy = py[q] - gm.y;
          const float d2 = __builtin_fmaf(dx, dx, dy * dy);
          const float G = __builtin_amdgcn_exp2f(gm.w * d2);
          const bool in = (d2 <= gm.z) && !done[q];
          const float alpha = in ? fminf(amax, pc.x * G) : 0.0f;
          const float wgt = alpha * T[q];
          acc[q][0] = __builtin_fmaf(pc.y, wgt, acc[q][0]);
          if (C == 3) {
            acc[q][1] = __builtin_fmaf(pc.z, wgt, acc[q][1]);
            acc[q][2] = __builtin_fmaf(pc.w, wgt, acc[q][2]);
          }
          T[q] = T[q] * (1.0f - alpha);
          const bool now = in && (T[q] < eps);
          jstop[q] = now ? j : jstop[q];
          done[q] = done[q] || now;
        }
      }
      bool mine = true;
#pragma unroll
      for (int q = 0; q < PPT; ++q) {
        if (jstop[q] >= 0) stop[q] = hi - 1 - wl[jstop[q]];
        mine = mine && done[q];
      }
      if (__syncthreads_and(mine)) break;
    }
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      int lx, ly;
      pixel_of<TILE>(tid, q, &lx, &ly);
      const int x = x0 + lx, y = y0 + ly;
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

// Sum over the 64 lanes of a wavefront with DPP row shifts and row
// broadcasts (no LDS traffic): inclusive sums inside each row of 16 lanes,
// then row 0 into row 1, row 2 into row 3, and rows 0-1 into row 3; lane 63
// ends with the total, which is returned to every lane.
__device__ inline float wave_total(float v) {
  int x = __float_as_int(v);
  x = __float_as_int(__int_as_float(x) + __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true)));
  x = __float_as_int(__int_as_float(x) + __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true)));
  x = __float_as_int(__int_as_float(x) + __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true)));
  x = __float_as_int(__int_as_float(x) + __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true)));
  x = __float_as_int(__int_as_float(x) + __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false)));
  x = __float_as_int(__int_as_float(x) + __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false)));
  return __int_as_float(__builtin_amdgcn_readlane(x, 63));
}

// Flushes one wavefront's running per-curve sums (colour, and opacity for a
// stroke curve) into the FP64 per-curve accumulators.
template <int C>
__device__ inline void flush_curve(double* gcurve, int c, bool fill, float (&accC)[3], float& accO) {
  double* dst = gcurve + 4 * (int64_t)c;
#pragma unroll
  for (int ch = 0; ch < C; ++ch) {
    const float t = wave_total(accC[ch]);
    if (__lane_id() == 0 && t != 0.0f) unsafeAtomicAdd(dst + 1 + ch, (double)t);
    accC[ch] = 0.0f;
  }
  if (!fill) {
    const float t = wave_total(accO);
    if (__lane_id() == 0 && t != 0.0f) unsafeAtomicAdd(dst, (double)t);
  }
  accO = 0.0f;
}

// Adjoint of the forward blend.  Per Gaussian it accumulates, over the
// pixels of the tile, dL/dmu and dL/dsigma for stroke Gaussians and dL/do_j
// for fill Gaussians (whose own opacity carries the SDF); colour gradients
// (and a stroke curve's opacity gradient, its o_j all being o) belong to the
// curve, so each lane keeps running per-curve sums that are flushed when the
// curve changes along the list or every FLUSH entries.
template <int C, int TILE>
__global__ __launch_bounds__(TileCfg<TILE>::THREADS) void k_blend_bwd(
    nsplat_curves cv, nsplat_params pr, Work w, int n_scenes, int n_tiles, const Gauss* __restrict__ gs,
    const int32_t* __restrict__ ranges, const int32_t* __restrict__ idx, const float* __restrict__ bg,
    const float* __restrict__ dL, const float* __restrict__ Tfin, const int32_t* __restrict__ nlast,
    int persistent) {
  using Cfg = TileCfg<TILE>;
  constexpr int THREADS = Cfg::THREADS, PPT = Cfg::PPT;
  constexpr int FLUSH = 32;
  __shared__ float4 s_geo[MAX_BATCH], s_pc[MAX_BATCH];
  __shared__ float s_rc[MAX_BATCH], s_is3[MAX_BATCH];
  __shared__ int s_g[MAX_BATCH], s_cur[MAX_BATCH];
  __shared__ int s_wl[Cfg::WAVES][MAX_BATCH + 4];
  __shared__ int s_item, s_lo;
  const int B = pr.batch;
  const float amax = pr.alpha_max, ks = pr.k_sigma;
  const float ln2 = (float)LN2;
  const int tid = threadIdx.x, lane = __lane_id(), wv = tid >> 6;
  int* wl = s_wl[wv];
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
    float px[PPT], py[PPT], T[PPT], A[PPT][4], gI[PPT][4];
    int stop[PPT];
    if (tid == 0) s_lo = end;
    __syncthreads();
    int my_lo = end;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      int lx, ly;
      pixel_of<TILE>(tid, q, &lx, &ly);
      px[q] = (float)lx;
      py[q] = (float)ly;
      T[q] = 1.0f;
      stop[q] = end;  // invalid pixels never take part
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        A[q][c] = c < C ? bg[s * C + c] : 0.0f;
        gI[q][c] = 0.0f;
      }
      if (x0 + lx < st.W && y0 + ly < st.H) {
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
    int cur = -1, since = 0;
    bool cur_fill = false;
    float accC[3] = {0.0f, 0.0f, 0.0f}, accO = 0.0f;
    for (int base = lo; base < end; base += B) {
      const int n = min(B, end - base);
      __syncthreads();
      for (int k = tid; k < n; k += THREADS) {
        const int g = idx[base + k];
        const Gauss r = gs[g];
        stage_entry(r, ox, oy, ks, cv.color, C, &s_geo[k], &s_pc[k], &s_rc[k]);
        const double sg = (double)r.sigma;
        s_g[k] = (cv.flags[r.curve] & NSPLAT_FILLED) ? ~g : g;
        s_cur[k] = r.curve;
        s_is3[k] = (float)(1.0 / (sg * sg * sg));
      }
      __syncthreads();
      const int cnt = compact_wave<TILE>(s_geo, s_rc, n, wl);
      __syncthreads();
      for (int j = 0; j < cnt; ++j) {
        const int k = wl[j];
        const int pos = base + k;
        const int gsig = __builtin_amdgcn_readfirstlane(s_g[k]);
        const int c_k = __builtin_amdgcn_readfirstlane(s_cur[k]);
        const bool fill = gsig < 0;
        if (c_k != cur || since >= FLUSH) {
          if (cur >= 0) flush_curve<C>(w.gcurve, cur, cur_fill, accC, accO);
          cur = c_k;
          cur_fill = fill;
          since = 0;
        }
        ++since;
        const float4 gm = s_geo[k];
        const float4 pc = s_pc[k];
        const float col[3] = {pc.y, pc.z, pc.w};
        float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        bool act = false;
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
          const float dx = px[q] - gm.x, dy = py[q] - gm.y;
          const float d2 = __builtin_fmaf(dx, dx, dy * dy);
          const bool in = (pos >= stop[q]) && (d2 <= gm.z);
          act = act || in;
          const float G = __builtin_amdgcn_exp2f(gm.w * d2);
          const float oG = pc.x * G;
          const float alpha = in ? fminf(amax, oG) : 0.0f;
          const float onem = 1.0f - alpha;
          T[q] = T[q] / onem;  // transmittance in front of this Gaussian (unchanged when alpha = 0)
          const float aT = alpha * T[q];
          float dLda = 0.0f;
#pragma unroll
          for (int c = 0; c < C; ++c) {
            dLda = __builtin_fmaf(gI[q][c], col[c] - A[q][c], dLda);
            accC[c] = __builtin_fmaf(gI[q][c], aT, accC[c]);
            A[q][c] = __builtin_fmaf(alpha, col[c], onem * A[q][c]);
          }
          dLda = (in && oG < amax) ? dLda * T[q] : 0.0f;
          v[3] = __builtin_fmaf(dLda, G, v[3]);  // dL/do_j
          if (!fill) {
            const float dG = dLda * pc.x;
            const float dd2 = dG * G * gm.w * ln2;  // d exp2(a d2) / d d2 = G a ln 2
            v[0] = __builtin_fmaf(-2.0f * dx, dd2, v[0]);
            v[1] = __builtin_fmaf(-2.0f * dy, dd2, v[1]);
            v[2] = __builtin_fmaf(dG * G, d2 * s_is3[k], v[2]);
          }
        }
        if (__ballot(act) == 0ull) continue;
        float* dst = ggrad + (int64_t)(fill ? ~gsig : gsig) * GG;
        if (fill) {
          const float t = wave_total(v[3]);
          if (lane == 0 && t != 0.0f) unsafeAtomicAdd(dst + 3, t);
        } else {
          accO += v[3];
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            const float t = wave_total(v[i]);
            if (lane == 0 && t != 0.0f) unsafeAtomicAdd(dst + i, t);
          }
        }
      }
    }
    if (cur >= 0) flush_curve<C>(w.gcurve, cur, cur_fill, accC, accO);
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
  Phase ph(L, NSPLAT_T_BLEND_FWD);
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
  Phase ph(L, NSPLAT_T_BLEND_BWD);
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
