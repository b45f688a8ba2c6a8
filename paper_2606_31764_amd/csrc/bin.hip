// nsplat_bin: Gaussians -> per-tile lists (Sec. 3.4).
//
//   k_bin_count   one lane per Gaussian: conservative tile rectangle in FP32
//   scan          exclusive prefix sum of the counts -> pair offsets
//   k_bin_emit    writes (global tile key, Gaussian index) pairs in Gaussian order
//   radix passes  stable LSD radix sort on the key (histogram, scan, scatter
//                 with wavefront match-ranking), so each tile keeps ascending
//                 Gaussian order
//   (up to RADIX_MAX tiles, one digit: k_bin_tilehist counts each block's
//   pairs per tile, one scan turns the counts into list positions and
//   k_bin_place writes every pair at its final place, in the same order)
//   k_tile_ranges [begin, end) of every tile's slice (after a one-pass sort the
//                 tile plan reads them off the scanned digit counts instead)
//   k_order_*     the blend kernels' tile order, longest lists first
//   k_chunk_counts, k_item_counts + scans: checkpoint slots per tile and the
//                 adjoint's (tile, quadrant, chunk) items in blend order
#include "nsplat_internal.h"

namespace nsp {

namespace {

struct Rect {
  int x0, x1, y0, y1;
};

// Tile rectangle of one Gaussian: centre m = fl32(mu), r = k_sigma * sigma in
// FP32, interval [(m - r) - 1, (m + r) + 1], tile = floor(x / tile), clamped
// (tile_axis, shared with the blend kernels' fill runs).
__device__ inline bool tile_rect(const Gauss& gs, float k_sigma, float inv_tile, const SceneTab& st, Rect* rc) {
  const float mx = (float)gs.mx, my = (float)gs.my;
  const float r = k_sigma * gs.sigma;
  float fx0, fx1, fy0, fy1;
  if (!tile_axis(mx, r, inv_tile, st.tiles_x, &fx0, &fx1) || !tile_axis(my, r, inv_tile, st.tiles_y, &fy0, &fy1))
    return false;
  if (fx0 > fx1 || fy0 > fy1) return false;
  rc->x0 = (int)fx0;
  rc->x1 = (int)fx1;
  rc->y0 = (int)fy0;
  rc->y1 = (int)fy1;
  return true;
}

// Also clears the tile ranges (n_ranges entries) that k_tile_ranges fills in
// after the sort.
__global__ __launch_bounds__(256) void k_bin_count(nsplat_curves cv, nsplat_params pr, Work w,
                                                   const Gauss* __restrict__ gs, const int32_t* counters,
                                                   uint32_t* __restrict__ cnt, int32_t* __restrict__ ranges,
                                                   int64_t n_ranges) {
  const int64_t G = counters[NSPLAT_CNT_GAUSS];
  const float inv = 1.0f / (float)pr.tile;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_ranges; i += (int64_t)gridDim.x * blockDim.x)
    ranges[i] = 0;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < G; g += (int64_t)gridDim.x * blockDim.x) {
    const Gauss r = gs[g];
    const SceneTab st = w.scenes[cv.scene[r.curve]];
    Rect rc;
    uint32_t n = 0;
    if (tile_rect(r, pr.k_sigma, inv, st, &rc)) n = (uint32_t)((rc.x1 - rc.x0 + 1) * (rc.y1 - rc.y0 + 1));
    cnt[g] = n;
  }
}

// Pair count from the scan total, its capped value (0 with none_on_cap: a
// binning that writes no pair on an overflow), and the capacity flag.
__device__ inline void pairs_total(int32_t* counters, const uint32_t* total, int64_t cap, bool none_on_cap = false) {
  const uint32_t t = *total;
  counters[NSPLAT_CNT_PAIRS_REQ] = t > 0x7fffffffu ? 0x7fffffff : (int32_t)t;
  counters[NSPLAT_CNT_PAIRS] = (int32_t)((int64_t)t <= cap ? (int64_t)t : (none_on_cap ? 0 : cap));
  int32_t st = counters[NSPLAT_CNT_STATUS] & ~NSPLAT_STATUS_PAIR_CAP;
  if ((int64_t)t > cap) st |= NSPLAT_STATUS_PAIR_CAP;
  counters[NSPLAT_CNT_STATUS] = st;
}

// Thread 0 also publishes the pair count (off[G_cap] holds the scan total);
// no thread of this kernel reads it.  With more pairs than `cap` no pair is
// written and the count is 0.
__global__ __launch_bounds__(256) void k_bin_emit(nsplat_curves cv, nsplat_params pr, Work w,
                                                  const Gauss* __restrict__ gs, int32_t* counters,
                                                  const uint32_t* __restrict__ off, const uint32_t* total,
                                                  uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                  int64_t cap) {
  if (blockIdx.x == 0 && threadIdx.x == 0) pairs_total(counters, total, cap, true);
  if ((int64_t)*total > cap) return;  // an overflow writes no pair (the lists stay empty)
  const int64_t G = counters[NSPLAT_CNT_GAUSS];
  const float inv = 1.0f / (float)pr.tile;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < G; g += (int64_t)gridDim.x * blockDim.x) {
    const Gauss r = gs[g];
    const SceneTab st = w.scenes[cv.scene[r.curve]];
    Rect rc;
    if (!tile_rect(r, pr.k_sigma, inv, st, &rc)) continue;
    int64_t pos = off[g];
    for (int ty = rc.y0; ty <= rc.y1; ++ty)
      for (int tx = rc.x0; tx <= rc.x1; ++tx, ++pos)
        if (pos < cap) {
          keys[pos] = (uint32_t)(st.tile_off + ty * st.tiles_x + tx);
          vals[pos] = (uint32_t)g;
        }
  }
}

// One-digit binning (at most RADIX_MAX tiles): the pairs go straight to
// their sorted places, in the order the emission and a stable one-pass
// radix sort give (tile, then Gaussian).  Block b owns the Gaussians
// [b FB_ITEMS, (b + 1) FB_ITEMS).  k_bin_tilehist stores its pair count per
// tile key in row `key`, column b, of hist, and its pair total in row nd;
// one exclusive scan over the rows makes row `key`, column b, the list
// position of the block's first pair with that key, and row nd, column 0,
// the pair total.  k_bin_place then recomputes each Gaussian's tile
// rectangle and writes its Gaussian index at the position: wavefront w of
// the block owns 64 FB_PER_LANE consecutive Gaussians, counts their pairs per
// key, adds the counts of the earlier wavefronts to the block's positions,
// and places its pairs in Gaussian order (rectangle rows, then columns, per
// Gaussian) 64 at a time, ranking equal keys with ballots, through a window
// of FB_WIN pairs staged in LDS.
constexpr int FB_THREADS = 1024;
constexpr int FB_WAVES = FB_THREADS / 64;
constexpr int FB_PER_LANE = FB_ITEMS / FB_THREADS;  // 4
constexpr int FB_WIN = 256;
static_assert(FB_ITEMS == FB_THREADS * FB_PER_LANE, "Gaussians per block");

__device__ inline uint32_t wave_incl_scan_u32(uint32_t v) {
  const int lane = __lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(v, off);
    if (lane >= off) v += o;
  }
  return v;
}

// Lanes whose Gaussian has the same tile rectangle as the previous lane's
// (fill lattice points in a row mostly do) are counted by the first lane of
// their run: it returns the run's length, the others 0.
__device__ inline uint32_t rect_run(bool ok, int key0, int wdt, int n) {
  const int lane = __lane_id();
  const int pk = __shfl_up(key0, 1), pw = __shfl_up(wdt, 1), pn = __shfl_up(n, 1);
  const bool pok = __shfl_up((int)ok, 1) != 0;
  const bool same = ok && lane > 0 && pok && pk == key0 && pw == wdt && pn == n;
  const uint64_t sm = __ballot(same);
  if (!ok || same) return 0u;
  const uint64_t after = lane == 63 ? 0ull : (sm >> (lane + 1));
  return 1u + (uint32_t)__builtin_ctzll(~after);
}

// Tile rectangles of the Gaussians g0 + i * stride, i < FB_PER_LANE, with
// their loads issued together: key of the first tile, width, tile count (0
// when none or past G), and the scene's tile columns.
__device__ inline void fb_rects(const nsplat_curves& cv, const nsplat_params& pr, const Work& w,
                                const Gauss* __restrict__ gs, int64_t G, int64_t g0, int stride, float inv,
                                int (&key0)[FB_PER_LANE], int (&wdt)[FB_PER_LANE], int (&n)[FB_PER_LANE],
                                int (&sx)[FB_PER_LANE]) {
  Gauss r[FB_PER_LANE];
  int sc[FB_PER_LANE];
#pragma unroll
  for (int i = 0; i < FB_PER_LANE; ++i) {
    const int64_t g = g0 + (int64_t)i * stride;
    if (g < G) r[i] = gs[g];
    else r[i].curve = -1;
  }
#pragma unroll
  for (int i = 0; i < FB_PER_LANE; ++i) sc[i] = r[i].curve >= 0 ? cv.scene[r[i].curve] : 0;
#pragma unroll
  for (int i = 0; i < FB_PER_LANE; ++i) {
    const SceneTab st = w.scenes[sc[i]];
    Rect rc;
    key0[i] = wdt[i] = n[i] = sx[i] = 0;
    if (r[i].curve >= 0 && tile_rect(r[i], pr.k_sigma, inv, st, &rc)) {
      key0[i] = st.tile_off + rc.y0 * st.tiles_x + rc.x0;
      sx[i] = st.tiles_x;
      wdt[i] = rc.x1 - rc.x0 + 1;
      n[i] = wdt[i] * (rc.y1 - rc.y0 + 1);
    }
  }
}

__device__ inline uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__global__ __launch_bounds__(FB_THREADS) void k_bin_tilehist(nsplat_curves cv, nsplat_params pr, Work w,
                                                             const Gauss* __restrict__ gs, const int32_t* counters,
                                                             int nd, int nb, uint32_t* __restrict__ hist,
                                                             int32_t* __restrict__ ranges, int64_t n_ranges) {
  __shared__ uint32_t h[RADIX_MAX];
  __shared__ uint32_t wt[FB_WAVES];
  const int col = blockIdx.x;
  const int64_t G = counters[NSPLAT_CNT_GAUSS];
  const float inv = 1.0f / (float)pr.tile;
  const int t = threadIdx.x;
  const uint32_t mask = (uint32_t)nd - 1u;  // the low digit of the tile key
  // (the tile ranges that k_tile_ranges fills in after a multi-pass sort)
  for (int64_t i = (int64_t)col * FB_THREADS + t; i < n_ranges; i += (int64_t)nb * FB_THREADS) ranges[i] = 0;
  for (int d = t; d < nd; d += FB_THREADS) h[d] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)col * FB_ITEMS;
  uint32_t tot = 0u;
  int key0[FB_PER_LANE], wdt[FB_PER_LANE], kn[FB_PER_LANE], sx[FB_PER_LANE];
  fb_rects(cv, pr, w, gs, G, base + t, FB_THREADS, inv, key0, wdt, kn, sx);
#pragma unroll
  for (int i = 0; i < FB_PER_LANE; ++i) {
    const uint32_t run = rect_run(kn[i] > 0, key0[i], wdt[i], kn[i]);
    if (run > 0u)
      for (int r = 0, key = key0[i]; r < kn[i]; r += wdt[i], key += sx[i])
        for (int x = 0; x < wdt[i]; ++x) atomicAdd(&h[(uint32_t)(key + x) & mask], run);
    tot += (uint32_t)kn[i];
  }
  tot = wave_sum_u32(tot);
  if (__lane_id() == 0) wt[t >> 6] = tot;
  __syncthreads();
  for (int d = t; d < nd; d += FB_THREADS) hist[(int64_t)d * nb + col] = h[d];
  if (t == 0) {
    uint32_t s = 0u;
#pragma unroll
    for (int q = 0; q < FB_WAVES; ++q) s += wt[q];
    hist[(int64_t)nd * nb + col] = s;
  }
}

// hist: scanned.  Block 0 publishes the pair count; with more pairs than
// `cap` nothing is written and the count is 0 (the tile plan then leaves
// every list empty).  Places by the low digit (nd = 2^bits values) of the
// tile key; with keys != nullptr also writes the keys (the input of the
// remaining radix passes of a key wider than one digit).
__global__ __launch_bounds__(FB_THREADS) void k_bin_place(nsplat_curves cv, nsplat_params pr, Work w,
                                                          const Gauss* __restrict__ gs, int32_t* counters, int nd,
                                                          int nb, int bits, const uint32_t* __restrict__ hist,
                                                          uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                          int64_t cap) {
  __shared__ uint32_t off[FB_WAVES][RADIX_MAX];
  __shared__ uint32_t lkey[FB_WAVES][FB_WIN], lval[FB_WAVES][FB_WIN];
  const uint32_t* total = hist + (int64_t)nd * nb;  // row nd, column 0: the pair total
  if (blockIdx.x == 0 && threadIdx.x == 0) pairs_total(counters, total, cap, true);
  if ((int64_t)*total > cap) return;
  const uint32_t mask = (uint32_t)nd - 1u;
  const int col = blockIdx.x;
  const int64_t G = counters[NSPLAT_CNT_GAUSS];
  const int64_t base = (int64_t)col * FB_ITEMS;
  if (base >= G) return;
  const float inv = 1.0f / (float)pr.tile;
  const int t = threadIdx.x, lane = __lane_id(), wid = t >> 6;
  for (int d = lane; d < nd; d += 64) off[wid][d] = 0u;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // this wavefront's Gaussians, lane-interleaved: g = wbase + 64 i + lane
  const int64_t wbase = base + (int64_t)wid * (64 * FB_PER_LANE);
  int kx0[FB_PER_LANE], kw[FB_PER_LANE], kn[FB_PER_LANE], ksx[FB_PER_LANE];
  fb_rects(cv, pr, w, gs, G, wbase + lane, 64, inv, kx0, kw, kn, ksx);
#pragma unroll
  for (int i = 0; i < FB_PER_LANE; ++i) {
    const uint32_t run = rect_run(kn[i] > 0, kx0[i], kw[i], kn[i]);
    if (run > 0u)
      for (int r = 0, key = kx0[i]; r < kn[i]; r += kw[i], key += ksx[i])
        for (int x = 0; x < kw[i]; ++x) atomicAdd(&off[wid][(uint32_t)(key + x) & mask], run);
  }
  __syncthreads();
  // per key: the block's first position plus the counts of the earlier
  // wavefronts (read only for the keys the block holds: a block's Gaussians
  // reach few tiles)
  for (int d = t; d < nd; d += FB_THREADS) {
    uint32_t c[FB_WAVES], any = 0u;
#pragma unroll
    for (int q = 0; q < FB_WAVES; ++q) {
      c[q] = off[q][d];
      any |= c[q];
    }
    if (any == 0u) continue;
    uint32_t run = hist[(int64_t)d * nb + col];
#pragma unroll
    for (int q = 0; q < FB_WAVES; ++q) {
      off[q][d] = run;
      run += c[q];
    }
  }
  __syncthreads();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int i = 0; i < FB_PER_LANE; ++i) {
    // this round's pairs in Gaussian order: lane l's at [e, e + kn)
    const uint32_t n = (uint32_t)kn[i];
    const uint32_t e = wave_incl_scan_u32(n) - n;
    const int R = __builtin_amdgcn_readlane((int)(e + n), 63);
    const uint32_t g = (uint32_t)(wbase + 64 * i + lane);
    // large rectangles (some lane with more than 16 pairs) are expanded by
    // list position: every lane fills window slots, each finding the lane
    // whose pairs hold it, so that one large rectangle does not serialise
    // the wavefront
    const bool spread = __ballot(n > 16u) != 0ull;
    for (int w0 = 0; w0 < R; w0 += FB_WIN) {
      if (!spread) {
        const int k0 = max(0, w0 - (int)e), k1 = min((int)n, w0 + FB_WIN - (int)e);
        if (k0 < k1) {
          // rectangle position of pair k0, then stepped along its rows
          const int ry = k0 / kw[i];
          int x = k0 - ry * kw[i], key = kx0[i] + ry * ksx[i];
          for (int k = k0; k < k1; ++k) {
            lkey[wid][(int)e + k - w0] = (uint32_t)(key + x);
            lval[wid][(int)e + k - w0] = g;
            if (++x == kw[i]) {
              x = 0;
              key += ksx[i];
            }
          }
        }
      } else {
        const int m = min(FB_WIN, R - w0);
        for (int j = 0; j < m; j += 64) {
          const int q = w0 + j + lane;  // list position of this slot
          // the last lane whose first position is at most q owns it
          int lo = 0;
#pragma unroll
          for (int step = 32; step >= 1; step >>= 1) {
            const int mid = lo + step;
            if ((int)__shfl((int)e, mid) <= q) lo = mid;
          }
          const int oe = __shfl((int)e, lo), ow = __shfl(kw[i], lo), ok0 = __shfl(kx0[i], lo),
                    osx = __shfl(ksx[i], lo);
          if (j + lane < m) {
            const int k = q - oe, ry = k / ow;
            lkey[wid][j + lane] = (uint32_t)(ok0 + ry * osx + (k - ry * ow));
            lval[wid][j + lane] = (uint32_t)(wbase + 64 * i + lo);
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const int m = min(FB_WIN, R - w0);
      for (int j = 0; j < m; j += 64) {
        const bool active = j + lane < m;
        const uint32_t key = active ? lkey[wid][j + lane] : 0u;
        const uint32_t val = active ? lval[wid][j + lane] : 0u;
        const uint32_t dig = key & mask;
        uint64_t peers = __ballot(active);
        for (int b = 0; b < bits; ++b) {
          const bool bit = (dig >> b) & 1u;
          const uint64_t bal = __ballot(bit);
          peers &= bit ? bal : ~bal;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
        const uint32_t o = off[wid][dig];
        if (active) {
          vals[o + rank] = val;
          if (keys) keys[o + rank] = key;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (active && rank == 0) off[wid][dig] = o + (uint32_t)__popcll(peers);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
  }
}

constexpr int SORT_THREADS = 256;
constexpr int SORT_ROUNDS = SORT_ITEMS / SORT_THREADS;  // 16
constexpr int SORT_WAVES = SORT_THREADS / 64;

__global__ __launch_bounds__(SORT_THREADS) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                             const int32_t* counters, int shift, int bits,
                                                             uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[RADIX_MAX];
  const int64_t n = counters[NSPLAT_CNT_PAIRS];
  const int nb = gridDim.x, nd = 1 << bits;
  const uint32_t mask = (1u << bits) - 1u;
  for (int d = threadIdx.x; d < nd; d += SORT_THREADS) h[d] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * SORT_ITEMS;
  for (int i = 0; i < SORT_ROUNDS; ++i) {
    const int64_t k = base + (int64_t)i * SORT_THREADS + threadIdx.x;
    if (k < n) atomicAdd(&h[(keys[k] >> shift) & mask], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < nd; d += SORT_THREADS) hist[(int64_t)d * nb + blockIdx.x] = h[d];
}

// Stable scatter for digits of 9 to RADIX_BITS_MAX bits.  Wavefront w of the
// block owns the contiguous items base + 1024 w .. base + 1024 w + 1023: it
// counts their digits into its own LDS row, the rows are turned into
// per-wavefront starting offsets (block offset from the scanned histogram
// plus the counts of the earlier wavefronts), and each wavefront then places
// its items in order, 64 at a time, ranking equal digits with ballots and
// advancing only its own offsets, so no block barrier is needed per round.
__global__ __launch_bounds__(SORT_THREADS) void k_radix_scatter_wide(const uint32_t* __restrict__ kin,
                                                                     const uint32_t* __restrict__ vin,
                                                                     uint32_t* __restrict__ kout,
                                                                     uint32_t* __restrict__ vout,
                                                                     const int32_t* counters, int shift, int bits,
                                                                     const uint32_t* __restrict__ hist) {
  static_assert(SORT_ITEMS == SORT_WAVES * 1024, "1024 items per wavefront");
  __shared__ uint32_t off[SORT_WAVES][RADIX_MAX];
  const int64_t n = counters[NSPLAT_CNT_PAIRS];
  const int nb = gridDim.x, nd = 1 << bits;
  const int64_t base = (int64_t)blockIdx.x * SORT_ITEMS;
  if (base >= n) return;
  const uint32_t mask = (1u << bits) - 1u;
  const int t = threadIdx.x, lane = __lane_id(), wid = t >> 6;
  for (int d = t; d < SORT_WAVES * nd; d += SORT_THREADS) off[d / nd][d % nd] = 0u;
  __syncthreads();
  const int64_t wbase = base + (int64_t)wid * 1024;
  uint32_t key[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t k = wbase + r * 64 + lane;
    key[r] = k < n ? kin[k] : 0u;
    if (k < n) atomicAdd(&off[wid][(key[r] >> shift) & mask], 1u);
  }
  __syncthreads();
  for (int d = t; d < nd; d += SORT_THREADS) {
    uint32_t run = hist[(int64_t)d * nb + blockIdx.x];
#pragma unroll
    for (int q = 0; q < SORT_WAVES; ++q) {
      const uint32_t c = off[q][d];
      off[q][d] = run;
      run += c;
    }
  }
  __syncthreads();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t k = wbase + r * 64 + lane;
    const bool active = k < n;
    const uint32_t dig = (key[r] >> shift) & mask;
    uint64_t peers = __ballot(active);
    for (int b = 0; b < bits; ++b) {
      const bool bit = (dig >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
    const uint32_t o = off[wid][dig];
    if (active) {
      kout[o + rank] = key[r];
      vout[o + rank] = vin[k];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (active && rank == 0) off[wid][dig] = o + (uint32_t)__popcll(peers);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// Stable scatter.  Round i handles items base + i * 256 + t, so ascending
// (round, thread) is ascending input order; each item's rank among the
// earlier items of the block with the same digit comes from wavefront ballots
// (lanes whose digit matches in every bit) plus per-wave and per-round running
// counts kept in LDS.
__global__ __launch_bounds__(SORT_THREADS) void k_radix_scatter(const uint32_t* __restrict__ kin,
                                                                const uint32_t* __restrict__ vin,
                                                                uint32_t* __restrict__ kout,
                                                                uint32_t* __restrict__ vout,
                                                                const int32_t* counters, int shift, int bits,
                                                                const uint32_t* __restrict__ hist) {
  __shared__ uint32_t base_off[256];
  __shared__ uint32_t wcnt[SORT_WAVES][256];
  const int64_t n = counters[NSPLAT_CNT_PAIRS];
  const int nb = gridDim.x;
  const int64_t base = (int64_t)blockIdx.x * SORT_ITEMS;
  if (base >= n) return;
  const uint32_t mask = (1u << bits) - 1u;
  const int t = threadIdx.x, lane = __lane_id(), wid = t >> 6;
  base_off[t] = (t < (1 << bits)) ? hist[(int64_t)t * nb + blockIdx.x] : 0u;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int i = 0; i < SORT_ROUNDS; ++i) {
#pragma unroll
    for (int q = 0; q < SORT_WAVES; ++q) wcnt[q][t] = 0;
    __syncthreads();
    const int64_t k = base + (int64_t)i * SORT_THREADS + t;
    const bool active = k < n;
    uint32_t key = 0, val = 0, dig = 0;
    if (active) {
      key = kin[k];
      val = vin[k];
      dig = (key >> shift) & mask;
    }
    uint64_t peers = __ballot(active);
    for (int b = 0; b < bits; ++b) {
      const bool bit = (dig >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
    if (active && rank == 0) wcnt[wid][dig] = (uint32_t)__popcll(peers);
    __syncthreads();
    // per digit: exclusive prefix over waves, then advance the running offset
    if (t < (1 << bits)) {
      uint32_t run = base_off[t];
#pragma unroll
      for (int q = 0; q < SORT_WAVES; ++q) {
        const uint32_t c = wcnt[q][t];
        wcnt[q][t] = run;
        run += c;
      }
      base_off[t] = run;
    }
    __syncthreads();
    if (active) {
      const uint32_t pos = wcnt[wid][dig] + rank;
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
  }
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ __launch_bounds__(256) void k_tile_ranges(const uint32_t* __restrict__ keys, const int32_t* counters,
                                                     int32_t* __restrict__ ranges) {
  const int64_t n = counters[NSPLAT_CNT_PAIRS];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t k = keys[i];
    if (i == 0 || keys[i - 1] != k) ranges[2 * (int64_t)k] = (int32_t)i;
    if (i == n - 1 || keys[i + 1] != k) ranges[2 * (int64_t)k + 1] = (int32_t)(i + 1);
  }
}

// Tiles in order of decreasing list length, by power-of-two class, so that
// the blend kernels start the long lists first and fill in with short ones.
// Only the processing order changes (each (tile, quadrant) item writes its
// own pixels); the order inside a class is whatever the atomics give.
__device__ inline int len_class(const int32_t* __restrict__ ranges, int t) {
  const int k = __clz(ranges[2 * t + 1] - ranges[2 * t]);  // 31 for one entry, smaller for longer lists
  return k > 31 ? 31 : k;
}

__global__ __launch_bounds__(256) void k_order_count(const int32_t* __restrict__ ranges, int n_tiles,
                                                     int32_t* obin) {
  __shared__ int h[32];
  if (threadIdx.x < 32) h[threadIdx.x] = 0;
  __syncthreads();
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t < n_tiles) atomicAdd(&h[len_class(ranges, t)], 1);
  __syncthreads();
  if (threadIdx.x < 32 && h[threadIdx.x] > 0) atomicAdd(&obin[threadIdx.x], h[threadIdx.x]);
}

__global__ void k_order_scan(int32_t* obin) {
  const int l = threadIdx.x;
  const int v = l < 32 ? obin[l] : 0;
  int incl = v;
#pragma unroll
  for (int off = 1; off < 32; off <<= 1) {
    const int o = __shfl_up(incl, off);
    if (l >= off) incl += o;
  }
  if (l < 32) obin[32 + l] = incl - v;
}

__global__ __launch_bounds__(256) void k_order_scatter(const int32_t* __restrict__ ranges, int n_tiles,
                                                       int32_t* obin, int32_t* __restrict__ order) {
  __shared__ int h[32], base[32];
  if (threadIdx.x < 32) h[threadIdx.x] = 0;
  __syncthreads();
  const int t = blockIdx.x * 256 + threadIdx.x;
  int k = 0, r = 0;
  if (t < n_tiles) {
    k = len_class(ranges, t);
    r = atomicAdd(&h[k], 1);
  }
  __syncthreads();
  if (threadIdx.x < 32 && h[threadIdx.x] > 0) base[threadIdx.x] = atomicAdd(&obin[32 + threadIdx.x], h[threadIdx.x]);
  __syncthreads();
  if (t < n_tiles) order[base[k] + r] = t;
}

// Forward-state checkpoints of tile t: one per chunk boundary inside its list.
// The launch's log2 chunk length: the caller's (ck_arg >= 0), or chosen from
// the pair count.
__device__ inline int launch_chunk_log2(int ck_arg, const int32_t* counters, int quads, int n_cu) {
  return ck_arg >= 0 ? ck_arg : auto_chunk_log2(counters[NSPLAT_CNT_PAIRS], quads, n_cu);
}

__global__ void k_chunk_counts(const int32_t* __restrict__ ranges, int n_tiles, int ck_arg, const int32_t* counters,
                               int quads, int n_cu, int32_t* __restrict__ queue, uint32_t* __restrict__ ck) {
  const int ck_lg = launch_chunk_log2(ck_arg, counters, quads, n_cu);
  if (blockIdx.x == 0 && threadIdx.x == 0) queue[Q_CKLG] = ck_lg;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n_tiles; t += gridDim.x * blockDim.x) {
    const int n = n_chunks(ranges[2 * t + 1] - ranges[2 * t], ck_lg);
    ck[t] = n > 0 ? (uint32_t)(n - 1) : 0u;
  }
}

// Marks the scenes that hold a filled curve (SceneTab.fills), which the
// adjoint takes in 8 x 8 pixel blocks at 32 x 32 tiles.  One block.
__global__ void k_scene_fills(nsplat_curves cv, SceneTab* st, int n_scenes) {
  for (int s = threadIdx.x; s < n_scenes; s += blockDim.x) st[s].fills = 0;
  __syncthreads();
  for (int c = threadIdx.x; c < cv.n_curves; c += blockDim.x) {
    const int s = cv.scene[c];
    if ((cv.flags[c] & NSPLAT_FILLED) && s >= 0 && s < n_scenes) st[s].fills = 1;
  }
}

// Adjoint pixel blocks per chunk of tile t: `blocks` (adj_blocks), where 16
// stands for 16 on the tiles of scenes with fills and 4 on the others.
__device__ inline int tile_blocks(int blocks, const SceneTab* st, int n_scenes, int t) {
  if (blocks != 16) return blocks;
  return st[scene_of_tile(st, n_scenes, t)].fills ? 16 : 4;
}

// Adjoint work items of the tile at blend-order position i: quadrants x chunks.
// (quads, the forward's quadrants per tile, feeds the chunk rule; blocks is
// the adjoint's pixel blocks per chunk, see tile_blocks)
__global__ void k_item_counts(const int32_t* __restrict__ ranges, const int32_t* __restrict__ order, int n_tiles,
                              int quads, int blocks, const SceneTab* st, int n_scenes, int ck_arg,
                              const int32_t* counters, int n_cu, uint32_t* __restrict__ items) {
  const int ck_lg = launch_chunk_log2(ck_arg, counters, quads, n_cu);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_tiles; i += gridDim.x * blockDim.x) {
    const int t = order[i];
    const int nb = tile_blocks(blocks, st, n_scenes, t);
    items[i] = (uint32_t)(nb * n_chunks(ranges[2 * t + 1] - ranges[2 * t], ck_lg));
  }
}

// The three steps above for up to SMALL_TILES tiles in one block (larger
// counts go through the multi-block kernels, which are faster there): the tile
// order by length class, then the checkpoint offsets (tile order) and the
// adjoint item offsets (blend order) as exclusive scans with their totals at
// index n_tiles, four entries per thread per round.
constexpr int PLAN_THREADS = 1024;
constexpr int SMALL_TILES = 8192;

__device__ inline uint32_t plan_wave_scan(uint32_t v) {
  const int lane = __lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(v, off);
    if (lane >= off) v += o;
  }
  return v;
}

// With `hist` (the scanned digit counts of a one-pass sort, `sb` blocks per
// digit, `nd` digits) it first writes every tile's range: tile t is digit t,
// its slice starts at the digit's first offset and ends where digit t + 1
// starts (or at the pair count); empty tiles get [0, 0).
__global__ __launch_bounds__(PLAN_THREADS) void k_tile_plan(int32_t* __restrict__ ranges, int n_tiles, int quads,
                                                            int blocks, const SceneTab* st, int n_scenes,
                                                            int ck_arg, int n_cu, int32_t* __restrict__ queue,
                                                            int32_t* __restrict__ order, int32_t* __restrict__ ck_off,
                                                            int32_t* __restrict__ item_off,
                                                            const uint32_t* __restrict__ hist, int sb, int nd,
                                                            const int32_t* counters, int empty_on_cap) {
  __shared__ int h[32], base[32];
  __shared__ uint32_t wsum[2][PLAN_THREADS / 64];
  const int tid = threadIdx.x, lane = __lane_id(), wid = tid >> 6;
  const int ck_lg = launch_chunk_log2(ck_arg, counters, quads, n_cu);
  if (tid == 0) queue[Q_CKLG] = ck_lg;
  if (hist) {
    const uint32_t total = (uint32_t)counters[NSPLAT_CNT_PAIRS];
    // (empty_on_cap: the one-digit binning writes no pairs on an overflow)
    const bool none = empty_on_cap && (counters[NSPLAT_CNT_STATUS] & NSPLAT_STATUS_PAIR_CAP);
    for (int t = tid; t < n_tiles; t += PLAN_THREADS) {
      const uint32_t s0 = hist[(int64_t)t * sb];
      const uint32_t s1 = t + 1 < nd ? hist[(int64_t)(t + 1) * sb] : total;
      const bool any = !none && s1 > s0;
      ranges[2 * t] = any ? (int32_t)s0 : 0;
      ranges[2 * t + 1] = any ? (int32_t)s1 : 0;
    }
    __syncthreads();
  }
  if (tid < 32) h[tid] = 0;
  __syncthreads();
  for (int t = tid; t < n_tiles; t += PLAN_THREADS) atomicAdd(&h[len_class(ranges, t)], 1);
  __syncthreads();
  if (tid < 64) {
    const int v = tid < 32 ? h[tid] : 0;
    int incl = v;
#pragma unroll
    for (int off = 1; off < 32; off <<= 1) {
      const int o = __shfl_up(incl, off);
      if (lane >= off) incl += o;
    }
    if (tid < 32) {
      base[tid] = incl - v;
      h[tid] = 0;
    }
  }
  __syncthreads();
  for (int t = tid; t < n_tiles; t += PLAN_THREADS) {
    const int k = len_class(ranges, t);
    order[base[k] + atomicAdd(&h[k], 1)] = t;
  }
  __syncthreads();
  uint32_t carry[2] = {0u, 0u};
  for (int b0 = 0; b0 < n_tiles; b0 += 4 * PLAN_THREADS) {
    const int i0 = b0 + 4 * tid;
    uint32_t v[2][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = i0 + j;
      uint32_t ck = 0u, it = 0u;
      if (i < n_tiles) {
        const int n = n_chunks(ranges[2 * i + 1] - ranges[2 * i], ck_lg);
        ck = n > 0 ? (uint32_t)(n - 1) : 0u;
        const int t = order[i];
        const int nb = tile_blocks(blocks, st, n_scenes, t);
        it = (uint32_t)(nb * n_chunks(ranges[2 * t + 1] - ranges[2 * t], ck_lg));
      }
      v[0][j] = ck;
      v[1][j] = it;
    }
    uint32_t incl[2], sum[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      sum[a] = (v[a][0] + v[a][1]) + (v[a][2] + v[a][3]);
      incl[a] = plan_wave_scan(sum[a]);
      if (lane == 63) wsum[a][wid] = incl[a];
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      uint32_t wb = 0, tot = 0;
#pragma unroll
      for (int q = 0; q < PLAN_THREADS / 64; ++q) {
        if (q < wid) wb += wsum[a][q];
        tot += wsum[a][q];
      }
      uint32_t run = carry[a] + wb + incl[a] - sum[a];
      int32_t* out = a == 0 ? ck_off : item_off;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (i0 + j < n_tiles) {
          out[i0 + j] = (int32_t)run;
          run += v[a][j];
        }
      carry[a] += tot;
    }
    __syncthreads();
  }
  if (tid == 0) {
    ck_off[n_tiles] = (int32_t)carry[0];
    item_off[n_tiles] = (int32_t)carry[1];
  }
}

}  // namespace

hipError_t launch_bin(const Launch& L) {
  const int64_t gcap = L.bf->caps.gauss, pcap = L.bf->caps.pairs;
  int32_t* cnt = L.bf->counters;
  const Gauss* gs = (const Gauss*)L.bf->gauss;
  const int gg = grid_for(gcap, 256, 8192);
  // number of key bits and radix passes (up to RADIX_BITS_MAX bits each)
  int key_bits = 0;
  while (key_bits < 31 && ((int64_t)1 << key_bits) < L.n_tiles) ++key_bits;
  const int passes = (key_bits + RADIX_BITS_MAX - 1) / RADIX_BITS_MAX;
  const int digit = passes ? (key_bits + passes - 1) / passes : 0;
  uint32_t* idx = (uint32_t*)L.bf->idx;
  // the last pass must land in (keys0, idx)
  uint32_t* ek = (passes % 2) ? L.w.keys1 : L.w.keys0;
  uint32_t* ev = (passes % 2) ? L.w.vals1 : idx;
  hipError_t e;
  const int sb = (int)((pcap + SORT_ITEMS - 1) / SORT_ITEMS);
  uint32_t *kin = ek, *vin = ev;  // input of the next radix pass
  int first = 0;                  // first radix pass still to run
  // The placement at once pays where a block's 4096 Gaussians carry few
  // pairs each and there are enough blocks to fill the GPU; a few Gaussians
  // with large tile rectangles (wide strokes, tangent-aligned ones) keep the
  // emission and radix passes, which spread their pairs over more wavefronts.
  const bool fused = passes >= 1 && gcap >= 65536 && pcap <= 8 * gcap;
  if (adj_blocks_of(L) == 16)
    hipLaunchKernelGGL(k_scene_fills, dim3(1), dim3(256), 0, L.stream, *L.cv, L.w.scenes, (int)L.sc->n_scenes);
  if (fused) {
    // the low digit at once: count per block and digit, scan, place the
    // pairs (k_bin_tilehist); the other digits, if any, by radix passes
    const int nd = 1 << digit;
    const int nbk = (int)std::max<int64_t>((gcap + FB_ITEMS - 1) / FB_ITEMS, 1);
    const bool one = passes == 1;
    uint32_t* k0 = (ek == L.w.keys0) ? L.w.keys1 : L.w.keys0;
    uint32_t* v0 = (ev == idx) ? L.w.vals1 : idx;
    {
      Phase ph(L, NSPLAT_T_BIN);
      hipLaunchKernelGGL(k_bin_tilehist, dim3(nbk), dim3(FB_THREADS), 0, L.stream, *L.cv, *L.pr, L.w, gs, cnt, nd,
                         nbk, L.w.hist, L.bf->ranges, one ? (int64_t)0 : 2 * L.n_tiles);
      e = launch_scan(L.w.hist, nullptr, (int64_t)(nd + 1) * nbk, nullptr, L.w.scan_tmp, L.stream);
      if (e != hipSuccess) return e;
    }
    {
      Phase ph(L, NSPLAT_T_SORT);
      hipLaunchKernelGGL(k_bin_place, dim3(nbk), dim3(FB_THREADS), 0, L.stream, *L.cv, *L.pr, L.w, gs, cnt, nd, nbk,
                         digit, (const uint32_t*)L.w.hist, one ? nullptr : k0, v0, pcap);
    }
    if (one) {
      Phase ph(L, NSPLAT_T_RANGES);
      hipLaunchKernelGGL(k_tile_plan, dim3(1), dim3(PLAN_THREADS), 0, L.stream, L.bf->ranges, (int)L.n_tiles,
                         L.pr->tile == 8 ? 1 : 4, adj_blocks_of(L), L.w.scenes, (int)L.sc->n_scenes, L.ck_lg,
                         L.n_cu, L.w.queue, L.w.order, L.w.ck_off, L.w.item_off,
                         (const uint32_t*)L.w.hist, nbk, nd, cnt, 1);
      return hipGetLastError();
    }
    kin = k0;
    vin = v0;
    first = 1;
  } else {
    Phase ph(L, NSPLAT_T_BIN);
    hipLaunchKernelGGL(k_bin_count, dim3(gg), dim3(256), 0, L.stream, *L.cv, *L.pr, L.w, gs, cnt, L.w.gcnt,
                       L.bf->ranges, 2 * L.n_tiles);
    e = launch_scan(L.w.gcnt, cnt + NSPLAT_CNT_GAUSS, gcap, L.w.gcnt + gcap, L.w.scan_tmp, L.stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_emit, dim3(gg), dim3(256), 0, L.stream, *L.cv, *L.pr, L.w, gs, cnt, L.w.gcnt,
                       L.w.gcnt + gcap, ek, ev, pcap);
  }
  {
    Phase ph(L, NSPLAT_T_SORT);
    for (int p = first; p < passes; ++p) {
      const int shift = p * digit;
      const int bits = (key_bits - shift) < digit ? (key_bits - shift) : digit;
      uint32_t* kout = (kin == L.w.keys0) ? L.w.keys1 : L.w.keys0;
      uint32_t* vout = (vin == idx) ? L.w.vals1 : idx;
      if (sb > 0) {
        hipLaunchKernelGGL(k_radix_hist, dim3(sb), dim3(SORT_THREADS), 0, L.stream, kin, cnt, shift, bits,
                           L.w.hist);
        e = launch_scan(L.w.hist, nullptr, (int64_t)(1 << bits) * sb, nullptr, L.w.scan_tmp, L.stream);
        if (e != hipSuccess) return e;
        if (bits > 8)
          hipLaunchKernelGGL(k_radix_scatter_wide, dim3(sb), dim3(SORT_THREADS), 0, L.stream, kin, vin, kout, vout,
                             cnt, shift, bits, L.w.hist);
        else
          hipLaunchKernelGGL(k_radix_scatter, dim3(sb), dim3(SORT_THREADS), 0, L.stream, kin, vin, kout, vout, cnt,
                             shift, bits, L.w.hist);
      }
      kin = kout;
      vin = vout;
    }
  }
  {
    Phase ph(L, NSPLAT_T_RANGES);
    const int nt = (int)L.n_tiles, ob = (nt + 255) / 256;
    // a one-pass radix sort's scanned digit counts are the tile ranges already
    const bool from_hist = !fused && passes == 1 && sb > 0 && nt > 0 && nt <= SMALL_TILES;
    if (!from_hist)
      hipLaunchKernelGGL(k_tile_ranges, dim3(grid_for(pcap, 256, 8192)), dim3(256), 0, L.stream, L.w.keys0, cnt,
                         L.bf->ranges);
    if (nt > 0 && nt <= SMALL_TILES) {
      hipLaunchKernelGGL(k_tile_plan, dim3(1), dim3(PLAN_THREADS), 0, L.stream, L.bf->ranges, nt,
                         L.pr->tile == 8 ? 1 : 4, adj_blocks_of(L), L.w.scenes, (int)L.sc->n_scenes, L.ck_lg,
                         L.n_cu, L.w.queue, L.w.order, L.w.ck_off, L.w.item_off,
                         from_hist ? (const uint32_t*)L.w.hist : nullptr, sb, 1 << key_bits, cnt, 0);
    } else if (nt > 0) {
      hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, L.stream, L.w.obin, 0, (int64_t)64);
      hipLaunchKernelGGL(k_order_count, dim3(ob), dim3(256), 0, L.stream, L.bf->ranges, nt, L.w.obin);
      hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(64), 0, L.stream, L.w.obin);
      hipLaunchKernelGGL(k_order_scatter, dim3(ob), dim3(256), 0, L.stream, L.bf->ranges, nt, L.w.obin, L.w.order);
      const int cb = grid_for(nt, 256, 4096);
      hipLaunchKernelGGL(k_chunk_counts, dim3(cb), dim3(256), 0, L.stream, L.bf->ranges, nt, L.ck_lg, cnt,
                         L.pr->tile == 8 ? 1 : 4, L.n_cu, L.w.queue, (uint32_t*)L.w.ck_off);
      e = launch_scan((uint32_t*)L.w.ck_off, nullptr, nt, (uint32_t*)L.w.ck_off + nt, L.w.scan_tmp, L.stream);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_item_counts, dim3(cb), dim3(256), 0, L.stream, L.bf->ranges, L.w.order, nt,
                         L.pr->tile == 8 ? 1 : 4, adj_blocks_of(L), L.w.scenes, (int)L.sc->n_scenes, L.ck_lg,
                         cnt, L.n_cu, (uint32_t*)L.w.item_off);
      e = launch_scan((uint32_t*)L.w.item_off, nullptr, nt, (uint32_t*)L.w.item_off + nt, L.w.scan_tmp, L.stream);
      if (e != hipSuccess) return e;
    } else {
      hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, L.stream, L.w.item_off, 0, (int64_t)1);
    }
  }
  return hipGetLastError();
}

}  // namespace nsp
