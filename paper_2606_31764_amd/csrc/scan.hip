// Device-wide exclusive prefix sums (one block for small arrays; else block
// sums, then the down-sweep, with the scan of the block sums done by a block
// of its own when there are many), fills, and the small helper kernels
// (grid-step annealing of Eq. 14, L2 loss gradient).
#include "nsplat_internal.h"

namespace nsp {

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_PER_THREAD = SCAN_ITEMS / SCAN_THREADS;  // 16

// Inclusive scan across a 64-wide wavefront.
__device__ inline uint32_t wave_incl_scan(uint32_t v) {
  const int lane = __lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(v, off);
    if (lane >= off) v += o;
  }
  return v;
}

// Exclusive scan across the block (blockDim.x = SCAN_THREADS); returns the
// block total in *total.
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* total) {
  __shared__ uint32_t wsum[SCAN_THREADS / 64];
  const int lane = __lane_id(), wid = threadIdx.x >> 6;
  const uint32_t incl = wave_incl_scan(v);
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < SCAN_THREADS / 64; ++i) {
    if (i < wid) base += wsum[i];
    tot += wsum[i];
  }
  __syncthreads();
  *total = tot;
  return base + incl - v;
}

__global__ void k_scan_reduce(const uint32_t* __restrict__ data, const int32_t* n_dev, int64_t n_cap,
                              uint32_t* __restrict__ tmp) {
  const int64_t n = n_dev ? (int64_t)min((int64_t)*n_dev, n_cap) : n_cap;
  const int64_t base = (int64_t)blockIdx.x * SCAN_ITEMS;
  uint32_t s = 0;
  for (int i = 0; i < SCAN_PER_THREAD; ++i) {
    const int64_t k = base + (int64_t)i * SCAN_THREADS + threadIdx.x;
    if (k < n) s += data[k];
  }
  uint32_t tot;
  block_excl_scan(s, &tot);
  if (threadIdx.x == 0) tmp[blockIdx.x] = tot;
}

__global__ void k_scan_top(uint32_t* tmp, int64_t nb, uint32_t* total_out) {
  // One block of SCAN_THREADS; each thread owns a contiguous run of entries.
  const int64_t per = (nb + SCAN_THREADS - 1) / SCAN_THREADS;
  const int64_t b0 = (int64_t)threadIdx.x * per;
  uint32_t s = 0;
  for (int64_t i = 0; i < per; ++i)
    if (b0 + i < nb) s += tmp[b0 + i];
  uint32_t tot;
  uint32_t run = block_excl_scan(s, &tot);
  for (int64_t i = 0; i < per; ++i)
    if (b0 + i < nb) {
      const uint32_t v = tmp[b0 + i];
      tmp[b0 + i] = run;
      run += v;
    }
  if (threadIdx.x == 0 && total_out) *total_out = tot;
}

__global__ void k_scan_down(uint32_t* __restrict__ data, const int32_t* n_dev, int64_t n_cap,
                            const uint32_t* __restrict__ tmp) {
  __shared__ uint32_t buf[SCAN_ITEMS];
  const int64_t n = n_dev ? (int64_t)min((int64_t)*n_dev, n_cap) : n_cap;
  const int64_t base = (int64_t)blockIdx.x * SCAN_ITEMS;
  if (base >= n) return;
  for (int i = 0; i < SCAN_PER_THREAD; ++i) {
    const int64_t k = base + (int64_t)i * SCAN_THREADS + threadIdx.x;
    buf[i * SCAN_THREADS + threadIdx.x] = k < n ? data[k] : 0u;
  }
  __syncthreads();
  uint32_t loc[SCAN_PER_THREAD];
  uint32_t s = 0;
  for (int i = 0; i < SCAN_PER_THREAD; ++i) {
    loc[i] = buf[threadIdx.x * SCAN_PER_THREAD + i];
    s += loc[i];
  }
  uint32_t tot;
  uint32_t run = block_excl_scan(s, &tot) + tmp[blockIdx.x];
  for (int i = 0; i < SCAN_PER_THREAD; ++i) {
    buf[threadIdx.x * SCAN_PER_THREAD + i] = run;
    run += loc[i];
  }
  __syncthreads();
  for (int i = 0; i < SCAN_PER_THREAD; ++i) {
    const int64_t k = base + (int64_t)i * SCAN_THREADS + threadIdx.x;
    if (k < n) data[k] = buf[i * SCAN_THREADS + threadIdx.x];
  }
}

// k_scan_down with the scan of the block sums folded in, for up to
// FUSED_BLOCKS blocks: each block adds up the sums of the blocks in front of
// it, and block 0 adds up all of them for the total.
constexpr int64_t FUSED_BLOCKS = 1024;

__global__ void k_scan_down_fused(uint32_t* __restrict__ data, const int32_t* n_dev, int64_t n_cap,
                                  const uint32_t* __restrict__ tmp, int64_t nb, uint32_t* total_out) {
  __shared__ uint32_t buf[SCAN_ITEMS];
  const int64_t n = n_dev ? (int64_t)min((int64_t)*n_dev, n_cap) : n_cap;
  const int64_t base = (int64_t)blockIdx.x * SCAN_ITEMS;
  const int64_t lim = blockIdx.x == 0 ? nb : (int64_t)blockIdx.x;
  uint32_t s = 0;
  for (int64_t i = threadIdx.x; i < lim; i += SCAN_THREADS) s += tmp[i];
  uint32_t front;
  block_excl_scan(s, &front);
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0 && total_out) *total_out = front;
    front = 0;
  }
  if (base >= n) return;
  for (int i = 0; i < SCAN_PER_THREAD; ++i) {
    const int64_t k = base + (int64_t)i * SCAN_THREADS + threadIdx.x;
    buf[i * SCAN_THREADS + threadIdx.x] = k < n ? data[k] : 0u;
  }
  __syncthreads();
  uint32_t loc[SCAN_PER_THREAD];
  uint32_t t = 0;
  for (int i = 0; i < SCAN_PER_THREAD; ++i) {
    loc[i] = buf[threadIdx.x * SCAN_PER_THREAD + i];
    t += loc[i];
  }
  uint32_t tot;
  uint32_t run = block_excl_scan(t, &tot) + front;
  for (int i = 0; i < SCAN_PER_THREAD; ++i) {
    buf[threadIdx.x * SCAN_PER_THREAD + i] = run;
    run += loc[i];
  }
  __syncthreads();
  for (int i = 0; i < SCAN_PER_THREAD; ++i) {
    const int64_t k = base + (int64_t)i * SCAN_THREADS + threadIdx.x;
    if (k < n) data[k] = buf[i * SCAN_THREADS + threadIdx.x];
  }
}

// Small scans (n <= SMALL_SCAN) in one launch: one block of 1024 threads
// walks the array in tiles of 4096 (four consecutive entries per thread),
// carrying the running total from tile to tile.
constexpr int SMALL_THREADS = 1024;
constexpr int64_t SMALL_SCAN = 65536;

__global__ __launch_bounds__(SMALL_THREADS) void k_scan_small(uint32_t* __restrict__ data, const int32_t* n_dev,
                                                              int64_t n_cap, uint32_t* total_out) {
  __shared__ uint32_t wsum[SMALL_THREADS / 64];
  const int64_t n = n_dev ? (int64_t)min((int64_t)*n_dev, n_cap) : n_cap;
  const int lane = __lane_id(), wid = threadIdx.x >> 6;
  uint32_t carry = 0;
  for (int64_t base = 0; base < n; base += 4 * SMALL_THREADS) {
    const int64_t k0 = base + 4 * (int64_t)threadIdx.x;
    uint32_t v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = k0 + i < n ? data[k0 + i] : 0u;
    const uint32_t s = (v[0] + v[1]) + (v[2] + v[3]);
    const uint32_t incl = wave_incl_scan(s);
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    uint32_t wbase = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < SMALL_THREADS / 64; ++i) {
      if (i < wid) wbase += wsum[i];
      tot += wsum[i];
    }
    __syncthreads();
    uint32_t run = carry + wbase + incl - s;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (k0 + i < n) {
        data[k0 + i] = run;
        run += v[i];
      }
    carry += tot;
  }
  if (threadIdx.x == 0 && total_out) *total_out = carry;
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Eq. 14, clamped outside (t_b, t_e).
__global__ void k_anneal(float* h_dev, int32_t* step_dev, int32_t step, int32_t total, float hmax, float hmin,
                         float tb, float te) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int32_t t = step_dev ? *step_dev : step;
  double phi = ((double)t / (double)total - (double)tb) / ((double)te - (double)tb);
  phi = phi < 0.0 ? 0.0 : (phi > 1.0 ? 1.0 : phi);
  const double h = (double)hmax + ((double)hmin - (double)hmax) * (1.0 + cos(M_PI * (1.0 - phi))) / 2.0;
  *h_dev = (float)h;
  if (step_dev) *step_dev = t + 1;
}

// One atomic per block: same-address float atomics serialise in L2, so the
// loss partials are reduced across the block first (and the grid is kept
// to a few hundred blocks, each thread taking many elements).  VEC: a, b and
// out are 16-byte aligned and read and written four floats at a time.
template <bool VEC>
__global__ __launch_bounds__(256) void k_l2(const float* __restrict__ a, const float* __restrict__ b,
                                            float* __restrict__ out, float* loss, int64_t n) {
  __shared__ float red[4];
  float s = 0.0f;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t n4 = 0;
  if (VEC) {
    n4 = n >> 2;
    const float4* a4 = (const float4*)a;
    const float4* b4 = (const float4*)b;
    float4* o4 = (float4*)out;
    for (int64_t i = i0; i < n4; i += stride) {
      const float4 x = a4[i], y = b4[i];
      const float d0 = x.x - y.x, d1 = x.y - y.y, d2 = x.z - y.z, d3 = x.w - y.w;
      o4[i] = make_float4(2.0f * d0, 2.0f * d1, 2.0f * d2, 2.0f * d3);
      s = __builtin_fmaf(d0, d0, s);
      s = __builtin_fmaf(d1, d1, s);
      s = __builtin_fmaf(d2, d2, s);
      s = __builtin_fmaf(d3, d3, s);
    }
  }
  for (int64_t i = 4 * n4 + i0; i < n; i += stride) {
    const float d = a[i] - b[i];
    out[i] = 2.0f * d;
    s = __builtin_fmaf(d, d, s);
  }
  if (loss) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    if (__lane_id() == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) unsafeAtomicAdd(loss, (red[0] + red[1]) + (red[2] + red[3]));
  }
}

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_scan(uint32_t* data, const int32_t* n_dev, int64_t n_cap, uint32_t* total_out, uint32_t* tmp,
                       hipStream_t s) {
  const int64_t nb = (n_cap + SCAN_ITEMS - 1) / SCAN_ITEMS;
  if (nb <= 0) return total_out ? launch_fill_u32(total_out, 0u, 1, s) : hipSuccess;
  if (n_cap <= SMALL_SCAN) {
    hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(SMALL_THREADS), 0, s, data, n_dev, n_cap, total_out);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, data, n_dev, n_cap, tmp);
  if (nb <= FUSED_BLOCKS) {
    hipLaunchKernelGGL(k_scan_down_fused, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, data, n_dev, n_cap, tmp, nb,
                       total_out);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_THREADS), 0, s, tmp, nb, total_out);
  hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, data, n_dev, n_cap, tmp);
  return hipGetLastError();
}

hipError_t launch_anneal(float* h_dev, int32_t* step_dev, int32_t step, int32_t total, float hmax, float hmin,
                         float tb, float te, hipStream_t s) {
  hipLaunchKernelGGL(k_anneal, dim3(1), dim3(64), 0, s, h_dev, step_dev, step, total, hmax, hmin, tb, te);
  return hipGetLastError();
}

hipError_t launch_l2(const float* a, const float* b, float* out, float* loss, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const bool vec = (((uintptr_t)a | (uintptr_t)b | (uintptr_t)out) & 15) == 0;
  if (vec)
    hipLaunchKernelGGL(k_l2<true>, dim3(grid_for((n + 15) / 16, 256, 512)), dim3(256), 0, s, a, b, out, loss, n);
  else
    hipLaunchKernelGGL(k_l2<false>, dim3(grid_for((n + 15) / 16, 256, 512)), dim3(256), 0, s, a, b, out, loss, n);
  return hipGetLastError();
}

}  // namespace nsp
