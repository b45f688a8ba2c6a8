// nsplat_sample: NURBS curves -> isotropic Gaussians (Sec. 3.1-3.3).
//
//   k_scene_setup   per-scene tile / pixel offsets and N_L (Table S1)
//   k_curve_prep    one block per curve: knot vector (cumulative sum of the
//                   intervals, Sec. 3.1), arc length by N_L midpoints (Eq. 3,
//                   Eq. 2 for C'), contour count M = ceil(delta_c L) or
//                   boundary count N_b = ceil(delta_b L) (Sec. 3.2 / 3.3)
//   k_curve_scan    exclusive scans over curves (boundary offsets, Gaussian
//                   offsets), capacity checks
//   k_boundary      one block per filled curve: N_b boundary points in FP64,
//                   padded AABB, global lattice window (Sec. 3.3)
//   k_emit          one lane per Gaussian: span search and span-local
//                   Cox-de Boor evaluation (Eq. 4-5), or the fill lattice
//                   point with its SDF opacity (Eq. 6-7, S1-S3)
#include <mutex>

#include "nsplat_internal.h"
#include "span_wave.h"

namespace nsp {

namespace {

constexpr int PREP_THREADS = 256;  // k_boundary, and k_curve_prep for many curves
constexpr int PREP_KNOTS = 4096;  // knots held in LDS by k_curve_prep (32 KB)

__global__ void k_scene_setup(nsplat_scenes sc, nsplat_params pr, SceneTab* st, int32_t* clear_counters) {
  if (clear_counters && blockIdx.x == 0)
    for (int i = threadIdx.x; i < NSPLAT_NUM_COUNTERS; i += blockDim.x) clear_counters[i] = 0;
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int32_t toff = 0, poff = 0;
  for (int s = 0; s < sc.n_scenes; ++s) {
    SceneTab t;
    t.H = sc.hw[2 * s];
    t.W = sc.hw[2 * s + 1];
    t.tiles_x = (t.W + pr.tile - 1) / pr.tile;
    t.tiles_y = (t.H + pr.tile - 1) / pr.tile;
    t.tile_off = toff;
    t.pix_off = poff;
    t.n_L = (int32_t)llrint((double)pr.nl_factor * (double)(t.H > t.W ? t.H : t.W));
    t.fills = 0;
    st[s] = t;
    toff += t.tiles_x * t.tiles_y;
    poff += t.H * t.W;
  }
  SceneTab e = {};
  e.tile_off = toff;
  e.pix_off = poff;
  st[sc.n_scenes] = e;
}

template <int THREADS>
__device__ inline double block_sum(double v, double* red) {
  const int t = threadIdx.x;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < THREADS / 64; ++i) s += red[i];
  __syncthreads();
  return s;
}

// Count rule of Sec. 3.2 / 3.3: ceil(delta L), at least floor_min.  Sets
// *near when delta L lies within 1e-9 of an integer at or above the floor
// (another summation order of L could round the count to the other side).
__device__ inline int count_rule(double delta, double L, int floor_min, int* near) {
  const double x = delta * L;
  const double r = rint(x);
  if (fabs(x - r) < 1e-9 && r >= (double)floor_min) *near = 1;
  const double M = ceil(x);
  if (!(M >= (double)floor_min)) return floor_min;  // also catches NaN
  if (M > 2.0e9) return 2000000000;
  return (int)M;
}

// Whether the values of curve c lie in the domain of Sec. 3.1 (w_i > 0,
// tau_j >= 0 with at least one tau_j > 0, so that the parameter domain is not
// empty; a stroke's widths > 0; everything finite), decided by the whole
// block.  Every thread of the block must call it.
__device__ inline bool curve_values_ok(const nsplat_curves& cv, const CurveView& v, int c) {
  int bad = 0, pos = 0;
  for (int k = threadIdx.x; k < v.nk; k += blockDim.x) {
    const int64_t i = v.k0 + k;
    const float x = cv.key_xy[2 * i], y = cv.key_xy[2 * i + 1], wt = cv.key_w[i];
    if (!isfinite(x) || !isfinite(y) || !(wt > 0.0f) || !isfinite(wt)) bad = 1;
    if (!v.filled()) {
      const float sw = cv.key_s[i];
      if (!(sw > 0.0f) || !isfinite(sw)) bad = 1;
    }
  }
  for (int k = threadIdx.x; k < v.nt; k += blockDim.x) {
    const float t = cv.tau[v.t0 + k];
    if (!(t >= 0.0f) || !isfinite(t)) bad = 1;
    if (t > 0.0f) pos = 1;
  }
  if (threadIdx.x == 0) {
    if (!isfinite(cv.opacity[c])) bad = 1;
    for (int ch = 0; ch < cv.channels; ++ch)
      if (!isfinite(cv.color[(int64_t)c * cv.channels + ch])) bad = 1;
  }
  bad = __syncthreads_or(bad);
  pos = __syncthreads_or(pos);
  return !bad && pos;
}

// THREADS lanes per curve: 1024 when there are few curves, so that the N_L
// midpoints of a curve are spread over more wavefronts.
template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_curve_prep(nsplat_curves cv, nsplat_params pr, Work w, int32_t* plan,
                                                        int32_t* counters, int frozen, int n_scenes) {
  __shared__ double red[THREADS / 64];
  __shared__ double Us[PREP_KNOTS];
  const int c = blockIdx.x;
  const CurveView v = curve_view(cv, w.knots, c);
  int32_t* row = plan + (int64_t)P_STRIDE * c;
  const int s = cv.scene[c];
  if (!curve_valid(v) || s < 0 || s >= n_scenes) {
    if (threadIdx.x == 0) {
      row[P_COUNT] = 0;
      row[P_NSAMP] = 0;
      row[P_FLAGS] = NSPLAT_PLAN_INVALID;
      w.L[c] = 0.0;
      atomicOr(&counters[NSPLAT_CNT_STATUS], NSPLAT_STATUS_DATA);
    }
    return;
  }
  if (!curve_values_ok(cv, v, c)) {
    // no Gaussians, also under a frozen plan (the kernels downstream see a
    // curve with no samples and leave its gradients at zero)
    if (threadIdx.x == 0) {
      row[P_COUNT] = 0;
      row[P_NSAMP] = 0;
      row[P_NX] = row[P_NY] = 0;
      row[P_FLAGS] = NSPLAT_PLAN_INVALID;
      w.L[c] = 0.0;
      atomicOr(&counters[NSPLAT_CNT_STATUS], NSPLAT_STATUS_VALUE);
    }
    return;
  }
  // Knot vector: U_0 = 0, U_{l+1} = U_l + delta_l with the interval list of
  // Sec. 3.1 (open: p zeros, tau, p zeros; closed: last p tau, tau, first p).
  // The intervals are gathered in parallel into LDS, one thread sums them in
  // order (the same additions as a plain running sum), and the block writes
  // the knots out and evaluates the arc length from the LDS copy.
  double* U = w.knots + v.t0 + (int64_t)c * KNOT_PAD;
  auto interval = [&](int l) {
    if (!v.closed()) return (l < v.p || l >= v.p + v.nt) ? 0.0 : (double)cv.tau[v.t0 + l - v.p];
    int t = (l - v.p) % v.nt;
    if (t < 0) t += v.nt;
    return (double)cv.tau[v.t0 + t];
  };
  CurveView vk = v;  // the view the quadrature evaluates: knots in LDS when they fit
  if (v.m + 1 <= PREP_KNOTS) {
    for (int l = threadIdx.x; l < v.m; l += THREADS) Us[l + 1] = interval(l);
    __syncthreads();
    if (threadIdx.x == 0) {
      double acc = 0.0;
      Us[0] = 0.0;
      for (int l = 0; l < v.m; ++l) {
        acc = acc + Us[l + 1];
        Us[l + 1] = acc;
      }
    }
    __syncthreads();
    for (int l = threadIdx.x; l <= v.m; l += THREADS) U[l] = Us[l];
    vk.U = Us;
  } else {
    if (threadIdx.x == 0) {
      double acc = 0.0;
      U[0] = 0.0;
      for (int l = 0; l < v.m; ++l) {
        acc = acc + interval(l);
        U[l + 1] = acc;
      }
    }
    __syncthreads();
  }
  // Eq. 3: L = sum_j ||C'(u_j)|| du over N_L midpoints of [u_p, u_{m-p}].
  const SceneTab* st = w.scenes + s;
  const int n_L = st->n_L;
  const double a = vk.U[v.p], b = vk.U[v.m - v.p];
  const double du = (b - a) / (double)n_L;
  double part = 0.0;
  for (int j = 1 + threadIdx.x; j <= n_L; j += THREADS) {
    const double u = a + ((double)j - 0.5) * du;
    const int span = find_span(vk.U, v.p, v.m, u);
    double pt[3], d[3];
    curve_point(cv, vk, u, span, pt, d);
    part += sqrt(d[0] * d[0] + d[1] * d[1]) * du;
  }
  const double L = block_sum<THREADS>(part, red);
  if (threadIdx.x == 0) {
    w.L[c] = L;
    int near = 0;
    if (!v.filled()) {
      const double delta = (double)(v.aniso() ? pr.delta_a : pr.delta_c);
      const int M = count_rule(delta, L, v.closed() ? 3 : 2, &near);
      if (!frozen) {
        row[P_NSAMP] = M;
        row[P_COUNT] = v.closed() ? M : M + 2 * pr.kappa;
        row[P_IX0] = row[P_IY0] = row[P_NX] = row[P_NY] = 0;
      }
    } else {
      const int nb = count_rule((double)pr.delta_b, L, 3, &near);
      if (!frozen) row[P_NSAMP] = nb;
    }
    row[P_FLAGS] = near ? NSPLAT_PLAN_NEAR_INT : 0;
  }
}

// Exclusive scan over curves of one plan column into another (single block).
// which == 0: boundary points of filled curves -> P_BOFF, total to
// counters[BOUND_REQ]; which == 1: Gaussians -> P_GOFF and goff[], total to
// counters[GAUSS_REQ], capped total to counters[GAUSS], and the number of
// fill Gaussians, of other (stroke) Gaussians and of tangent-aligned stroke
// Gaussians to kinds[0], kinds[1], kinds[2].
__global__ __launch_bounds__(1024) void k_curve_scan(nsplat_curves cv, int32_t* plan, int32_t* goff,
                                                     int32_t* counters, int which, int64_t cap, int32_t* kinds) {
  __shared__ int64_t wsum[16];
  __shared__ int64_t fsum[16];
  __shared__ int64_t asum[16];
  const int n = cv.n_curves;
  const int per = (n + 1023) / 1024;
  const int c0 = threadIdx.x * per;
  int64_t s = 0, sf = 0, sa = 0;
  for (int i = 0; i < per; ++i) {
    const int c = c0 + i;
    if (c < n) {
      const int32_t* row = plan + (int64_t)P_STRIDE * c;
      if (which == 0) {
        s += ((cv.flags[c] & NSPLAT_FILLED) && row[P_NSAMP] > 0) ? row[P_NSAMP] : 0;
      } else {
        s += row[P_COUNT];
        if (cv.flags[c] & NSPLAT_FILLED) sf += row[P_COUNT];
        else if (cv.flags[c] & NSPLAT_ANISO) sa += row[P_COUNT];
      }
    }
  }
  if (which == 1) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      sf += __shfl_xor(sf, off);
      sa += __shfl_xor(sa, off);
    }
    if (__lane_id() == 0) {
      fsum[threadIdx.x >> 6] = sf;
      asum[threadIdx.x >> 6] = sa;
    }
  }
  // block exclusive scan of s
  int64_t incl = s;
  const int lane = __lane_id(), wid = threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t o = __shfl_up(incl, off);
    if (lane >= off) incl += o;
  }
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  int64_t base = 0, tot = 0;
  for (int i = 0; i < 16; ++i) {
    if (i < wid) base += wsum[i];
    tot += wsum[i];
  }
  int64_t run = base + incl - s;
  for (int i = 0; i < per; ++i) {
    const int c = c0 + i;
    if (c < n) {
      int32_t* row = plan + (int64_t)P_STRIDE * c;
      if (which == 0) {
        row[P_BOFF] = (int32_t)run;
        if ((cv.flags[c] & NSPLAT_FILLED) && row[P_NSAMP] > 0) run += row[P_NSAMP];
      } else {
        row[P_GOFF] = (int32_t)run;
        goff[c] = (int32_t)run;
        run += row[P_COUNT];
      }
    }
  }
  if (threadIdx.x == 0) {
    const int32_t t32 = tot > 0x7fffffff ? 0x7fffffff : (int32_t)tot;
    if (which == 0) {
      counters[NSPLAT_CNT_BOUND_REQ] = t32;
      counters[NSPLAT_CNT_BOUND] = (int32_t)(tot < cap ? tot : cap);
      if (tot > cap) atomicOr(&counters[NSPLAT_CNT_STATUS], NSPLAT_STATUS_BOUND_CAP);
    } else {
      goff[n] = t32;
      int64_t fills = 0, anis = 0;
      for (int i = 0; i < 16; ++i) {
        fills += fsum[i];
        anis += asum[i];
      }
      kinds[0] = fills > 0x7fffffff ? 0x7fffffff : (int32_t)fills;
      kinds[1] = tot - fills > 0x7fffffff ? 0x7fffffff : (int32_t)(tot - fills);
      kinds[2] = anis > 0x7fffffff ? 0x7fffffff : (int32_t)anis;
      counters[NSPLAT_CNT_GAUSS_REQ] = t32;
      counters[NSPLAT_CNT_GAUSS] = (int32_t)(tot < cap ? tot : cap);
      if (tot > cap) atomicOr(&counters[NSPLAT_CNT_STATUS], NSPLAT_STATUS_GAUSS_CAP);
    }
  }
}

// Boundary points b_j = C(u_j), u_j = u_p + j (u_{m-p} - u_p) / N_b, their
// padded AABB clipped to the canvas, and the lattice window
// i in [ceil(x0 / h - 1/2), floor(x1 / h - 1/2)] (same for rows).
// With own_offsets (up to PREP_THREADS * 4 curves) each block also takes the
// boundary offset of its curve (the sum of the boundary counts of the filled
// curves before it, as k_curve_scan with which = 0 gives it), and block 0
// publishes the boundary counters, so that scan need not run.
__global__ __launch_bounds__(PREP_THREADS) void k_boundary(nsplat_curves cv, nsplat_params pr, Work w,
                                                           int32_t* plan, int64_t cap, int frozen, int own_offsets,
                                                           int32_t* counters) {
  __shared__ double red[4][PREP_THREADS / 64];
  __shared__ int64_t psum[2][PREP_THREADS / 64];
  const int c = blockIdx.x;
  if (own_offsets) {
    int64_t before = 0, all = 0;
    for (int k = threadIdx.x; k < cv.n_curves; k += PREP_THREADS) {
      const int nbk = plan[(int64_t)P_STRIDE * k + P_NSAMP];
      const int64_t v = ((cv.flags[k] & NSPLAT_FILLED) && nbk > 0) ? nbk : 0;
      all += v;
      if (k < c) before += v;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      before += __shfl_xor(before, off);
      all += __shfl_xor(all, off);
    }
    if (__lane_id() == 0) {
      psum[0][threadIdx.x >> 6] = before;
      psum[1][threadIdx.x >> 6] = all;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t b = 0, t = 0;
      for (int q = 0; q < PREP_THREADS / 64; ++q) {
        b += psum[0][q];
        t += psum[1][q];
      }
      plan[(int64_t)P_STRIDE * c + P_BOFF] = (int32_t)b;
      if (c == 0) {
        counters[NSPLAT_CNT_BOUND_REQ] = t > 0x7fffffff ? 0x7fffffff : (int32_t)t;
        counters[NSPLAT_CNT_BOUND] = (int32_t)(t < cap ? t : cap);
        if (t > cap) atomicOr(&counters[NSPLAT_CNT_STATUS], NSPLAT_STATUS_BOUND_CAP);
      }
    }
    __syncthreads();
  }
  if (!(cv.flags[c] & NSPLAT_FILLED)) return;
  const CurveView v = curve_view(cv, w.knots, c);
  if (!curve_valid(v)) return;
  int32_t* row = plan + (int64_t)P_STRIDE * c;
  const int nb = row[P_NSAMP];
  const int64_t boff = row[P_BOFF];
  if (nb <= 0 || boff + nb > cap) {
    if (threadIdx.x == 0) row[P_COUNT] = 0;
    return;
  }
  const double a = v.U[v.p], b = v.U[v.m - v.p];
  double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
  for (int j = threadIdx.x; j < nb; j += PREP_THREADS) {
    const double u = sample_u(a, b, j, nb, true, nullptr);
    double pt[3];
    curve_point(cv, v, u, find_span(v.U, v.p, v.m, u), pt, nullptr);
    w.bpts[boff + j] = make_double2(pt[0], pt[1]);
    x0 = fmin(x0, pt[0]);
    x1 = fmax(x1, pt[0]);
    y0 = fmin(y0, pt[1]);
    y1 = fmax(y1, pt[1]);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    x0 = fmin(x0, __shfl_xor(x0, off));
    x1 = fmax(x1, __shfl_xor(x1, off));
    y0 = fmin(y0, __shfl_xor(y0, off));
    y1 = fmax(y1, __shfl_xor(y1, off));
  }
  // Bounding box of each chunk of SDF_CHUNK segments: points k*SDF_CHUNK up to
  // and including the chunk's end point (point 0 closes the last chunk).
  __syncthreads();
  {
    const int K = (nb + SDF_CHUNK - 1) / SDF_CHUNK;
    double4* box = w.cbox + cbox_base(boff, c) + 1;
    const double2* bp = w.bpts + boff;
    for (int k = threadIdx.x; k < K; k += PREP_THREADS) {
      const int i0 = k * SDF_CHUNK, i1 = i0 + SDF_CHUNK < nb ? i0 + SDF_CHUNK : nb;
      double2 e = bp[i1 < nb ? i1 : 0];
      double4 r = make_double4(e.x, e.x, e.y, e.y);
      for (int i = i0; i < i1; ++i) {
        e = bp[i];
        r.x = fmin(r.x, e.x);
        r.y = fmax(r.y, e.x);
        r.z = fmin(r.z, e.y);
        r.w = fmax(r.w, e.y);
      }
      box[k] = r;
    }
    // segment records, padded to whole chunks
    double* sg = w.segs + SEG_WORDS * seg_base(boff, c);
    for (int i = threadIdx.x; i < K * SDF_CHUNK; i += PREP_THREADS) {
      double* o = sg + SEG_WORDS * (int64_t)i;
      if (i < nb) {
        const double2 A = bp[i], B = bp[i + 1 < nb ? i + 1 : 0];
        const double ex = B.x - A.x, ey = B.y - A.y;
        const double ee = ex * ex + ey * ey;
        o[0] = A.x;
        o[1] = A.y;
        o[2] = ex;
        o[3] = ey;
        o[4] = ee > 0.0 ? 1.0 / ee : 0.0;
        o[5] = B.y;
      } else {
        o[0] = SEG_FAR;
        o[1] = SEG_FAR;
        o[2] = 0.0;
        o[3] = 0.0;
        o[4] = 0.0;
        o[5] = SEG_FAR;
      }
    }
  }
  const int t = threadIdx.x;
  if ((t & 63) == 0) {
    red[0][t >> 6] = x0;
    red[1][t >> 6] = x1;
    red[2][t >> 6] = y0;
    red[3][t >> 6] = y1;
  }
  __syncthreads();
  if (t != 0) return;
  for (int i = 1; i < PREP_THREADS / 64; ++i) {
    x0 = fmin(x0, red[0][i]);
    x1 = fmax(x1, red[1][i]);
    y0 = fmin(y0, red[2][i]);
    y1 = fmax(y1, red[3][i]);
  }
  x0 = fmin(x0, red[0][0]);
  x1 = fmax(x1, red[1][0]);
  y0 = fmin(y0, red[2][0]);
  y1 = fmax(y1, red[3][0]);
  w.cbox[cbox_base(boff, c)] = make_double4(x0, x1, y0, y1);
  if (!frozen) {
    const SceneTab* st = w.scenes + cv.scene[c];
    const double h = (double)read_h(pr), pad = (double)pr.fill_pad;
    const double px = pad * (x1 - x0), py = pad * (y1 - y0);
    const double bx0 = fmax(0.0, x0 - px), bx1 = fmin((double)st->W, x1 + px);
    const double by0 = fmax(0.0, y0 - py), by1 = fmin((double)st->H, y1 + py);
    const int ix0 = (int)ceil(bx0 / h - 0.5), ix1 = (int)floor(bx1 / h - 0.5);
    const int iy0 = (int)ceil(by0 / h - 0.5), iy1 = (int)floor(by1 / h - 0.5);
    const int nx = ix1 - ix0 + 1 > 0 ? ix1 - ix0 + 1 : 0;
    const int ny = iy1 - iy0 + 1 > 0 ? iy1 - iy0 + 1 : 0;
    row[P_IX0] = ix0;
    row[P_IY0] = iy0;
    row[P_NX] = nx;
    row[P_NY] = ny;
    row[P_COUNT] = nx * ny;
  }
}

// Signed distance of q to the closed polyline b[0..nb) (Suppl. S2): minimum
// distance over segments (projection clamped to [0, 1], lowest index wins a
// tie) and the sign of the exact integer winding number (crossing rule with
// orientation tests); inside <=> winding >= 1.  Returns the argmin segment
// and its projection parameter.
//
// The result is the one of the plain loop over all segments, computed with
// the same arithmetic on a subset of them.  Segments come in chunks of
// SDF_CHUNK with a bounding box each.  A chunk whose box is farther from q
// than an upper bound on the minimum (the nearest chunk start point, or the
// running minimum) cannot hold the argmin, with a relative margin of 1e-8
// that covers the rounding of both sides; skipping it changes neither the
// minimum nor the lowest index reaching it.  Its crossings are counted
// without visiting its segments when the box lies entirely above, below,
// left or right of q: a chain of segments right of q crosses the ray from q
// upward as many times, net, as its end point lies above q minus its start
// point does, and one left of q never crosses it.  The left/right decision
// keeps a margin that makes every orientation test in the chunk exact in
// sign, so the count equals the plain one.
// Element access for polyline_sdf: P is a pointer to double in the generic
// or the constant address space (points as (x, y) pairs, boxes as 4-tuples).
template <class P>
__device__ inline double2 ld_pt(P p, int i) {
  return make_double2(p[2 * i], p[2 * i + 1]);
}
template <class P>
__device__ inline double4 ld_box(P p, int i) {
  return make_double4(p[4 * i], p[4 * i + 1], p[4 * i + 2], p[4 * i + 3]);
}

// One chunk k of polyline_sdf for the point q: the lower bound of its box
// against thr = min(ub, best) decides whether its segments are visited;
// otherwise its crossings are counted in closed form where the box allows.
template <class P>
__device__ inline void sdf_chunk_box(int k, const double4& b, double qx, double qy, P bpd, P segd, int nb, double ub,
                                     double abs_margin, double mx, double* best, int* ibest, double* tbest, int* wn) {
  const double ex0 = fmax(fmax(b.x - qx, qx - b.y), 0.0);
  const double ey0 = fmax(fmax(b.z - qy, qy - b.w), 0.0);
  const double lb = ex0 * ex0 + ey0 * ey0;
  const double thr = fmin(ub, *best);
  bool visit = lb <= thr + 1e-8 * thr + abs_margin;
  const int i0 = k * SDF_CHUNK;
  const int i1 = i0 + SDF_CHUNK < nb ? i0 + SDF_CHUNK : nb;
  int wk = 0;
  if (!visit && b.z <= qy && qy < b.w) {
    if (b.x > qx + mx) {
      const double2 E = ld_pt(bpd, i1 < nb ? i1 : 0);
      wk = (E.y > qy ? 1 : 0) - (ld_pt(bpd, i0).y > qy ? 1 : 0);
    } else if (!(b.y < qx - mx)) {
      visit = true;
    }
  }
  if (visit) {
    // the chunk's SDF_CHUNK records (padding included), t = (r . e) / |e|^2
    // taken as a product with the stored reciprocal; two records per step keep
    // the scalar registers free enough for five wavefronts per SIMD unspilled
#pragma unroll 2
    for (int j = 0; j < SDF_CHUNK; ++j) {
      const int i = i0 + j;
      const int64_t o = (int64_t)SEG_WORDS * i;
      const double ax = segd[o], ay = segd[o + 1], ex = segd[o + 2], ey = segd[o + 3];
      const double inv = segd[o + 4], by = segd[o + 5];
      // fused forms: p - q = t e - r, one rounding each
      const double rx = qx - ax, ry = qy - ay;
      double t = __builtin_fma(rx, ex, ry * ey) * inv;
      t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
      const double px = __builtin_fma(t, ex, -rx), py = __builtin_fma(t, ey, -ry);
      const double d2 = __builtin_fma(px, px, py * py);
      const bool nearer = d2 < *best;
      *best = nearer ? d2 : *best;
      *ibest = nearer ? i : *ibest;
      *tbest = nearer ? t : *tbest;
      const double cr = __builtin_fma(ex, ry, -(rx * ey));  // > 0: q left of a -> b
      const bool below = ay <= qy;
      wk += (below && by > qy && cr > 0.0) ? 1 : 0;
      wk -= (!below && by <= qy && cr < 0.0) ? 1 : 0;
    }
  }
  *wn += wk;
}

// The same with the chunk's box (x0, x1, y0, y1) read here.
template <class P>
__device__ inline void sdf_chunk(int k, double qx, double qy, P bpd, P boxd, P segd, int nb, double ub,
                                 double abs_margin, double mx, double* best, int* ibest, double* tbest, int* wn) {
  sdf_chunk_box(k, ld_box(boxd, 1 + k), qx, qy, bpd, segd, nb, ub, abs_margin, mx, best, ibest, tbest, wn);
}

__device__ inline double sdf_scale(double ax, double ay, const double4& hb) {
  return 1.0 + ax + ay + 2.0 * fmax(fmax(fabs(hb.x), fabs(hb.y)), fmax(fabs(hb.z), fabs(hb.w)));
}

template <class P>
__device__ inline double polyline_sdf(double qx, double qy, P bpd, P boxd, P segd, int nb, int* arg, double* targ,
                                      double* sgn_out) {
  const int K = (nb + SDF_CHUNK - 1) / SDF_CHUNK;
  const double4 hb = ld_box(boxd, 0);  // the whole boundary's box
  const double scale = sdf_scale(fabs(qx), fabs(qy), hb);
  double ub = INFINITY;
  for (int k = 0; k < K; ++k) {
    const double2 V = ld_pt(bpd, k * SDF_CHUNK);
    const double dx = V.x - qx, dy = V.y - qy;
    ub = fmin(ub, dx * dx + dy * dy);
  }
  const double abs_margin = 1e-18 * scale * scale, mx = 1e-9 * scale;
  double best = INFINITY, tbest = 0.0;
  int ibest = 0, wn = 0;
  for (int k = 0; k < K; ++k) sdf_chunk(k, qx, qy, bpd, boxd, segd, nb, ub, abs_margin, mx, &best, &ibest, &tbest, &wn);
  *arg = ibest;
  *targ = tbest;
  *sgn_out = wn >= 1 ? 1.0 : -1.0;
  return sqrt(best);
}

// Lane l's value of v (wavefront-uniform).
__device__ inline double readlane_f64(double v, int l) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ inline double wave_min_f64(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off));
  return v;
}

// polyline_sdf for a full wavefront of points on one curve, inside the box
// [wx0, wx1] x [wy0, wy1] (lane values; the boundary arrays are read through
// the constant address space).  The chunk scan is shared: the wavefront's
// upper bound ubW is the least, over chunk starts V, of the distance from V
// to the farthest corner of the box, which bounds every lane's minimum; the
// lanes then classify one chunk each against the box.  A chunk that some
// lane would visit (its box within a lane's bound, or a lane's crossing test
// needing its segments) is in the visited list, because the box distance and
// ubW bound the lanes' own values and rounding is monotone; a chunk wholly
// right of the box with rows in the box's y-range adds its crossings in
// closed form; every other chunk adds nothing to any lane.  The visited
// chunks run sdf_chunk in order with ub = ubW, so each lane's result is that
// of polyline_sdf (and of the plain loop).
template <class P>
__device__ inline double polyline_sdf_wave(double qx, double qy, double wx0, double wx1, double wy0, double wy1,
                                           P bpd, P boxd, P segd, int nb, int* arg, double* targ, double* sgn_out) {
  const int K = (nb + SDF_CHUNK - 1) / SDF_CHUNK;
  const int lane = __lane_id();
  typedef const double* gdp;
  const gdp bpv = (gdp)bpd, boxv = (gdp)boxd;  // per-lane (vector) reads
  // the first 64 chunks' boxes are requested with their start points, so
  // that both arrive in one round trip
  double fb0 = 0.0, fb1 = 0.0, fb2 = 0.0, fb3 = 0.0;
  if (lane < K) {
    fb0 = boxv[4 * (1 + lane)];
    fb1 = boxv[4 * (1 + lane) + 1];
    fb2 = boxv[4 * (1 + lane) + 2];
    fb3 = boxv[4 * (1 + lane) + 3];
  }
  double u = INFINITY;
  for (int k = lane; k < K; k += 64) {
    const double vx = bpv[2 * k * SDF_CHUNK], vy = bpv[2 * k * SDF_CHUNK + 1];
    const double dx = fmax(fabs(vx - wx0), fabs(vx - wx1)), dy = fmax(fabs(vy - wy0), fabs(vy - wy1));
    u = fmin(u, dx * dx + dy * dy);
  }
  const double ubW = wave_min_f64(u);
  const double4 hb = ld_box(boxd, 0);
  const double scale = sdf_scale(fabs(qx), fabs(qy), hb);
  const double abs_margin = 1e-18 * scale * scale, mx = 1e-9 * scale;
  const double scaleW = sdf_scale(fmax(fabs(wx0), fabs(wx1)), fmax(fabs(wy0), fabs(wy1)), hb);
  const double amW = 1e-18 * scaleW * scaleW, mxW = 1e-9 * scaleW;
  double best = INFINITY, tbest = 0.0;
  int ibest = 0, wn = 0;
  for (int k0 = 0; k0 < K; k0 += 64) {
    const int k = k0 + lane;
    bool full = false, endp = false;
    double b0 = fb0, b1 = fb1, b2 = fb2, b3 = fb3;  // chunk k's box: x0, x1, y0, y1
    if (k < K) {
      if (k0 > 0) {
        b0 = boxv[4 * (1 + k)];
        b1 = boxv[4 * (1 + k) + 1];
        b2 = boxv[4 * (1 + k) + 2];
        b3 = boxv[4 * (1 + k) + 3];
      }
      const double ex0 = fmax(fmax(b0 - wx1, wx0 - b1), 0.0);
      const double ey0 = fmax(fmax(b2 - wy1, wy0 - b3), 0.0);
      const bool cand = ex0 * ex0 + ey0 * ey0 <= ubW + 1e-8 * ubW + amW;
      const bool yov = b2 <= wy1 && wy0 < b3;
      const bool right = b0 > wx1 + mxW, left = b1 < wx0 - mxW;
      full = cand || (yov && !right && !left);
      endp = !full && yov && right;
    }
    const uint64_t fm = __ballot(full), em = __ballot(endp);
    uint64_t m = fm | em;
    while (m) {
      const int bit = __builtin_ctzll(m);
      m &= m - 1;
      const int kk = k0 + bit;
      // the chunk's box from the lane that classified it
      const double4 b = make_double4(readlane_f64(b0, bit), readlane_f64(b1, bit), readlane_f64(b2, bit),
                                     readlane_f64(b3, bit));
      if ((fm >> bit) & 1ull) {
        sdf_chunk_box(kk, b, qx, qy, bpd, segd, nb, ubW, abs_margin, mx, &best, &ibest, &tbest, &wn);
      } else {
        if (b.z <= qy && qy < b.w) {
          const int i0 = kk * SDF_CHUNK, i1 = i0 + SDF_CHUNK < nb ? i0 + SDF_CHUNK : nb;
          const double2 E = ld_pt(bpd, i1 < nb ? i1 : 0);
          wn += (E.y > qy ? 1 : 0) - (ld_pt(bpd, i0).y > qy ? 1 : 0);
        }
      }
    }
  }
  *arg = ibest;
  *targ = tbest;
  *sgn_out = wn >= 1 ? 1.0 : -1.0;
  return sqrt(best);
}

// (colour channels of curve c, zero-padded to three; `tag` in w): the
// compositing kernels read it by Gaussian index, beside the record.
__device__ inline float4 curve_colour(const nsplat_curves& cv, int c, float tag) {
  const float* col = cv.color + (int64_t)c * cv.channels;
  return make_float4(col[0], cv.channels == 3 ? col[1] : 0.0f, cv.channels == 3 ? col[2] : 0.0f, tag);
}

// Stroke samples of a wavefront whose 64 lanes all lie on one curve: the
// wavefront finds the span window of its samples with a 64-ary search (one
// knot per lane per round, so two rounds cover 4096 knots instead of a
// binary search of a dozen dependent loads per lane), stages the window's
// knots and control points in LDS, and each lane finds its span and
// evaluates its sample there.  WIN spans at most per window.
constexpr int WIN = 64;
struct StrokeStage {
  double U[WIN + 2 * MAXP];   // knots s_lo - p + 1 .. s_hi + p
  float cp[WIN + MAXP][4];    // control points s_lo - p .. s_hi: x, y, w, width
};

// Sample point (and derivative) of this lane's u; false (nothing computed)
// when the wavefront's samples span more than WIN knot spans.  The result is
// curve_point at find_span(u): the span is the largest in [s_lo, s_hi] with
// U[span] <= u (s_lo, s_hi the spans of the wavefront's lowest and highest u,
// find_span being monotone), and the arithmetic is curve_point's.
__device__ bool stroke_point_wave(const nsplat_curves& cv, const CurveView& v, double u, StrokeStage* st,
                                  double (&pt)[3], double* d) {
  double umin = u, umax = u;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    umin = fmin(umin, __shfl_xor(umin, off));
    umax = fmax(umax, __shfl_xor(umax, off));
  }
  const int s_lo = __builtin_amdgcn_readfirstlane(span_uniform(v.U, v.p, v.m, umin));
  const int s_hi = __builtin_amdgcn_readfirstlane(span_uniform(v.U, v.p, v.m, umax));
  const int W = s_hi - s_lo + 1;
  if (W > WIN) return false;
  const int p = v.p, lane = __lane_id();
  const int kb = s_lo - p + 1, cb = s_lo - p;  // first staged knot and control point
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (int t = lane; t < W + 2 * p; t += 64) st->U[t] = v.U[kb + t];
  for (int t = lane; t < W + p; t += 64) {
    const int k = v.k0 + v.key_of_cp(cb + t);
    st->cp[t][0] = cv.key_xy[2 * k];
    st->cp[t][1] = cv.key_xy[2 * k + 1];
    st->cp[t][2] = cv.key_w[k];
    st->cp[t][3] = cv.key_s[k];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // the lane's span, relative to the first staged knot (span s sits at s - kb)
  int a = s_lo - kb, b = s_hi - kb;  // U[a] <= u unless u is left of the domain
  while (a < b) {
    const int mid = (a + b + 1) >> 1;
    if (st->U[mid] <= u) a = mid;
    else b = mid - 1;
  }
  const int span = a;  // in the staged knots' numbering
  double N[MAXP + 1], dN[MAXP + 1];
  basis_funs(st->U, span, p, u, N, d ? dN : nullptr);
  double S[3] = {0.0, 0.0, 0.0}, Sd[3] = {0.0, 0.0, 0.0}, Wt = 0.0, Wd = 0.0;
#pragma unroll
  for (int r = 0; r <= MAXP; ++r) {
    if (r > p) break;
    const float* c = st->cp[span + kb - p + r - cb];
    const double w = (double)c[2];
    const double P[3] = {(double)c[0], (double)c[1], (double)c[3]};
    const double nw = N[r] * w;
    Wt += nw;
#pragma unroll
    for (int q = 0; q < 3; ++q) S[q] += nw * P[q];
    if (d) {
      const double dnw = dN[r] * w;
      Wd += dnw;
#pragma unroll
      for (int q = 0; q < 3; ++q) Sd[q] += dnw * P[q];
    }
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) pt[q] = S[q] / Wt;
  if (d) {
#pragma unroll
    for (int q = 0; q < 3; ++q) d[q] = (Wt * Sd[q] - S[q] * Wd) / (Wt * Wt);
  }
  return true;
}

// One lane per Gaussian.  Emission order per curve: open strokes kappa copies
// of sample 0, samples 0..M-1, kappa copies of sample M-1; closed strokes
// samples 0..M-1; fills the lattice window row by row.  FILLS: the batch
// declares fills (nsplat_curves.any_flags).  Batches without them take their
// stroke samples through the wavefront-staged evaluation (stroke_point_wave);
// with the fill path in the same kernel that evaluation's registers would
// spill, so batches with fills evaluate every sample on its own.
template <bool FILLS>
__global__ __launch_bounds__(256, 5) void k_emit(nsplat_curves cv, nsplat_params pr, Work w, const int32_t* plan,
                                              const int32_t* counters, Gauss* __restrict__ out) {
  const int64_t G = counters[NSPLAT_CNT_GAUSS];
  const bool capped = (int64_t)counters[NSPLAT_CNT_GAUSS_REQ] > G;
  const int n = cv.n_curves;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < G; g += (int64_t)gridDim.x * blockDim.x) {
    const int c = curve_of_wave(w.goff, n, g);  // the last c with goff[c] <= g
    const CurveView v = curve_view(cv, w.knots, c);
    const int32_t* row = plan + (int64_t)P_STRIDE * c;
    const int local = (int)(g - w.goff[c]);
    Gauss r;
    r.curve = c;
    r.local = local;
    const double o = (double)cv.opacity[c];
    if (!(FILLS && v.filled())) {  // (a batch without fills has no Gaussian of a filled curve)
      const int M = row[P_NSAMP];
      int j = v.closed() ? local : local - pr.kappa;
      j = j < 0 ? 0 : (j > M - 1 ? M - 1 : j);
      const double u = sample_u(v.U[v.p], v.U[v.m - v.p], j, M, v.closed(), nullptr);
      double pt[3], d[3];
      const bool an = v.aniso();
      bool staged = false;
      if constexpr (!FILLS) {
        __shared__ StrokeStage stage[4];  // one per wavefront of the 256-thread block
        const int cu = __builtin_amdgcn_readfirstlane(c);
        staged = __ballot(c != cu) == 0ull && __ballot(true) == ~0ull &&
                 stroke_point_wave(cv, v, u, &stage[threadIdx.x >> 6], pt, an ? d : nullptr);
      }
      if constexpr (FILLS) {
        // the span only: one cooperative search when all 64 lanes sample one curve
        const int cu = __builtin_amdgcn_readfirstlane(c);
        const bool uni = __ballot(c != cu) == 0ull && __ballot(true) == ~0ull;
        curve_point(cv, v, u, uni ? span_wave(v.U, v.p, v.m, u) : find_span(v.U, v.p, v.m, u), pt,
                    an ? d : nullptr);
      } else if (!staged) {
        curve_point(cv, v, u, find_span(v.U, v.p, v.m, u), pt, an ? d : nullptr);
      }
      r.mx = pt[0];
      r.my = pt[1];
      const double sg = pt[2] / (double)pr.rho;
      r.sigma = (float)sg;  // Eq. 5
      r.opacity = (float)o;
      if (an) {
        // tangent-aligned: the axis across the curve keeps s / rho, the axis
        // along t = C' / |C'| (Eq. 2) covers the spacing |C'| du of the
        // samples with the same ratio rho, and never falls below the other
        const double len = sqrt(d[0] * d[0] + d[1] * d[1]);
        const double du = (v.U[v.m - v.p] - v.U[v.p]) / (double)(v.closed() ? M : M - 1);
        float tx = 1.0f, ty = 0.0f;
        double sig = sg;
        if (len > 0.0) {
          tx = (float)(d[0] / len);
          ty = (float)(d[1] / len);
          const double along = len * du / (double)pr.rho;
          if (along > sg) sig = along;
        }
        r.sigma = (float)sig;
        // the axis ratio sigma / sp is exactly 1 where the axes agree
        w.gaux[g] = make_float4(tx, ty, (float)sg, (float)(sig / sg));
      }
      out[g] = r;
      w.gcol[g] = curve_colour(cv, c, an ? KIND_ANISO : KIND_STROKE);
      continue;
    } else {
      // Lanes take the window in bands of 8 rows, column by column inside a
      // band, so that a wavefront covers an 8 x 8 block of lattice points
      // (nearby points visit the same boundary chunks); each point still
      // lands at its row-major place g = goff + iy nx + ix.  When the
      // Gaussian count was capped (capacity overflow), lanes keep their own
      // row-major point instead, so that every record below the cap is
      // written.
      const int nx = row[P_NX], ny = row[P_NY];
      int ix, iy;
      if (!capped) {
        const int band = local / (8 * nx);
        const int rows = min(8, ny - 8 * band);
        const int i = local - band * 8 * nx;
        ix = i / rows;
        iy = 8 * band + (i - ix * rows);
      } else {
        iy = local / nx;
        ix = local - iy * nx;
      }
      const int lin = iy * nx + ix;
      const int64_t gp = (int64_t)w.goff[c] + lin;
      r.local = lin;
      const double h = (double)read_h(pr);
      const double qx = ((double)(row[P_IX0] + ix) + 0.5) * h;
      const double qy = ((double)(row[P_IY0] + iy) + 0.5) * h;
      int arg;
      double t, sgn;
      double d;
      const int cu = __builtin_amdgcn_readfirstlane(c);
      if (__ballot(c != cu) == 0ull) {
        // the whole wavefront is on one curve: its boundary is read through
        // the constant address space with uniform indices (scalar loads)
        typedef const __attribute__((address_space(4))) double* cdp;
        const int32_t* ru = plan + (int64_t)P_STRIDE * cu;
        const cdp bp = (cdp)(w.bpts + ru[P_BOFF]), bx = (cdp)(w.cbox + cbox_base(ru[P_BOFF], cu)),
                  sg = (cdp)(w.segs + SEG_WORDS * seg_base(ru[P_BOFF], cu));
        if (!capped && __ballot(true) == ~0ull) {
          // all 64 lanes: the chunk scan is shared over the lattice box of
          // the wavefront (the same formula as qx, qy at the extreme indices)
          int ix0 = ix, ix1 = ix, iy0 = iy, iy1 = iy;
#pragma unroll
          for (int off = 32; off >= 1; off >>= 1) {
            ix0 = min(ix0, __shfl_xor(ix0, off));
            ix1 = max(ix1, __shfl_xor(ix1, off));
            iy0 = min(iy0, __shfl_xor(iy0, off));
            iy1 = max(iy1, __shfl_xor(iy1, off));
          }
          const double wx0 = ((double)(row[P_IX0] + ix0) + 0.5) * h, wx1 = ((double)(row[P_IX0] + ix1) + 0.5) * h;
          const double wy0 = ((double)(row[P_IY0] + iy0) + 0.5) * h, wy1 = ((double)(row[P_IY0] + iy1) + 0.5) * h;
          d = polyline_sdf_wave(qx, qy, wx0, wx1, wy0, wy1, bp, bx, sg, ru[P_NSAMP], &arg, &t, &sgn);
        } else {
          d = polyline_sdf(qx, qy, bp, bx, sg, ru[P_NSAMP], &arg, &t, &sgn);
        }
      } else {
        d = polyline_sdf(qx, qy, (const double*)(w.bpts + row[P_BOFF]),
                         (const double*)(w.cbox + cbox_base(row[P_BOFF], c)),
                         (const double*)(w.segs + SEG_WORDS * seg_base(row[P_BOFF], c)), row[P_NSAMP], &arg, &t,
                         &sgn);
      }
      const double z = ((double)pr.gamma / h) * (sgn * d);
      r.mx = qx;
      r.my = qy;
      r.sigma = (float)((double)pr.eta * h / (double)pr.rho);  // Eq. 6
      r.opacity = (float)(o * (1.0 / (1.0 + exp(-z))));        // Eq. 7
      if (gp < G) {  // a capped (overflowing) emission may map past the capacity
        w.aux[gp] = arg | (sgn < 0.0 ? (int32_t)0x80000000 : 0);
        w.gop[gp] = r.opacity;
        out[gp] = r;
        w.gcol[gp] = curve_colour(cv, c, KIND_FILL);
      }
      continue;
    }
  }
}

// Squared distance from q to the closed polyline b[0..nb) (with its chunk
// boxes), or `best` if that is smaller: chunks whose box lies farther than
// the running minimum (with a relative margin of 1e-12) are not visited.
__device__ inline double polyline_dist2(double qx, double qy, const double2* __restrict__ bp,
                                        const double4* __restrict__ box, int nb, double best) {
  const int K = (nb + SDF_CHUNK - 1) / SDF_CHUNK;
  for (int k = 0; k < K; ++k) {
    const double4 b = box[k];
    const double ex0 = fmax(fmax(b.x - qx, qx - b.y), 0.0);
    const double ey0 = fmax(fmax(b.z - qy, qy - b.w), 0.0);
    if (ex0 * ex0 + ey0 * ey0 > best * (1.0 + 1e-12)) continue;
    const int i0 = k * SDF_CHUNK;
    const int i1 = i0 + SDF_CHUNK < nb ? i0 + SDF_CHUNK : nb;
    double2 A = bp[i0];
    for (int i = i0; i < i1; ++i) {
      const double2 B = bp[i + 1 < nb ? i + 1 : 0];
      const double ex = B.x - A.x, ey = B.y - A.y;
      const double ee = ex * ex + ey * ey;
      const double rx = qx - A.x, ry = qy - A.y;
      double t = 0.0;
      if (ee > 0.0) t = (rx * ex + ry * ey) / ee;
      t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
      const double px = A.x + t * ex - qx, py = A.y + t * ey - qy;
      best = fmin(best, px * px + py * py);
      A = B;
    }
  }
  return best;
}

__global__ void k_fill_f64(double* p, double v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// The scene of global pixel index i: the last s with pix_off <= i.
__device__ inline int scene_of_pixel(const SceneTab* st, int n_scenes, int64_t i) {
  int lo = 0, hi = n_scenes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (st[mid].pix_off <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Distance-weighted loss, pass 1: per pixel q, d(q) = distance to the nearest
// boundary segment of the scene's selected filled curves, w(q) =
// max(0, tau - d(q)) stored in the first channel plane of dL, and the per-scene
// sums of w.
__global__ __launch_bounds__(256) void k_udf_weight(nsplat_curves cv, Work w, const int32_t* plan, int64_t bcap,
                                                    int n_scenes, int C, const int32_t* sel, float tau,
                                                    float* __restrict__ dL) {
  const int64_t npix = w.scenes[n_scenes].pix_off;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x + threadIdx.x - __lane_id(); base < npix;
       base += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = base + __lane_id();
    int s = -1;
    double wq = 0.0;
    if (i < npix) {
      s = scene_of_pixel(w.scenes, n_scenes, i);
      const SceneTab st = w.scenes[s];
      const int64_t li = i - st.pix_off;
      const int y = (int)(li / st.W), x = (int)(li - (int64_t)y * st.W);
      const double qx = x + 0.5, qy = y + 0.5;
      // curves of scene s: [c0, c1)
      int lo = 0, hi = cv.n_curves;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cv.scene[mid] < s) lo = mid + 1;
        else hi = mid;
      }
      const int c0 = lo;
      hi = cv.n_curves;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cv.scene[mid] <= s) lo = mid + 1;
        else hi = mid;
      }
      double best = INFINITY;
      for (int c = c0; c < lo; ++c) {
        if (!(cv.flags[c] & NSPLAT_FILLED) || (sel && !sel[c])) continue;
        const int32_t* row = plan + (int64_t)P_STRIDE * c;
        const int nb = row[P_NSAMP];
        const int64_t boff = row[P_BOFF];
        if (nb <= 0 || boff + nb > bcap || !curve_valid(curve_view(cv, w.knots, c))) continue;
        const double4* box = w.cbox + cbox_base(boff, c);
        const double4 hb = box[0];
        const double ex0 = fmax(fmax(hb.x - qx, qx - hb.y), 0.0);
        const double ey0 = fmax(fmax(hb.z - qy, qy - hb.w), 0.0);
        if (ex0 * ex0 + ey0 * ey0 > best * (1.0 + 1e-12)) continue;
        best = polyline_dist2(qx, qy, w.bpts + boff, box + 1, nb, best);
      }
      wq = fmax(0.0, (double)tau - sqrt(best));
      dL[st.pix_off * C + li] = (float)wq;
    }
    // per-scene sums: one atomic per wavefront when its pixels share a scene
    const int s0 = __builtin_amdgcn_readfirstlane(s);
    const bool same = __ballot(i < npix && s != s0) == 0ull;
    if (same) {
      double t = wq;
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off);
      if (__lane_id() == 0 && s0 >= 0 && t != 0.0) unsafeAtomicAdd(&w.sacc[s0], t);
    } else if (s >= 0 && wq != 0.0) {
      unsafeAtomicAdd(&w.sacc[s], wq);
    }
  }
}

// Pass 2: dL/dI_c(q) = 2 w(q) / W_s (I_c - I*_c) / C with W_s the scene's sum
// of w (0 when it is 0), and the loss sum_q w / W_s (1/C) sum_c (I_c - I*_c)^2.
__global__ __launch_bounds__(256) void k_udf_grad(Work w, int n_scenes, int C, const float* __restrict__ image,
                                                  const float* __restrict__ target, float* __restrict__ dL,
                                                  float* loss) {
  __shared__ double red[4];
  const int64_t npix = w.scenes[n_scenes].pix_off;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npix; i += (int64_t)gridDim.x * blockDim.x) {
    const int s = scene_of_pixel(w.scenes, n_scenes, i);
    const SceneTab st = w.scenes[s];
    const int64_t li = i - st.pix_off, plane = (int64_t)st.H * st.W;
    const double sum = w.sacc[s];
    const double wn = sum > 0.0 ? (double)dL[st.pix_off * C + li] / sum : 0.0;
    for (int c = 0; c < C; ++c) {
      const int64_t k = st.pix_off * C + c * plane + li;
      const double e = (double)image[k] - (double)target[k];
      acc += wn * e * e / C;
      dL[k] = (float)(2.0 * wn * e / C);
    }
  }
  if (loss) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if (__lane_id() == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) unsafeAtomicAdd(loss, (float)((red[0] + red[1]) + (red[2] + red[3])));
  }
}

}  // namespace

hipError_t launch_udf(const Launch& L, const int32_t* sel, float tau, const float* image, const float* target,
                      float* dL, float* loss, double* sacc) {
  const int S = L.sc->n_scenes, C = L.cv->channels;
  int64_t npix = 0;
  for (int s = 0; s < S; ++s) npix += (int64_t)L.sc->hw_host[2 * s] * L.sc->hw_host[2 * s + 1];
  Work w = L.w;
  if (sacc) w.sacc = sacc;  // per-scene weight sums somewhere else than the workspace
  hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(256), 0, L.stream, w.sacc, 0.0, (int64_t)(S + 1));
  if (npix <= 0) return hipGetLastError();
  hipLaunchKernelGGL(k_udf_weight, dim3(grid_for(npix, 256, 8192)), dim3(256), 0, L.stream, *L.cv, w,
                     L.bf->plan, (int64_t)L.bf->caps.boundary, S, C, sel, tau, dL);
  hipLaunchKernelGGL(k_udf_grad, dim3(grid_for(npix, 256, 2048)), dim3(256), 0, L.stream, w, S, C, image, target,
                     dL, loss);
  return hipGetLastError();
}

// Device scratch of nsplat_udf_loss_noalloc: the per-scene weight sums live
// in this file-scope array instead of the caller's workspace, so that entry
// point needs no memory of its own.  Each device holds its own copy for the
// life of the process; host code must use the address udf_scratch_setup took
// with hipGetSymbolAddress on that device, never the array's name (which on
// the host only stands in for the symbol).
static __device__ __align__(256) double scratch[UDF_SCRATCH_SLOTS];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t udf_scratch_setup(int device) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

double* udf_scratch(int device) {
  if (device < 0 || device >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (double*)g_scratch_ptr[device];
}

hipError_t launch_scene_setup(const Launch& L, int32_t* clear_counters) {
  hipLaunchKernelGGL(k_scene_setup, dim3(1), dim3(64), 0, L.stream, *L.sc, *L.pr, L.w.scenes, clear_counters);
  return hipGetLastError();
}

hipError_t launch_sample(const Launch& L, int frozen) {
  const int n = L.cv->n_curves;
  int32_t* plan = L.bf->plan;
  int32_t* cnt = L.bf->counters;
  {
  Phase ph(L, NSPLAT_T_PLAN);
  if (n < 1024)
    hipLaunchKernelGGL(k_curve_prep<1024>, dim3(n), dim3(1024), 0, L.stream, *L.cv, *L.pr, L.w, plan, cnt, frozen,
                       L.sc->n_scenes);
  else
    hipLaunchKernelGGL(k_curve_prep<PREP_THREADS>, dim3(n), dim3(PREP_THREADS), 0, L.stream, *L.cv, *L.pr, L.w, plan,
                       cnt, frozen, L.sc->n_scenes);
  // up to 1024 curves the boundary blocks take their own offsets
  const int own = n <= 4 * PREP_THREADS;
  if (!own)
    hipLaunchKernelGGL(k_curve_scan, dim3(1), dim3(1024), 0, L.stream, *L.cv, plan, L.w.goff, cnt, 0,
                       (int64_t)L.bf->caps.boundary, L.w.queue + Q_NFILL);
  hipLaunchKernelGGL(k_boundary, dim3(n), dim3(PREP_THREADS), 0, L.stream, *L.cv, *L.pr, L.w, plan,
                     (int64_t)L.bf->caps.boundary, frozen, own, cnt);
  hipLaunchKernelGGL(k_curve_scan, dim3(1), dim3(1024), 0, L.stream, *L.cv, plan, L.w.goff, cnt, 1,
                     (int64_t)L.bf->caps.gauss, L.w.queue + Q_NFILL);
  }
  Phase ph(L, NSPLAT_T_EMIT);
  if (L.cv->any_flags & NSPLAT_FILLED)
    hipLaunchKernelGGL(k_emit<true>, dim3(grid_for(L.bf->caps.gauss, 256, 8192)), dim3(256), 0, L.stream, *L.cv,
                       *L.pr, L.w, plan, cnt, (Gauss*)L.bf->gauss);
  else
    hipLaunchKernelGGL(k_emit<false>, dim3(grid_for(L.bf->caps.gauss, 256, 8192)), dim3(256), 0, L.stream, *L.cv,
                       *L.pr, L.w, plan, cnt, (Gauss*)L.bf->gauss);
  return hipGetLastError();
}

}  // namespace nsp
