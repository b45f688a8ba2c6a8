// Second half of nsplat_backward: per-Gaussian adjoints -> curve parameters.
//
//   k_adj_stroke    one lane per stroke Gaussian: dL/d(mu, sigma) ->
//                   dL/d(x, y, s) of C(u_j) (sigma = s / rho, Eq. 5) -> reverse
//                   mode through the rational point (Eq. 1) and the Cox-de Boor
//                   triangle: control points, weights, widths, the 2p knots of
//                   the span, and dL/du_j -> the domain ends u_p, u_{m-p}
//                   (u_j is uniform in the domain).
//   k_adj_fill      one lane per fill Gaussian: dL/do_j -> curve opacity and,
//                   through the sigmoid and the SDF (Eq. 7, S1-S3, sign
//                   detached, nearest segment), the two end points of the
//                   nearest boundary segment.
//   (Colour gradients, and the opacity gradient of stroke curves, are
//   accumulated per curve by the compositing adjoint.)
//   k_adj_boundary  one lane per boundary point: the same point adjoint.
//   Both reduce within the wavefront by (curve, span) segment before the FP64
//   global atomics.
//   k_fold          one wavefront per curve: control points -> key points
//                   (the closed wrap), knots -> intervals (suffix sums of the
//                   cumulative sum) -> tau, FP32 outputs.
#include "nsplat_internal.h"

namespace nsp {

namespace {

constexpr int TRI = (MAXP + 1) * (MAXP + 2) / 2;

struct PtAdj {
  double cp[MAXP + 1][4];  // (x, y, w, s) of control points span-p..span
  double knot[2 * MAXP];   // slot k <-> knot index span - MAXP + 1 + k
  double ubar;
};

// Reverse-mode adjoint of the rational point (x, y, s) at u on `span` for the
// upstream gradient ab[3].
__device__ inline void point_adjoint(const nsplat_curves& cv, const CurveView& v, double u, int span,
                                     const double (&ab)[3], PtAdj& out) {
  const double* U = v.U;
  const int p = v.p;
  double tri[TRI];
  double N[MAXP + 1], left[MAXP + 1], right[MAXP + 1];
  N[0] = 1.0;
  tri[0] = 1.0;
#pragma unroll
  for (int d = 1; d <= MAXP; ++d) {
    if (d > p) break;
    left[d] = u - U[span + 1 - d];
    right[d] = U[span + d] - u;
    double saved = 0.0;
#pragma unroll
    for (int r = 0; r < d; ++r) {
      const double temp = N[r] / (right[r + 1] + left[d - r]);
      N[r] = saved + right[r + 1] * temp;
      saved = left[d - r] * temp;
    }
    N[d] = saved;
#pragma unroll
    for (int r = 0; r <= d; ++r) tri[d * (d + 1) / 2 + r] = N[r];
  }
  // C = S / W over the span's control points
  double P[MAXP + 1][3], wt[MAXP + 1];
  double S[3] = {0.0, 0.0, 0.0}, W = 0.0;
#pragma unroll
  for (int r = 0; r <= MAXP; ++r) {
    if (r > p) break;
    const int k = v.k0 + v.key_of_cp(span - p + r);
    wt[r] = (double)cv.key_w[k];
    P[r][0] = (double)cv.key_xy[2 * k];
    P[r][1] = (double)cv.key_xy[2 * k + 1];
    P[r][2] = (double)cv.key_s[k];
    const double nw = N[r] * wt[r];
    W += nw;
#pragma unroll
    for (int q = 0; q < 3; ++q) S[q] += nw * P[r][q];
  }
  const double invW = 1.0 / W;
  const double Cp[3] = {S[0] * invW, S[1] * invW, S[2] * invW};
  double Nb[MAXP + 1];
#pragma unroll
  for (int r = 0; r <= MAXP; ++r) {
    Nb[r] = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) out.cp[r][q] = 0.0;
    if (r > p) continue;
    const double gdot = ab[0] * (P[r][0] - Cp[0]) + ab[1] * (P[r][1] - Cp[1]) + ab[2] * (P[r][2] - Cp[2]);
    const double nwW = N[r] * wt[r] * invW;
    out.cp[r][0] = ab[0] * nwW;            // dC/dP = N w / W
    out.cp[r][1] = ab[1] * nwW;
    out.cp[r][2] = N[r] * gdot * invW;     // dC/dw = N (P - C) / W
    out.cp[r][3] = ab[2] * nwW;
    Nb[r] = wt[r] * gdot * invW;           // dC/dN = w (P - C) / W
  }
  // Reverse through N_{i,d} = (u - U_i)/(U_{i+d} - U_i) N_{i,d-1}
  //                          + (U_{i+d+1} - u)/(U_{i+d+1} - U_{i+1}) N_{i+1,d-1}
  double ub = 0.0;
#pragma unroll
  for (int k = 0; k < 2 * MAXP; ++k) out.knot[k] = 0.0;
#pragma unroll
  for (int d = MAXP; d >= 1; --d) {
    if (d > p) continue;
    double Np[MAXP + 1];
#pragma unroll
    for (int r = 0; r <= MAXP; ++r) Np[r] = 0.0;
#pragma unroll
    for (int r = 0; r <= d; ++r) {
      const double nb = Nb[r];
      const int i = span - d + r;
      if (r >= 1) {
        const double Ui = U[i], Uid = U[i + d];
        const double D = Uid - Ui;
        const double al = (u - Ui) / D;
        Np[r - 1] += nb * al;
        const double g = nb * tri[(d - 1) * d / 2 + r - 1];
        ub += g / D;
        out.knot[MAXP - 1 - d + r] -= g * (Uid - u) / (D * D);
        out.knot[MAXP - 1 + r] -= g * (u - Ui) / (D * D);
      }
      if (r <= d - 1) {
        const double Ui1 = U[i + 1], Uid1 = U[i + d + 1];
        const double D = Uid1 - Ui1;
        const double be = (Uid1 - u) / D;
        Np[r] += nb * be;
        const double g = nb * tri[(d - 1) * d / 2 + r];
        ub -= g / D;
        out.knot[MAXP + r] += g * (u - Ui1) / (D * D);
        out.knot[MAXP - d + r] += g * (Uid1 - u) / (D * D);
      }
    }
#pragma unroll
    for (int r = 0; r <= MAXP; ++r) Nb[r] = Np[r];
  }
  out.ubar = ub;
}

// Segmented suffix sum across the wavefront.  A run is a maximal group of
// adjacent lanes with equal keys (two runs may share a key); afterwards the
// first lane of each run holds the run total.  Each lane carries a flag that
// says whether its partial interval already reaches the end of its run.
template <int NV>
__device__ inline void seg_reduce(int64_t key, double (&v)[NV]) {
  const int lane = __lane_id();
  const int64_t next = __shfl_down(key, 1);
  bool f = (lane == 63) || (next != key);
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const bool fo = __shfl_down((int)f, off) != 0;
    const bool take = !f && (lane + off < 64);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const double o = __shfl_down(v[i], off);
      if (take) v[i] += o;
    }
    if (take) f = fo;
  }
}

__device__ inline bool seg_head(int64_t key) {
  const int lane = __lane_id();
  const int64_t prev = __shfl_up(key, 1);
  return key >= 0 && (lane == 0 || prev != key);
}

// Wave-cooperative accumulation of point adjoints into the FP64 control-point
// and knot buffers.  Every lane of the wavefront must call it.
__device__ inline void accumulate_points(const Work& w, int64_t key, int c, const CurveView& v, int span,
                                         PtAdj& pa, bool any) {
  if (!any) return;
  constexpr int NCP = 4 * (MAXP + 1);
  double buf[NCP + 2 * MAXP];
#pragma unroll
  for (int r = 0; r <= MAXP; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) buf[4 * r + q] = pa.cp[r][q];
#pragma unroll
  for (int k = 0; k < 2 * MAXP; ++k) buf[NCP + k] = pa.knot[k];
  seg_reduce(key, buf);
  if (seg_head(key)) {
    double* gcp = w.gcp + 4 * ((int64_t)v.k0 + (int64_t)c * CP_PAD);
    double* gk = w.gknot + (int64_t)v.t0 + (int64_t)c * KNOT_PAD;
#pragma unroll
    for (int r = 0; r <= MAXP; ++r) {
      if (r > v.p) break;
      const int j = span - v.p + r;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (buf[4 * r + q] != 0.0) unsafeAtomicAdd(gcp + 4 * j + q, buf[4 * r + q]);
    }
#pragma unroll
    for (int k = 0; k < 2 * MAXP; ++k) {
      if (k < MAXP - v.p || k > MAXP + v.p - 1) continue;
      if (buf[NCP + k] != 0.0) unsafeAtomicAdd(gk + span - MAXP + 1 + k, buf[NCP + k]);
    }
  }
}

// Curve-level sums (opacity, colour, domain ends), reduced by curve.
__device__ inline void accumulate_curve(const Work& w, int64_t key, int c, const CurveView& v, double (&cur)[6]) {
  seg_reduce(key, cur);
  if (seg_head(key)) {
    double* gc = w.gcurve + 4 * (int64_t)c;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (cur[i] != 0.0) unsafeAtomicAdd(gc + i, cur[i]);
    double* gk = w.gknot + (int64_t)v.t0 + (int64_t)c * KNOT_PAD;
    if (cur[4] != 0.0) unsafeAtomicAdd(gk + v.p, cur[4]);
    if (cur[5] != 0.0) unsafeAtomicAdd(gk + v.m - v.p, cur[5]);
  }
}

__device__ inline int curve_of(const int32_t* goff, int n, int64_t g) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (goff[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Stroke Gaussians: dL/d(mu, sigma) -> the curve point adjoint at u_j.
__global__ __launch_bounds__(256) void k_adj_stroke(nsplat_curves cv, nsplat_params pr, Work w,
                                                    const int32_t* plan, const int32_t* counters,
                                                    const Gauss* __restrict__ gs) {
  const int64_t G = counters[NSPLAT_CNT_GAUSS];
  const int lane = __lane_id();
  const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) - lane;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = wave0; base < G; base += stride) {
    const int64_t g = base + lane;
    int64_t kspan = -1 - lane, kcur = -1 - lane;
    double cur[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    PtAdj pa;
    int c = 0, span = 0;
    CurveView v;
    v.p = 0;
    bool stroke = false;
    if (g < G) {
      const Gauss r = gs[g];
      c = r.curve;
      if (!(cv.flags[c] & NSPLAT_FILLED)) {
        stroke = true;
        v = curve_view(cv, w.knots, c);
        const float* gg = w.ggrad + g * GG;
        const double ab[3] = {(double)gg[0], (double)gg[1], (double)gg[2] / (double)pr.rho};  // sigma = s / rho
        const int32_t* row = plan + (int64_t)P_STRIDE * c;
        const int M = row[P_NSAMP];
        int j = v.closed() ? r.local : r.local - pr.kappa;
        j = j < 0 ? 0 : (j > M - 1 ? M - 1 : j);
        double dt;
        const double u = sample_u(v.U[v.p], v.U[v.m - v.p], j, M, v.closed(), &dt);
        span = find_span(v.U, v.p, v.m, u);
        point_adjoint(cv, v, u, span, ab, pa);
        cur[4] = pa.ubar * (1.0 - dt);  // u_j = u_p + t_j (u_{m-p} - u_p)
        cur[5] = pa.ubar * dt;
        kspan = (int64_t)v.t0 + (int64_t)c * KNOT_PAD + span;
        kcur = c;
      }
    }
    if (!stroke) {
#pragma unroll
      for (int r = 0; r <= MAXP; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) pa.cp[r][q] = 0.0;
#pragma unroll
      for (int k = 0; k < 2 * MAXP; ++k) pa.knot[k] = 0.0;
    }
    const bool any = __ballot(stroke) != 0ull;
    accumulate_points(w, kspan, c, v, span, pa, any);
    if (any) accumulate_curve(w, kcur, c, v, cur);
  }
}

// Fill Gaussians: o_j = o sigmoid(z), z = gamma / h * sgn * d(q) with the
// nearest segment and the sign recorded at emission.  dL/do_j -> curve
// opacity, and dL/dd -> the segment's end points (d(d)/da = -(1 - t) n,
// d(d)/db = -t n at the projection, n the unit vector from it to q).
__global__ __launch_bounds__(256) void k_adj_fill(nsplat_curves cv, nsplat_params pr, Work w, const int32_t* plan,
                                                  const int32_t* counters, const Gauss* __restrict__ gs) {
  const int64_t G = counters[NSPLAT_CNT_GAUSS];
  const int lane = __lane_id();
  const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) - lane;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const double h = (double)read_h(pr);
  const double gh = (double)pr.gamma / h;
  for (int64_t base = wave0; base < G; base += stride) {
    const int64_t g = base + lane;
    int64_t kcur = -1 - lane;
    double cur[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int64_t skey = -1 - lane, sj = 0;  // boundary segment (start, end point) this lane's SDF gradient goes to
    double sv[4] = {0.0, 0.0, 0.0, 0.0};
    int c = 0;
    CurveView v;
    v.p = 0;
    bool fill = false;
    if (g < G) {
      const Gauss r = gs[g];
      c = r.curve;
      if (cv.flags[c] & NSPLAT_FILLED) {
        fill = true;
        kcur = c;
        v = curve_view(cv, w.knots, c);
        const double dO = (double)w.ggrad[g * GG + 3];
        const int32_t* row = plan + (int64_t)P_STRIDE * c;
        const int nx = row[P_NX];
        const int iy = r.local / nx, ix = r.local - iy * nx;
        const double qx = ((double)(row[P_IX0] + ix) + 0.5) * h;
        const double qy = ((double)(row[P_IY0] + iy) + 0.5) * h;
        const int nb = row[P_NSAMP];
        const int32_t ax = w.aux[g];
        const int ib = ax & 0x7fffffff;
        const double sgn = ax < 0 ? -1.0 : 1.0;
        const double2* bp = w.bpts + row[P_BOFF];
        const int jb = ib + 1 < nb ? ib + 1 : 0;
        const double2 A = bp[ib], Bq = bp[jb];
        const double ex = Bq.x - A.x, ey = Bq.y - A.y;
        const double ee = ex * ex + ey * ey;
        const double rx = qx - A.x, ry = qy - A.y;
        double t = 0.0;
        if (ee > 0.0) t = (rx * ex + ry * ey) / ee;
        t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
        const double px = A.x + t * ex - qx, py = A.y + t * ey - qy;
        const double d = sqrt(px * px + py * py);
        const double z = gh * (sgn * d);
        const double sz = 1.0 / (1.0 + exp(-z));
        cur[0] = dO * sz;
        const double ds = sz * (1.0 - sz);
        if (d > 0.0 && dO != 0.0 && ds > 1e-18) {
          const double dd = dO * (double)cv.opacity[c] * ds * gh * sgn;  // dL/dd
          const double nxv = -px / d, nyv = -py / d;
          skey = (int64_t)row[P_BOFF] + ib;
          sj = (int64_t)row[P_BOFF] + jb;
          sv[0] = -dd * (1.0 - t) * nxv;
          sv[1] = -dd * (1.0 - t) * nyv;
          sv[2] = -dd * t * nxv;
          sv[3] = -dd * t * nyv;
        }
      }
    }
    // lanes on the same boundary segment (neighbouring lattice points) are
    // summed in the wavefront before the FP64 atomics
    if (__ballot(skey >= 0) != 0ull) {
      seg_reduce(skey, sv);
      if (seg_head(skey)) {
        unsafeAtomicAdd(&w.gb[skey].x, sv[0]);
        unsafeAtomicAdd(&w.gb[skey].y, sv[1]);
        unsafeAtomicAdd(&w.gb[sj].x, sv[2]);
        unsafeAtomicAdd(&w.gb[sj].y, sv[3]);
      }
    }
    if (__ballot(fill) != 0ull) accumulate_curve(w, kcur, c, v, cur);
  }
}

__global__ __launch_bounds__(256) void k_adj_boundary(nsplat_curves cv, Work w, const int32_t* plan,
                                                      const int32_t* counters) {
  const int64_t NB = counters[NSPLAT_CNT_BOUND];
  const int lane = __lane_id();
  const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) - lane;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int n = cv.n_curves;
  for (int64_t base = wave0; base < NB; base += stride) {
    const int64_t b = base + lane;
    bool act = false;
    int64_t kspan = -1 - lane, kcur = -1 - lane;
    PtAdj pa;
#pragma unroll
    for (int r = 0; r <= MAXP; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) pa.cp[r][q] = 0.0;
#pragma unroll
    for (int k = 0; k < 2 * MAXP; ++k) pa.knot[k] = 0.0;
    pa.ubar = 0.0;
    double cur[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int c = 0, span = 0;
    CurveView v;
    v.p = 0;
    if (b < NB) {
      // curve: the last c with boff <= b
      int lo = 0, hi = n - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (plan[(int64_t)P_STRIDE * mid + P_BOFF] <= b) lo = mid;
        else hi = mid - 1;
      }
      c = lo;
      v = curve_view(cv, w.knots, c);
      const int32_t* row = plan + (int64_t)P_STRIDE * c;
      const int nb = row[P_NSAMP];
      const int j = (int)(b - row[P_BOFF]);
      const double2 adj = w.gb[b];
      if ((v.flags & NSPLAT_FILLED) && j >= 0 && j < nb && curve_valid(v) && (adj.x != 0.0 || adj.y != 0.0)) {
        act = true;
        const double ab[3] = {adj.x, adj.y, 0.0};
        double dt;
        const double u = sample_u(v.U[v.p], v.U[v.m - v.p], j, nb, true, &dt);
        span = find_span(v.U, v.p, v.m, u);
        point_adjoint(cv, v, u, span, ab, pa);
        cur[4] = pa.ubar * (1.0 - dt);
        cur[5] = pa.ubar * dt;
        kspan = (int64_t)v.t0 + (int64_t)c * KNOT_PAD + span;
        kcur = c;
      }
    }
    const bool any = __ballot(act) != 0ull;
    accumulate_points(w, kspan, c, v, span, pa, any);
    if (any) accumulate_curve(w, kcur, c, v, cur);
  }
}

// One thread per curve: fold the FP64 control-point and knot adjoints into
// the key-point and interval parametrisation and write FP32 gradients.
// One wavefront per curve: colour / opacity sums to FP32, control-point
// adjoints folded back onto key points (the closed wrap sends several control
// points to one key point), and the knot adjoints turned into interval
// adjoints: U_k = sum_{l<k} delta_l gives dL/d delta_l = sum_{k>l} dL/dU_k, a
// suffix sum taken 64 knots at a time from the top with a carried total.
__global__ __launch_bounds__(64) void k_fold(nsplat_curves cv, Work w, nsplat_grads gr) {
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  const CurveView v = curve_view(cv, w.knots, c);
  const int C = cv.channels;
  const double* gc = w.gcurve + 4 * (int64_t)c;
  if (lane == 0) gr.opacity[c] = (float)gc[0];
  if (lane < C) gr.color[(int64_t)c * C + lane] = (float)gc[1 + lane];
  const bool ok = curve_valid(v);
  const double* gcp = w.gcp + 4 * ((int64_t)v.k0 + (int64_t)c * CP_PAD);
  for (int k = lane; k < v.nk; k += 64) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (ok) {
      if (!v.closed()) {
        for (int q = 0; q < 4; ++q) acc[q] = gcp[4 * k + q];
      } else {
        // control points j with key_of_cp(j) == k: j = (k + ceil(p/2)) mod n_k, and that + n_k
        const int j0 = (k + (v.p + 1) / 2) % v.nk;
        for (int j = j0; j < v.ncp; j += v.nk)
          for (int q = 0; q < 4; ++q) acc[q] += gcp[4 * j + q];
      }
    }
    const int64_t kk = v.k0 + k;
    gr.key_xy[2 * kk] = (float)acc[0];
    gr.key_xy[2 * kk + 1] = (float)acc[1];
    gr.key_w[kk] = (float)acc[2];
    gr.key_s[kk] = (float)acc[3];
  }
  float* gt = gr.tau + v.t0;
  if (!ok) {
    for (int t = lane; t < v.nt; t += 64) gt[t] = 0.0f;
    return;
  }
  double* gk = w.gknot + (int64_t)v.t0 + (int64_t)c * KNOT_PAD;
  double carry = 0.0;  // sum of dL/dU_k above the current chunk
  for (int b = (v.m / 64) * 64; b >= 0; b -= 64) {
    const int l = b + lane;
    const double x = l <= v.m ? gk[l] : 0.0;
    double incl = x;  // sum over k >= l inside the chunk
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const double o = __shfl_down(incl, off);
      if (lane + off < 64) incl += o;
    }
    double excl = __shfl_down(incl, 1);  // sum over k > l inside the chunk
    if (lane == 63) excl = 0.0;
    const double total = __shfl(incl, 0);
    if (l < v.m) gk[l] = excl + carry;
    carry += total;
  }
  __syncthreads();
  if (!v.closed()) {
    for (int t = lane; t < v.nt; t += 64) gt[t] = (float)gk[v.p + t];
  } else {
    for (int t = lane; t < v.nt; t += 64) {
      double acc = 0.0;
      for (int l = t + v.p - v.nt; l < v.m; l += v.nt)
        if (l >= 0) acc += gk[l];
      gt[t] = (float)acc;
    }
  }
}

__global__ void k_zero_f64(double* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

__global__ void k_zero_dev(float* p, const int32_t* count, int64_t mult, int64_t cap) {
  int64_t n = (int64_t)*count;
  n = (n < cap ? n : cap) * mult;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

}  // namespace

hipError_t launch_zero_grads(const Launch& L) {
  Phase ph(L, NSPLAT_T_FOLD);
  const nsplat_curves& cv = *L.cv;
  const int64_t ncp = (int64_t)cv.n_keys + (int64_t)cv.n_curves * CP_PAD;
  const int64_t nkn = (int64_t)cv.n_taus + (int64_t)cv.n_curves * KNOT_PAD;
  hipLaunchKernelGGL(k_zero_dev, dim3(grid_for(L.bf->caps.gauss * GG, 256, 8192)), dim3(256), 0, L.stream,
                     L.w.ggrad, L.bf->counters + NSPLAT_CNT_GAUSS, (int64_t)GG, (int64_t)L.bf->caps.gauss);
  hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(4 * ncp, 256, 4096)), dim3(256), 0, L.stream, L.w.gcp, 4 * ncp);
  hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(nkn, 256, 4096)), dim3(256), 0, L.stream, L.w.gknot, nkn);
  hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(4 * cv.n_curves, 256, 4096)), dim3(256), 0, L.stream, L.w.gcurve,
                     (int64_t)4 * cv.n_curves);
  if (L.bf->caps.boundary > 0)
    hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(2 * L.bf->caps.boundary, 256, 4096)), dim3(256), 0, L.stream,
                       (double*)L.w.gb, 2 * L.bf->caps.boundary);
  return hipGetLastError();
}

hipError_t launch_adjoint(const Launch& L, const nsplat_grads* g) {
  {
    Phase ph(L, NSPLAT_T_ADJ_GAUSS);
    hipLaunchKernelGGL(k_adj_stroke, dim3(grid_for(L.bf->caps.gauss, 256, 8192)), dim3(256), 0, L.stream, *L.cv,
                       *L.pr, L.w, L.bf->plan, L.bf->counters, (const Gauss*)L.bf->gauss);
    hipLaunchKernelGGL(k_adj_fill, dim3(grid_for(L.bf->caps.gauss, 256, 8192)), dim3(256), 0, L.stream, *L.cv,
                       *L.pr, L.w, L.bf->plan, L.bf->counters, (const Gauss*)L.bf->gauss);
  }
  if (L.bf->caps.boundary > 0) {
    Phase ph(L, NSPLAT_T_ADJ_BOUND);
    hipLaunchKernelGGL(k_adj_boundary, dim3(grid_for(L.bf->caps.boundary, 256, 4096)), dim3(256), 0, L.stream,
                       *L.cv, L.w, L.bf->plan, L.bf->counters);
  }
  Phase ph(L, NSPLAT_T_FOLD);
  if (L.cv->n_curves > 0)
    hipLaunchKernelGGL(k_fold, dim3(L.cv->n_curves), dim3(64), 0, L.stream, *L.cv, L.w, *g);
  return hipGetLastError();
}

}  // namespace nsp
