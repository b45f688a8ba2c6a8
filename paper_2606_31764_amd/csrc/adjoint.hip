// Second half of nsplat_backward: per-Gaussian adjoints -> curve parameters.
//
//   k_adj_stroke    one lane per stroke Gaussian: dL/d(mu, sigma) ->
//                   dL/d(x, y, s) of C(u_j) (sigma = s / rho, Eq. 5) -> reverse
//                   mode through the rational point (Eq. 1) and the Cox-de Boor
//                   triangle: control points, weights, widths, the 2p knots of
//                   the span, and dL/du_j -> the domain ends u_p, u_{m-p}
//                   (u_j is uniform in the domain).
//   k_adj_aniso     one lane per tangent-aligned stroke Gaussian: the same,
//                   plus dL/d(sp, theta) and the spacing term of sigma through
//                   the first derivative C'(u_j) and the domain ends.
//   k_adj_fill      one lane per fill Gaussian: dL/do_j -> curve opacity and,
//                   through the sigmoid and the SDF (Eq. 7, S1-S3, sign
//                   detached, nearest segment), the two end points of the
//                   nearest boundary segment.
//   (Colour gradients, and the opacity gradient of stroke curves, are
//   accumulated per curve by the compositing adjoint.)
//   k_adj_boundary  one lane per boundary point: the same point adjoint.
//   Both reduce within the wavefront by (curve, span) segment before the FP64
//   global atomics.
//   k_reg_stroke,   the geometric regularisers of Sec. 3.5 at stroke samples
//   k_reg_boundary  and fill boundary points: bounding-box penalty (Eq. 12)
//                   into the centre / boundary-point adjoints, derivative
//                   loss (Eq. 11) by reverse mode straight to the curve.
//   k_fold          one wavefront per curve: control points -> key points
//                   (the closed wrap), knots -> intervals (suffix sums of the
//                   cumulative sum) -> tau, FP32 outputs.
#include "nsplat_internal.h"

namespace nsp {

namespace {

// The point and derivative adjoints below hold basis functions and control
// points in register arrays sized for degree PD, the batch's degree bound (3,
// or NSPLAT_MAX_DEGREE): smaller arrays for the usual quadratic and cubic
// curves keep more wavefronts resident.
constexpr int tri_n(int d) { return (d + 1) * (d + 2) / 2; }

template <int PD>
struct PtAdj {
  double cp[PD + 1][4];  // (x, y, w, s) of control points span-p..span
  double knot[2 * PD];   // slot k <-> knot index span - PD + 1 + k
  double ubar;
};

// Reverse-mode adjoint of the rational point (x, y, s) at u on `span` for the
// upstream gradient ab[3].
template <int PD>
__device__ inline void point_adjoint(const nsplat_curves& cv, const CurveView& v, double u, int span,
                                     const double (&ab)[3], PtAdj<PD>& out) {
  const double* U = v.U;
  const int p = v.p;
  double tri[tri_n(PD)];
  double N[PD + 1], left[PD + 1], right[PD + 1];
  N[0] = 1.0;
  tri[0] = 1.0;
#pragma unroll
  for (int d = 1; d <= PD; ++d) {
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
  double P[PD + 1][3], wt[PD + 1];
  double S[3] = {0.0, 0.0, 0.0}, W = 0.0;
#pragma unroll
  for (int r = 0; r <= PD; ++r) {
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
  double Nb[PD + 1];
#pragma unroll
  for (int r = 0; r <= PD; ++r) {
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
  for (int k = 0; k < 2 * PD; ++k) out.knot[k] = 0.0;
#pragma unroll
  for (int d = PD; d >= 1; --d) {
    if (d > p) continue;
    double Np[PD + 1];
#pragma unroll
    for (int r = 0; r <= PD; ++r) Np[r] = 0.0;
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
        out.knot[PD - 1 - d + r] -= g * (Uid - u) / (D * D);
        out.knot[PD - 1 + r] -= g * (u - Ui) / (D * D);
      }
      if (r <= d - 1) {
        const double Ui1 = U[i + 1], Uid1 = U[i + d + 1];
        const double D = Uid1 - Ui1;
        const double be = (Uid1 - u) / D;
        Np[r] += nb * be;
        const double g = nb * tri[(d - 1) * d / 2 + r];
        ub -= g / D;
        out.knot[PD + r] += g * (u - Ui1) / (D * D);
        out.knot[PD - d + r] += g * (Uid1 - u) / (D * D);
      }
    }
#pragma unroll
    for (int r = 0; r <= PD; ++r) Nb[r] = Np[r];
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
template <int PD>
__device__ inline void accumulate_points(const Work& w, int64_t key, int c, const CurveView& v, int span,
                                         PtAdj<PD>& pa, bool any) {
  if (!any) return;
  constexpr int NCP = 4 * (PD + 1);
  double buf[NCP + 2 * PD];
#pragma unroll
  for (int r = 0; r <= PD; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) buf[4 * r + q] = pa.cp[r][q];
#pragma unroll
  for (int k = 0; k < 2 * PD; ++k) buf[NCP + k] = pa.knot[k];
  seg_reduce(key, buf);
  if (seg_head(key)) {
    double* gcp = w.gcp + 4 * ((int64_t)v.k0 + (int64_t)c * CP_PAD);
    double* gk = w.gknot + (int64_t)v.t0 + (int64_t)c * KNOT_PAD;
#pragma unroll
    for (int r = 0; r <= PD; ++r) {
      if (r > v.p) break;
      const int j = span - v.p + r;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (buf[4 * r + q] != 0.0) unsafeAtomicAdd(gcp + 4 * j + q, buf[4 * r + q]);
    }
#pragma unroll
    for (int k = 0; k < 2 * PD; ++k) {
      if (k < PD - v.p || k > PD + v.p - 1) continue;
      if (buf[NCP + k] != 0.0) unsafeAtomicAdd(gk + span - PD + 1 + k, buf[NCP + k]);
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

// Stroke Gaussians: dL/d(mu, sigma) -> the curve point adjoint at u_j.
template <int PD>
__global__ __launch_bounds__(256) void k_adj_stroke(nsplat_curves cv, nsplat_params pr, Work w,
                                                    const int32_t* plan, const int32_t* counters,
                                                    const Gauss* __restrict__ gs) {
  if (w.queue[Q_NSTROKE] == 0) return;  // no Gaussians of this kind
  const int64_t G = counters[NSPLAT_CNT_GAUSS];
  const int lane = __lane_id();
  const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) - lane;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = wave0; base < G; base += stride) {
    const int64_t g = base + lane;
    int64_t kspan = -1 - lane, kcur = -1 - lane;
    double cur[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    PtAdj<PD> pa;
    int c = 0, span = 0;
    CurveView v;
    v.p = 0;
    bool stroke = false;
    if (g < G) {
      // curve and sample index from the emission offsets, as in k_adj_fill
      typedef const __attribute__((address_space(4))) Gauss* const_gauss;
      const int64_t g0 = first_lane_i64(g);
      c = curve_walk(w.goff, cv.n_curves, g, g0, ((const_gauss)gs)[g0].curve);
      if (!(cv.flags[c] & (NSPLAT_FILLED | NSPLAT_ANISO))) {
        stroke = true;
        const int local = (int)(g - w.goff[c]);
        v = curve_view(cv, w.knots, c);
        const float* gg = w.ggrad + g * GG;
        const double ab[3] = {(double)gg[0], (double)gg[1], (double)gg[2] / (double)pr.rho};  // sigma = s / rho
        const int32_t* row = plan + (int64_t)P_STRIDE * c;
        const int M = row[P_NSAMP];
        int j = v.closed() ? local : local - pr.kappa;
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
      for (int r = 0; r <= PD; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) pa.cp[r][q] = 0.0;
#pragma unroll
      for (int k = 0; k < 2 * PD; ++k) pa.knot[k] = 0.0;
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
  if (w.queue[Q_NFILL] == 0) return;  // no Gaussians of this kind
  const int64_t G = counters[NSPLAT_CNT_GAUSS];
  const int lane = __lane_id();
  const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) - lane;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const double h = (double)read_h(pr);
  const double gh = (double)pr.gamma / h;
  for (int64_t base = wave0; base < G; base += stride) {
    const int64_t g = base + lane;
    int64_t kcur = -1 - lane;
    double dop[1] = {0.0};  // dL/d(curve opacity): the only curve-level sum of a fill Gaussian
    int64_t skey = -1 - lane, sj = 0;  // boundary segment (start, end point) this lane's SDF gradient goes to
    double sv[4] = {0.0, 0.0, 0.0, 0.0};
    int c = 0;
    bool fill = false;
    if (g < G) {
      // the curve and lattice index of Gaussian g from the emission offsets
      // (the record holds the same two values), starting from the curve in
      // the record of the wavefront's first Gaussian (one scalar load)
      typedef const __attribute__((address_space(4))) Gauss* const_gauss;
      const int64_t g0 = first_lane_i64(g);
      c = curve_walk(w.goff, cv.n_curves, g, g0, ((const_gauss)gs)[g0].curve);
      if (cv.flags[c] & NSPLAT_FILLED) {
        fill = true;
        kcur = c;
        const int local = (int)(g - w.goff[c]);
        const double dO = (double)w.ggrad[g * GG + 3];
        const int32_t* row = plan + (int64_t)P_STRIDE * c;
        const int nx = row[P_NX];
        const int iy = local / nx, ix = local - iy * nx;
        const double qx = ((double)(row[P_IX0] + ix) + 0.5) * h;
        const double qy = ((double)(row[P_IY0] + iy) + 0.5) * h;
        const int nb = row[P_NSAMP];
        const int32_t xa = w.aux[g];
        const int ib = xa & 0x7fffffff;
        const double sgn = xa < 0 ? -1.0 : 1.0;
        // the nearest segment's record, with the arithmetic of the emission
        const double* sr = w.segs + SEG_WORDS * (seg_base(row[P_BOFF], c) + ib);
        const int jb = ib + 1 < nb ? ib + 1 : 0;
        const double ax = sr[0], ay = sr[1], ex = sr[2], ey = sr[3], inv = sr[4];
        const double rx = qx - ax, ry = qy - ay;
        double t = __builtin_fma(rx, ex, ry * ey) * inv;
        t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
        const double px = __builtin_fma(t, ex, -rx), py = __builtin_fma(t, ey, -ry);
        const double d = sqrt(__builtin_fma(px, px, py * py));
        const double z = gh * (sgn * d);
        const double sz = 1.0 / (1.0 + exp(-z));
        dop[0] = dO * sz;
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
    if (__ballot(fill) != 0ull) {
      const int64_t k0 = __builtin_amdgcn_readfirstlane((int)kcur);
      if (__ballot(kcur != k0) == 0ull) {  // one curve across the wavefront: a plain sum
        double s = dop[0];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0 && s != 0.0) unsafeAtomicAdd(w.gcurve + 4 * k0, s);
      } else {
        seg_reduce(kcur, dop);
        if (seg_head(kcur) && dop[0] != 0.0) unsafeAtomicAdd(w.gcurve + 4 * (int64_t)c, dop[0]);
      }
    }
  }
}

template <int PD>
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
    PtAdj<PD> pa;
#pragma unroll
    for (int r = 0; r <= PD; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) pa.cp[r][q] = 0.0;
#pragma unroll
    for (int k = 0; k < 2 * PD; ++k) pa.knot[k] = 0.0;
    pa.ubar = 0.0;
    double cur[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int c = 0, span = 0;
    CurveView v;
    v.p = 0;
    if (b < NB) {
      c = last_le_wave<P_STRIDE, P_BOFF>(plan, n, b);  // curve: the last c with boff <= b
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
  // a NULL output leaves that gradient group out
  if (lane == 0 && gr.opacity) gr.opacity[c] = (float)gc[0];
  if (lane < C && gr.color) gr.color[(int64_t)c * C + lane] = (float)gc[1 + lane];
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
    if (gr.key_xy) {
      gr.key_xy[2 * kk] = (float)acc[0];
      gr.key_xy[2 * kk + 1] = (float)acc[1];
    }
    if (gr.key_w) gr.key_w[kk] = (float)acc[2];
    if (gr.key_s) gr.key_s[kk] = (float)acc[3];
  }
  if (!gr.tau) return;
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

// Zeroes up to four FP64 arrays in one launch (index space n0 + n1 + n2 + n3).
struct ZeroSet {
  double* p[4];
  int64_t n[4];
};

// Clears the per-Gaussian adjoints (min(*count, cap) * mult floats at p) and
// the FP64 arrays of z, in one launch.
__global__ void k_zero_grads(float* p, const int32_t* count, int64_t mult, int64_t cap, ZeroSet z) {
  int64_t n = (int64_t)*count;
  n = (n < cap ? n : cap) * mult;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = i0; i < n; i += stride) p[i] = 0.0f;
  const int64_t total = z.n[0] + z.n[1] + z.n[2] + z.n[3];
  for (int64_t i = i0; i < total; i += stride) {
    int64_t j = i;
    int a = 0;
    while (a < 3 && j >= z.n[a]) j -= z.n[a++];
    z.p[a][j] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Geometric regularisers (Sec. 3.5): derivative loss (Eq. 11) and
// bounding-box loss (Eq. 12), at the parameters of each curve's own samples.
// ---------------------------------------------------------------------------

constexpr int MAXR = 3;  // highest derivative order of the derivative loss

// Value scale * ||C^(r)(u)||^2 of the planar curve at u on `span` and its
// reverse-mode adjoint.  Forward: the span's homogeneous control points
// H_j = (w x, w y, w); derivative control points
//   PK_k[j] = (p - k + 1) (PK_{k-1}[j+1] - PK_{k-1}[j]) / (U[span+j+1] - U[span-p+j+k])
// (every denominator spans the non-empty span, so none vanishes);
// S^(k)(u) = sum_j N_{span-p+k+j, p-k}(u) PK_k[j], the homogeneous k-th
// derivative; and the rational Leibniz rule
//   C^(k) = (A^(k) - sum_{i=1..k} binom(k, i) W^(i) C^(k-i)) / W, (A, W) = S.
// Reverse: the same steps backwards, with the adjoint of the degree p - k
// basis functions entering the Cox-de Boor triangle at its level p - k.  With
// `up` set, the reverse pass starts from the given adjoint up[0..1] of
// C^(r)(u) instead of that of the value (whose scale is then unused).
template <int PD>
__device__ inline double deriv_adjoint(const nsplat_curves& cv, const CurveView& v, double u, int span, int r,
                                       double scale, PtAdj<PD>& out, const double* up = nullptr) {
  const double* U = v.U;
  const int p = v.p;
  const int R = r < p ? r : p;
  double tri[tri_n(PD)];
  double N[PD + 1], left[PD + 1], right[PD + 1];
  N[0] = 1.0;
  tri[0] = 1.0;
#pragma unroll
  for (int d = 1; d <= PD; ++d) {
    if (d > p) break;
    left[d] = u - U[span + 1 - d];
    right[d] = U[span + d] - u;
    double saved = 0.0;
#pragma unroll
    for (int q = 0; q < d; ++q) {
      const double temp = N[q] / (right[q + 1] + left[d - q]);
      N[q] = saved + right[q + 1] * temp;
      saved = left[d - q] * temp;
    }
    N[d] = saved;
#pragma unroll
    for (int q = 0; q <= d; ++q) tri[d * (d + 1) / 2 + q] = N[q];
  }
  double X[PD + 1], Y[PD + 1], Wt[PD + 1];
  double PK[MAXR + 1][PD + 1][3];
#pragma unroll
  for (int j = 0; j <= PD; ++j) {
    X[j] = Y[j] = Wt[j] = 0.0;
    if (j > p) continue;
    const int k = v.k0 + v.key_of_cp(span - p + j);
    Wt[j] = (double)cv.key_w[k];
    X[j] = (double)cv.key_xy[2 * k];
    Y[j] = (double)cv.key_xy[2 * k + 1];
    PK[0][j][0] = Wt[j] * X[j];
    PK[0][j][1] = Wt[j] * Y[j];
    PK[0][j][2] = Wt[j];
  }
#pragma unroll
  for (int k = 1; k <= MAXR; ++k) {
    if (k > R) break;
#pragma unroll
    for (int j = 0; j < PD; ++j) {
      if (j > p - k) break;
      const double c = (double)(p - k + 1) / (U[span + j + 1] - U[span - p + j + k]);
#pragma unroll
      for (int q = 0; q < 3; ++q) PK[k][j][q] = c * (PK[k - 1][j + 1][q] - PK[k - 1][j][q]);
    }
  }
  // (register arrays are indexed with compile-time indices only: the degree
  // d = p - k is matched by an unrolled loop instead of computed)
  double S[MAXR + 1][3];
#pragma unroll
  for (int k = 0; k <= MAXR; ++k) {
    S[k][0] = S[k][1] = S[k][2] = 0.0;
    if (k > R) continue;
#pragma unroll
    for (int d = 0; d <= PD; ++d) {
      if (d != p - k) continue;
#pragma unroll
      for (int j = 0; j <= d; ++j) {
        const double n = tri[d * (d + 1) / 2 + j];
#pragma unroll
        for (int q = 0; q < 3; ++q) S[k][q] += n * PK[k][j][q];
      }
    }
  }
  const double binom[MAXR + 1][MAXR + 1] = {{1, 0, 0, 0}, {1, 1, 0, 0}, {1, 2, 1, 0}, {1, 3, 3, 1}};
  const double W0 = S[0][2];
  double Cx[MAXR + 1], Cy[MAXR + 1];
#pragma unroll
  for (int k = 0; k <= MAXR; ++k) {
    Cx[k] = Cy[k] = 0.0;
    if (k > r) continue;
    double ax = S[k][0], ay = S[k][1];  // zero for k > R
#pragma unroll
    for (int i = 1; i <= MAXR; ++i) {
      if (i > k) break;
      ax -= binom[k][i] * S[i][2] * Cx[k - i];
      ay -= binom[k][i] * S[i][2] * Cy[k - i];
    }
    Cx[k] = ax / W0;
    Cy[k] = ay / W0;
  }
  const double value = scale * (Cx[r] * Cx[r] + Cy[r] * Cy[r]);
  // reverse: Leibniz rule
  double dCx[MAXR + 1], dCy[MAXR + 1], dS[MAXR + 1][3];
#pragma unroll
  for (int k = 0; k <= MAXR; ++k) {
    dCx[k] = dCy[k] = 0.0;
    dS[k][0] = dS[k][1] = dS[k][2] = 0.0;
  }
  dCx[r] = up ? up[0] : 2.0 * scale * Cx[r];
  dCy[r] = up ? up[1] : 2.0 * scale * Cy[r];
#pragma unroll
  for (int k = MAXR; k >= 0; --k) {
    if (k > r) continue;
    const double gx = dCx[k] / W0, gy = dCy[k] / W0;
    dS[k][0] += gx;
    dS[k][1] += gy;
#pragma unroll
    for (int i = 1; i <= MAXR; ++i) {
      if (i > k) break;
      dS[i][2] -= binom[k][i] * (gx * Cx[k - i] + gy * Cy[k - i]);
      dCx[k - i] -= binom[k][i] * S[i][2] * gx;
      dCy[k - i] -= binom[k][i] * S[i][2] * gy;
    }
    dS[0][2] -= gx * Cx[k] + gy * Cy[k];
  }
  // reverse: S^(k) = sum_j N_{p-k}[j] PK_k[j]
  double dPK[MAXR + 1][PD + 1][3], dN[MAXR + 1][PD + 1];
#pragma unroll
  for (int k = 0; k <= MAXR; ++k)
#pragma unroll
    for (int j = 0; j <= PD; ++j) {
      dN[k][j] = 0.0;
      dPK[k][j][0] = dPK[k][j][1] = dPK[k][j][2] = 0.0;
    }
#pragma unroll
  for (int k = 0; k <= MAXR; ++k) {
    if (k > R) continue;
#pragma unroll
    for (int d = 0; d <= PD; ++d) {
      if (d != p - k) continue;
#pragma unroll
      for (int j = 0; j <= d; ++j) {
        const double n = tri[d * (d + 1) / 2 + j];
#pragma unroll
        for (int q = 0; q < 3; ++q) dPK[k][j][q] = n * dS[k][q];
        dN[k][j] = dS[k][0] * PK[k][j][0] + dS[k][1] * PK[k][j][1] + dS[k][2] * PK[k][j][2];
      }
    }
  }
  // reverse: derivative control points; knot slot s <-> knot index span - PD + 1 + s
#pragma unroll
  for (int k = 0; k < 2 * PD; ++k) out.knot[k] = 0.0;
#pragma unroll
  for (int k = MAXR; k >= 1; --k) {
    if (k > R) continue;
#pragma unroll
    for (int j = 0; j < PD; ++j) {
      if (j > p - k) break;
      const int hi = span + j + 1, lo = span - p + j + k;
      const double D = U[hi] - U[lo];
      const double c = (double)(p - k + 1) / D;
      double dD = 0.0;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        dPK[k - 1][j + 1][q] += c * dPK[k][j][q];
        dPK[k - 1][j][q] -= c * dPK[k][j][q];
        dD -= dPK[k][j][q] * PK[k][j][q];
      }
      dD /= D;
      out.knot[j + PD] += dD;  // slot of knot hi = span + j + 1
#pragma unroll
      for (int sl = 0; sl < 2 * PD; ++sl)
        if (sl == lo - span + PD - 1) out.knot[sl] -= dD;
    }
  }
  // homogeneous control points -> (x, y, w); the width does not enter
#pragma unroll
  for (int j = 0; j <= PD; ++j) {
    out.cp[j][0] = out.cp[j][1] = out.cp[j][2] = out.cp[j][3] = 0.0;
    if (j > p) continue;
    out.cp[j][0] = Wt[j] * dPK[0][j][0];
    out.cp[j][1] = Wt[j] * dPK[0][j][1];
    out.cp[j][2] = X[j] * dPK[0][j][0] + Y[j] * dPK[0][j][1] + dPK[0][j][2];
  }
  // reverse through the Cox-de Boor triangle (as point_adjoint), the degree
  // p - k adjoint dN[k] joining at level p - k
  double Nb[PD + 1];
#pragma unroll
  for (int q = 0; q <= PD; ++q) Nb[q] = dN[0][q];
  double ub = 0.0;
#pragma unroll
  for (int d = PD; d >= 1; --d) {
    if (d > p) continue;
#pragma unroll
    for (int k = 1; k <= MAXR; ++k)
      if (k <= R && d == p - k) {
#pragma unroll
        for (int q = 0; q <= PD; ++q) Nb[q] += dN[k][q];
      }
    double Np[PD + 1];
#pragma unroll
    for (int q = 0; q <= PD; ++q) Np[q] = 0.0;
#pragma unroll
    for (int q = 0; q <= d; ++q) {
      const double nb = Nb[q];
      const int i = span - d + q;
      if (q >= 1) {
        const double Ui = U[i], Uid = U[i + d];
        const double D = Uid - Ui;
        Np[q - 1] += nb * (u - Ui) / D;
        const double g = nb * tri[(d - 1) * d / 2 + q - 1];
        ub += g / D;
        out.knot[PD - 1 - d + q] -= g * (Uid - u) / (D * D);
        out.knot[PD - 1 + q] -= g * (u - Ui) / (D * D);
      }
      if (q <= d - 1) {
        const double Ui1 = U[i + 1], Uid1 = U[i + d + 1];
        const double D = Uid1 - Ui1;
        Np[q] += nb * (Uid1 - u) / D;
        const double g = nb * tri[(d - 1) * d / 2 + q];
        ub -= g / D;
        out.knot[PD + q] += g * (u - Ui1) / (D * D);
        out.knot[PD - d + q] += g * (Uid1 - u) / (D * D);
      }
    }
#pragma unroll
    for (int q = 0; q <= PD; ++q) Nb[q] = Np[q];
  }
  out.ubar = ub;
  return value;
}

// Penalty of Eq. 12 and its derivative: ReLU (kind 0) or softplus (kind 1).
__device__ inline double penalty(double x, int kind, double* d) {
  if (kind == 0) {
    *d = x > 0.0 ? 1.0 : 0.0;
    return x > 0.0 ? x : 0.0;
  }
  *d = 1.0 / (1.0 + exp(-x));
  return x > 0.0 ? x + log1p(exp(-x)) : log1p(exp(x));
}

struct RegArgs {
  double bbox_weight, deriv_weight;
  int bbox_kind, deriv_order;
  const float* bbox;
  float* loss;
};

// The scene's box: the given one, or the canvas [0, W] x [0, H].
__device__ inline void scene_box(const RegArgs& ra, const SceneTab* scenes, int s, double (&b)[4]) {
  if (ra.bbox) {
#pragma unroll
    for (int i = 0; i < 4; ++i) b[i] = (double)ra.bbox[4 * s + i];
  } else {
    b[0] = 0.0;
    b[1] = 0.0;
    b[2] = (double)scenes[s].W;
    b[3] = (double)scenes[s].H;
  }
}

// Bounding-box penalty of one point and its gradient.
__device__ inline double box_penalty(const RegArgs& ra, const double (&b)[4], double x, double y, double* gx,
                                     double* gy) {
  double d0, d1, d2, d3;
  const double v = penalty(b[0] - x, ra.bbox_kind, &d0) + penalty(x - b[2], ra.bbox_kind, &d1) +
                   penalty(b[1] - y, ra.bbox_kind, &d2) + penalty(y - b[3], ra.bbox_kind, &d3);
  *gx = ra.bbox_weight * (d1 - d0);
  *gy = ra.bbox_weight * (d3 - d2);
  return ra.bbox_weight * v;
}

// Number of curves of scene s (curves are grouped by scene in ascending order).
__device__ inline int curves_in_scene(const nsplat_curves& cv, int s) {
  int lo = 0, hi = cv.n_curves;  // first curve with scene >= s
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (cv.scene[mid] < s) lo = mid + 1;
    else hi = mid;
  }
  int a = lo;
  hi = cv.n_curves;  // first curve with scene > s
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (cv.scene[mid] <= s) lo = mid + 1;
    else hi = mid;
  }
  return lo - a;
}

// Trapezoid (open) or rectangle (closed) weight of sample j of `count`.
__device__ inline double quad_weight(int j, int count, bool closed) {
  if (closed) return 1.0 / (double)count;
  return (j == 0 || j == count - 1) ? 0.5 / (double)(count - 1) : 1.0 / (double)(count - 1);
}

// Block sum of two values into loss[0], loss[1] (one atomic each per block).
__device__ inline void block_loss(double a, double b, float* loss) {
  __shared__ double red[2][4];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    a += __shfl_xor(a, off);
    b += __shfl_xor(b, off);
  }
  if (__lane_id() == 0) {
    red[0][threadIdx.x >> 6] = a;
    red[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0 && loss) {
    const double ta = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    const double tb = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    if (ta != 0.0) unsafeAtomicAdd(loss, (float)ta);
    if (tb != 0.0) unsafeAtomicAdd(loss + 1, (float)tb);
  }
}

// Stroke samples (one lane per stroke Gaussian; endpoint copies skipped): the
// box gradient joins the Gaussian's centre adjoint, the derivative loss goes
// straight to the control points, knots and domain ends.
template <int PD>
__global__ __launch_bounds__(256, PD <= 3 ? 2 : 1) void k_reg_stroke(nsplat_curves cv, Work w, RegArgs ra, const int32_t* plan,
                                                    const int32_t* counters, const Gauss* __restrict__ gs,
                                                    int kappa) {
  if (w.queue[Q_NSTROKE] == 0) return;  // no Gaussians of this kind
  const int64_t G = counters[NSPLAT_CNT_GAUSS];
  const int lane = __lane_id();
  const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) - lane;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double lb = 0.0, ld = 0.0;
  for (int64_t base = wave0; base < G; base += stride) {
    const int64_t g = base + lane;
    int64_t kspan = -1 - lane, kcur = -1 - lane;
    double cur[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    PtAdj<PD> pa;
    int c = 0, span = 0;
    CurveView v;
    v.p = 0;
    bool act = false;
    if (g < G) {
      const Gauss rec = gs[g];
      c = rec.curve;
      v = curve_view(cv, w.knots, c);
      const int32_t* row = plan + (int64_t)P_STRIDE * c;
      const int M = row[P_NSAMP];
      const int j = v.closed() ? rec.local : rec.local - kappa;
      if (!v.filled() && curve_valid(v) && j >= 0 && j < M) {
        if (ra.bbox_weight != 0.0) {
          double b[4], gx, gy;
          scene_box(ra, w.scenes, cv.scene[c], b);
          lb += box_penalty(ra, b, rec.mx, rec.my, &gx, &gy);
          float* gg = w.ggrad + g * GG;
          gg[0] += (float)gx;
          gg[1] += (float)gy;
        }
        if (ra.deriv_weight != 0.0) {
          act = true;
          double dt;
          const double u = sample_u(v.U[v.p], v.U[v.m - v.p], j, M, v.closed(), &dt);
          span = find_span(v.U, v.p, v.m, u);
          const double sc = ra.deriv_weight / (double)curves_in_scene(cv, cv.scene[c]) *
                            quad_weight(j, M, v.closed());
          ld += deriv_adjoint(cv, v, u, span, ra.deriv_order, sc, pa);
          cur[4] = pa.ubar * (1.0 - dt);
          cur[5] = pa.ubar * dt;
          kspan = (int64_t)v.t0 + (int64_t)c * KNOT_PAD + span;
          kcur = c;
        }
      }
    }
    if (!act) {
#pragma unroll
      for (int q = 0; q <= PD; ++q)
#pragma unroll
        for (int k = 0; k < 4; ++k) pa.cp[q][k] = 0.0;
#pragma unroll
      for (int k = 0; k < 2 * PD; ++k) pa.knot[k] = 0.0;
    }
    const bool any = __ballot(act) != 0ull;
    accumulate_points(w, kspan, c, v, span, pa, any);
    if (any) accumulate_curve(w, kcur, c, v, cur);
  }
  block_loss(lb, ld, ra.loss);
}

// Fill boundary samples (one lane per boundary point): the box gradient joins
// the boundary-point adjoint, the derivative loss goes straight to the curve.
template <int PD>
__global__ __launch_bounds__(256, PD <= 3 ? 2 : 1) void k_reg_boundary(nsplat_curves cv, Work w, RegArgs ra, const int32_t* plan,
                                                      const int32_t* counters) {
  const int64_t NB = counters[NSPLAT_CNT_BOUND];
  const int lane = __lane_id();
  const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) - lane;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int n = cv.n_curves;
  double lb = 0.0, ld = 0.0;
  for (int64_t base = wave0; base < NB; base += stride) {
    const int64_t bi = base + lane;
    int64_t kspan = -1 - lane, kcur = -1 - lane;
    double cur[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    PtAdj<PD> pa;
    int c = 0, span = 0;
    CurveView v;
    v.p = 0;
    bool act = false;
    if (bi < NB) {
      c = last_le_wave<P_STRIDE, P_BOFF>(plan, n, bi);  // the last c with boff <= bi
      v = curve_view(cv, w.knots, c);
      const int32_t* row = plan + (int64_t)P_STRIDE * c;
      const int nb = row[P_NSAMP];
      const int j = (int)(bi - row[P_BOFF]);
      if (v.filled() && curve_valid(v) && j >= 0 && j < nb) {
        if (ra.bbox_weight != 0.0) {
          double b[4], gx, gy;
          scene_box(ra, w.scenes, cv.scene[c], b);
          const double2 q = w.bpts[bi];
          lb += box_penalty(ra, b, q.x, q.y, &gx, &gy);
          w.gb[bi].x += gx;
          w.gb[bi].y += gy;
        }
        if (ra.deriv_weight != 0.0) {
          act = true;
          double dt;
          const double u = sample_u(v.U[v.p], v.U[v.m - v.p], j, nb, true, &dt);
          span = find_span(v.U, v.p, v.m, u);
          const double sc = ra.deriv_weight / (double)curves_in_scene(cv, cv.scene[c]) * quad_weight(j, nb, true);
          ld += deriv_adjoint(cv, v, u, span, ra.deriv_order, sc, pa);
          cur[4] = pa.ubar * (1.0 - dt);
          cur[5] = pa.ubar * dt;
          kspan = (int64_t)v.t0 + (int64_t)c * KNOT_PAD + span;
          kcur = c;
        }
      }
    }
    if (!act) {
#pragma unroll
      for (int q = 0; q <= PD; ++q)
#pragma unroll
        for (int k = 0; k < 4; ++k) pa.cp[q][k] = 0.0;
#pragma unroll
      for (int k = 0; k < 2 * PD; ++k) pa.knot[k] = 0.0;
    }
    const bool any = __ballot(act) != 0ull;
    accumulate_points(w, kspan, c, v, span, pa, any);
    if (any) accumulate_curve(w, kcur, c, v, cur);
  }
  block_loss(lb, ld, ra.loss);
}

// Tangent-aligned stroke Gaussians: centre mu = C(u_j), sp = s(u_j) / rho
// across the curve, sigma = max(sp, |C'(u_j)| du / rho) along
// t = C'(u_j) / |C'(u_j)| = (cos theta, sin theta), du the sample spacing.
// dL/d(mu, sp) and, where sigma = sp, dL/dsigma go to the point adjoint;
// dL/dtheta (d theta / d C' = n / |C'|, n = (-t_y, t_x)) and, where the
// spacing term is the larger, dL/dsigma (d sigma / d C' = t du / rho) go to
// the adjoint of the first derivative C'(u_j), whose reverse pass is that of
// the derivative loss; dL/d du = dL/dsigma |C'| / rho goes to the domain
// ends (du = (u_{m-p} - u_p) / (M - 1), or / M closed).
template <int PD>
__global__ __launch_bounds__(256) void k_adj_aniso(nsplat_curves cv, nsplat_params pr, Work w,
                                                   const int32_t* plan, const int32_t* counters,
                                                   const Gauss* __restrict__ gs) {
  if (w.queue[Q_NANISO] == 0) return;  // no Gaussians of this kind
  const int64_t G = counters[NSPLAT_CNT_GAUSS];
  const int lane = __lane_id();
  const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) - lane;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const double rho = (double)pr.rho;
  for (int64_t base = wave0; base < G; base += stride) {
    const int64_t g = base + lane;
    int64_t kspan = -1 - lane, kcur = -1 - lane;
    double cur[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    PtAdj<PD> pa;
    int c = 0, span = 0;
    CurveView v;
    v.p = 0;
    bool act = false;
    if (g < G) {
      const Gauss r = gs[g];
      c = r.curve;
      if ((cv.flags[c] & (NSPLAT_FILLED | NSPLAT_ANISO)) == NSPLAT_ANISO) {
        act = true;
        v = curve_view(cv, w.knots, c);
        const float* gg = w.ggrad + g * GG;
        const int32_t* row = plan + (int64_t)P_STRIDE * c;
        const int M = row[P_NSAMP];
        int j = v.closed() ? r.local : r.local - pr.kappa;
        j = j < 0 ? 0 : (j > M - 1 ? M - 1 : j);
        double dt;
        const double u = sample_u(v.U[v.p], v.U[v.m - v.p], j, M, v.closed(), &dt);
        span = find_span(v.U, v.p, v.m, u);
        double pt[3], d[3];
        curve_point(cv, v, u, span, pt, d);
        const double len = sqrt(d[0] * d[0] + d[1] * d[1]);
        const double den = (double)(v.closed() ? M : M - 1);
        const double du = (v.U[v.m - v.p] - v.U[v.p]) / den;
        const double sp = pt[2] / rho;
        const bool wide = len > 0.0 && len * du / rho > sp;  // the spacing term sets sigma
        const double gsig = (double)gg[2], gsp = (double)gg[3], gth = (double)gg[4];
        const double ab[3] = {(double)gg[0], (double)gg[1], (gsp + (wide ? 0.0 : gsig)) / rho};
        point_adjoint(cv, v, u, span, ab, pa);
        double ddu = 0.0;
        if (len > 0.0) {
          const double tx = d[0] / len, ty = d[1] / len;
          double up[2] = {-ty * gth / len, tx * gth / len};
          if (wide) {
            up[0] += gsig * tx * du / rho;
            up[1] += gsig * ty * du / rho;
            ddu = gsig * len / rho;
          }
          PtAdj<PD> pd;
          deriv_adjoint(cv, v, u, span, 1, 0.0, pd, up);
#pragma unroll
          for (int q = 0; q <= PD; ++q)
#pragma unroll
            for (int k = 0; k < 4; ++k) pa.cp[q][k] += pd.cp[q][k];
#pragma unroll
          for (int k = 0; k < 2 * PD; ++k) pa.knot[k] += pd.knot[k];
          pa.ubar += pd.ubar;
        }
        cur[4] = pa.ubar * (1.0 - dt) - ddu / den;  // u_j = u_p + t_j (u_{m-p} - u_p)
        cur[5] = pa.ubar * dt + ddu / den;
        kspan = (int64_t)v.t0 + (int64_t)c * KNOT_PAD + span;
        kcur = c;
      }
    }
    if (!act) {
#pragma unroll
      for (int q = 0; q <= PD; ++q)
#pragma unroll
        for (int k = 0; k < 4; ++k) pa.cp[q][k] = 0.0;
#pragma unroll
      for (int k = 0; k < 2 * PD; ++k) pa.knot[k] = 0.0;
    }
    const bool any = __ballot(act) != 0ull;
    accumulate_points(w, kspan, c, v, span, pa, any);
    if (any) accumulate_curve(w, kcur, c, v, cur);
  }
}

}  // namespace

hipError_t launch_zero_grads(const Launch& L) {
  Phase ph(L, NSPLAT_T_FOLD);
  const nsplat_curves& cv = *L.cv;
  const int64_t ncp = (int64_t)cv.n_keys + (int64_t)cv.n_curves * CP_PAD;
  const int64_t nkn = (int64_t)cv.n_taus + (int64_t)cv.n_curves * KNOT_PAD;
  ZeroSet z;
  z.p[0] = L.w.gcp;
  z.n[0] = 4 * ncp;
  z.p[1] = L.w.gknot;
  z.n[1] = nkn;
  z.p[2] = L.w.gcurve;
  z.n[2] = (int64_t)4 * cv.n_curves;
  z.p[3] = (double*)L.w.gb;
  z.n[3] = L.bf->caps.boundary > 0 ? 2 * L.bf->caps.boundary : 0;
  const int64_t total = z.n[0] + z.n[1] + z.n[2] + z.n[3];
  const int64_t most = std::max<int64_t>(L.bf->caps.gauss * GG, total);
  hipLaunchKernelGGL(k_zero_grads, dim3(grid_for(most, 256, 8192)), dim3(256), 0, L.stream, L.w.ggrad,
                     L.bf->counters + NSPLAT_CNT_GAUSS, (int64_t)GG, (int64_t)L.bf->caps.gauss, z);
  return hipGetLastError();
}

// Array bound of the point and derivative adjoints: 3 when the batch declares
// no degree above 3 (curve_valid rejects any curve above the bound).
inline bool low_degree(const Launch& L) { return L.cv->max_degree >= 1 && L.cv->max_degree <= 3; }

template <int PD>
void launch_reg_d(const Launch& L, const RegArgs& ra) {
  hipLaunchKernelGGL(k_reg_stroke<PD>, dim3(grid_for(L.bf->caps.gauss, 256, 4096)), dim3(256), 0, L.stream, *L.cv,
                     L.w, ra, L.bf->plan, L.bf->counters, (const Gauss*)L.bf->gauss, L.pr->kappa);
  if (L.bf->caps.boundary > 0)
    hipLaunchKernelGGL(k_reg_boundary<PD>, dim3(grid_for(L.bf->caps.boundary, 256, 4096)), dim3(256), 0, L.stream,
                       *L.cv, L.w, ra, L.bf->plan, L.bf->counters);
}

template <int PD>
void launch_adj_stroke_d(const Launch& L) {
  hipLaunchKernelGGL(k_adj_stroke<PD>, dim3(grid_for(L.bf->caps.gauss, 256, 8192)), dim3(256), 0, L.stream, *L.cv,
                     *L.pr, L.w, L.bf->plan, L.bf->counters, (const Gauss*)L.bf->gauss);
}

template <int PD>
void launch_adj_aniso_d(const Launch& L) {
  hipLaunchKernelGGL(k_adj_aniso<PD>, dim3(grid_for(L.bf->caps.gauss, 256, 4096)), dim3(256), 0, L.stream, *L.cv,
                     *L.pr, L.w, L.bf->plan, L.bf->counters, (const Gauss*)L.bf->gauss);
}

template <int PD>
void launch_adj_boundary_d(const Launch& L) {
  hipLaunchKernelGGL(k_adj_boundary<PD>, dim3(grid_for(L.bf->caps.boundary, 256, 4096)), dim3(256), 0, L.stream,
                     *L.cv, L.w, L.bf->plan, L.bf->counters);
}

hipError_t launch_reg(const Launch& L, const nsplat_reg* reg) {
  Phase ph(L, NSPLAT_T_REG);
  RegArgs ra;
  ra.bbox_weight = (double)reg->bbox_weight;
  ra.deriv_weight = (double)reg->deriv_weight;
  ra.bbox_kind = reg->bbox_kind;
  ra.deriv_order = reg->deriv_order;
  ra.bbox = reg->bbox;
  ra.loss = reg->loss;
  if (low_degree(L)) launch_reg_d<3>(L, ra);
  else launch_reg_d<MAXP>(L, ra);
  return hipGetLastError();
}

hipError_t launch_adjoint(const Launch& L, const nsplat_grads* g) {
  {
    Phase ph(L, NSPLAT_T_ADJ_GAUSS);
    // kinds the batch declares none of are not launched (any_flags, all_flags)
    const bool ani = (L.cv->any_flags & NSPLAT_ANISO) != 0;
    const bool strokes = (L.cv->all_flags & NSPLAT_FILLED) == 0;
    const bool fills = (L.cv->any_flags & NSPLAT_FILLED) != 0;
    if (low_degree(L)) {
      if (strokes) launch_adj_stroke_d<3>(L);
      if (ani) launch_adj_aniso_d<3>(L);
    } else {
      if (strokes) launch_adj_stroke_d<MAXP>(L);
      if (ani) launch_adj_aniso_d<MAXP>(L);
    }
    if (fills)
      hipLaunchKernelGGL(k_adj_fill, dim3(grid_for(L.bf->caps.gauss, 256, 8192)), dim3(256), 0, L.stream, *L.cv,
                         *L.pr, L.w, L.bf->plan, L.bf->counters, (const Gauss*)L.bf->gauss);
  }
  if (L.bf->caps.boundary > 0 && (L.cv->any_flags & NSPLAT_FILLED)) {
    Phase ph(L, NSPLAT_T_ADJ_BOUND);
    if (low_degree(L)) launch_adj_boundary_d<3>(L);
    else launch_adj_boundary_d<MAXP>(L);
  }
  Phase ph(L, NSPLAT_T_FOLD);
  if (L.cv->n_curves > 0)
    hipLaunchKernelGGL(k_fold, dim3(L.cv->n_curves), dim3(64), 0, L.stream, *L.cv, L.w, *g);
  return hipGetLastError();
}

}  // namespace nsp
