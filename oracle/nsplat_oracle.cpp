// TEST INFRASTRUCTURE ONLY -- the FP64 CPU oracle for the NURBS Splatting
// render path (Qiu & Zhou, "NURBS Splatting: A Unified Differentiable
// Rendering Framework for Vector Graphics").
//
// A deliberately plain, slow, brute-force reference.  Only the test suite,
// the smoke check and the CPU-baseline leg of the benchmark load it.  It
// shares no code, header, table or helper with the GPU library, and the GPU
// library never calls it.
//
// What it computes, step by step, in the order of the paper:
//   Sec. 3.1     key points -> control polygon, weights, widths, knot vector
//   Eq. 1, 2     rational curve point and its u-derivative (Cox-de Boor)
//   Eq. 3        arc length by N_L-point quadrature
//   Sec. 3.2     M = ceil(delta_c L) contour samples, uniform in the domain,
//   Eq. 4, 5     span-local evaluation, isotropic sigma = s / rho, o_j = o,
//                endpoint replication (kappa copies)
//   Sec. 3.3     fill: ceil(delta_b L) boundary points, padded AABB, grid,
//   Eq. 6, 7     sigma = eta h / rho, o_j = o sigmoid(gamma / h sdf(q_j))
//   Suppl. S2    sdf = sgn(wn) d, d = distance to the closed polyline,
//   Eq. S1-S3    wn = angle-sum winding number (detached)
//   Sec. 3.4     tile binning (emulated in FP32 from the oracle's own centres)
//   Eq. 8, 9     front-to-back alpha compositing of EVERY Gaussian at EVERY
//                pixel, residual transmittance onto the background
//   Eq. 14       grid-step annealing schedule
//   Sec. 3.5     the geometric regularisers: derivative (fairing) loss,
//                Eq. 11, from k-th basis derivatives (NURBS Book Eq. 2.9) and
//                the rational Leibniz rule, and the bounding-box loss, Eq. 12
//   Sec. 4.2     the distance-weighted image loss of layer-wise vectorisation
//                (LIVE's unsigned-distance weights, udf_weight)
// and the exact derivative of the image loss with respect to every curve
// parameter: the compositing adjoint is written out per pixel; the map from
// curve parameters to Gaussians is differentiated in forward mode with dual
// numbers (one seeded parameter at a time), so no hand-derived NURBS adjoint
// is involved.
//
// Readings where the paper is silent (span rule at the right end, midpoint
// quadrature, sample spacing, count floors, endpoint replicas, global fill
// lattice, stacking order, alpha clamp, termination) are parameters or are
// stated at the function that takes them.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------------------
// Dual numbers: value and the derivative with respect to one seeded input.
// ---------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual(double v_ = 0.0, double d_ = 0.0) : v(v_), d(d_) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual sqrt(Dual a) {
  double s = std::sqrt(a.v);
  return Dual(s, s > 0.0 ? a.d / (2.0 * s) : 0.0);  // gradient 0 at distance 0
}
inline Dual exp(Dual a) { double e = std::exp(a.v); return Dual(e, e * a.d); }
inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
inline double sqrt(double x) { return std::sqrt(x); }
inline double exp(double x) { return std::exp(x); }

template <class T> T lift(double v, bool seed);
template <> double lift<double>(double v, bool) { return v; }
template <> Dual lift<Dual>(double v, bool seed) { return Dual(v, seed ? 1.0 : 0.0); }

template <class T> T sigmoid(const T& z) { return T(1.0) / (T(1.0) + exp(-z)); }

}  // namespace

extern "C" {

// Curve batch (CSR over curves, host arrays, FP64 copies of the FP32 inputs).
typedef struct {
  int32_t n_curves, channels;
  const int32_t *scene, *degree, *flags, *key_off, *tau_off;
  const double *key_xy, *key_w, *key_s, *tau, *color, *opacity;
} or_curves;

typedef struct {
  int32_t n_scenes;
  const int32_t* hw;   // [S][2] = {height, width}
  const double* bg;    // [S][channels]
} or_scenes;

typedef struct {
  double delta_c, delta_b, rho, eta, gamma, nl_factor, fill_pad, h;
  double alpha_max;  // per-pixel opacity clamp (1 = none)
  double eps_T;      // stop a pixel once T < eps_T (0 = never)
  double cutoff;     // support radius in sigmas (<= 0: none)
  double delta_a;    // contour density of tangent-aligned (anisotropic) strokes
  int32_t kappa;     // extra copies of each open-curve endpoint
} or_params;

// Geometric regularisers of Sec. 3.5, evaluated at the parameters u_j of the
// curve's own samples (contour samples of a stroke, boundary points of a fill).
typedef struct {
  double bbox_weight;    // lambda of Eq. 12 (0: off)
  int32_t bbox_kind;     // penalty phi: 0 ReLU, 1 softplus
  const double* bbox;    // [S][4] = {x_min, y_min, x_max, y_max}, or NULL for [0, W] x [0, H]
  double deriv_weight;   // lambda of Eq. 11 (0: off)
  int32_t deriv_order;   // r
} or_reg;

}  // extern "C"

namespace {

enum { F_CLOSED = 1, F_FILLED = 2, F_ANISO = 4 };
enum { S_NONE = 0, S_KEY_X = 1, S_KEY_Y = 2, S_KEY_W = 3, S_KEY_S = 4, S_TAU = 5, S_OPACITY = 6 };
enum { P_COUNT = 0, P_NSAMP = 1, P_IX0 = 2, P_IY0 = 3, P_NX = 4, P_NY = 5, P_GOFF = 6, P_FLAG = 7, P_STRIDE = 8 };

// ---------------------------------------------------------------------------
// Sec. 3.1: a NURBS curve built from its key points.
// ---------------------------------------------------------------------------
template <class T>
struct Curve {
  int p = 0, nk = 0, ncp = 0, m = 0;  // degree, key points, control points, last knot index
  bool closed = false, filled = false;
  std::vector<T> U;                   // knots u_0..u_m
  std::vector<T> X, Y, S, W;          // control points (x, y, width) and weights
  int key_of_cp(int j) const { return closed ? ((j - (p + 1) / 2) % nk + nk) % nk : j; }
};

// Builds control polygon and knot vector of curve c; the input (kind, index)
// given by `seed` carries derivative 1 (index is local to the curve).
template <class T>
Curve<T> build_curve(const or_curves* in, int c, int seed_kind, int seed_index) {
  Curve<T> cv;
  cv.p = in->degree[c];
  cv.closed = (in->flags[c] & F_CLOSED) != 0;
  cv.filled = (in->flags[c] & F_FILLED) != 0;
  const int k0 = in->key_off[c];
  cv.nk = in->key_off[c + 1] - k0;
  const int t0 = in->tau_off[c];
  const int nt = in->tau_off[c + 1] - t0;
  const int p = cv.p;
  // Open: control points = key points.  Closed: wrap the last ceil(p/2) and the
  // first floor(p/2) key points around, n_k + p control points.
  cv.ncp = cv.closed ? cv.nk + p : cv.nk;
  for (int j = 0; j < cv.ncp; ++j) {
    const int k = cv.key_of_cp(j);
    cv.X.push_back(lift<T>(in->key_xy[2 * (k0 + k)], seed_kind == S_KEY_X && seed_index == k));
    cv.Y.push_back(lift<T>(in->key_xy[2 * (k0 + k) + 1], seed_kind == S_KEY_Y && seed_index == k));
    cv.W.push_back(lift<T>(in->key_w[k0 + k], seed_kind == S_KEY_W && seed_index == k));
    cv.S.push_back(lift<T>(in->key_s[k0 + k], seed_kind == S_KEY_S && seed_index == k));
  }
  // Knot intervals.  Open: p zero intervals, the n_k - p stored intervals, p
  // zero intervals.  Closed: last p stored intervals, all n_k, first p.
  std::vector<T> tau;
  for (int j = 0; j < nt; ++j) tau.push_back(lift<T>(in->tau[t0 + j], seed_kind == S_TAU && seed_index == j));
  std::vector<T> delta;
  if (!cv.closed) {
    for (int j = 0; j < p; ++j) delta.push_back(T(0.0));
    for (int j = 0; j < nt; ++j) delta.push_back(tau[j]);
    for (int j = 0; j < p; ++j) delta.push_back(T(0.0));
  } else {
    for (int l = 0; l < nt + 2 * p; ++l) delta.push_back(tau[((l - p) % nt + nt) % nt]);
  }
  // Cumulative sum, starting at 0.
  cv.U.push_back(T(0.0));
  for (size_t l = 0; l < delta.size(); ++l) cv.U.push_back(cv.U.back() + delta[l]);
  cv.m = (int)cv.U.size() - 1;
  return cv;
}

template <class T> double dom_lo(const Curve<T>& cv) { return val(cv.U[cv.p]); }
template <class T> double dom_hi(const Curve<T>& cv) { return val(cv.U[cv.m - cv.p]); }

// Knot span containing u: the largest i in [p, m-p-1] with u_i <= u < u_{i+1};
// at (or beyond) the right end of the domain, the last non-empty span.
template <class T>
int find_span(const Curve<T>& cv, double u) {
  const int lo = cv.p, hi = cv.m - cv.p - 1;
  const auto& U = cv.U;
  // first index with U[k] > u, minus one: the largest k with U[k] <= u
  int i = (int)(std::upper_bound(U.begin(), U.end(), u,
                                 [](double x, const T& k) { return x < val(k); }) - U.begin()) - 1;
  if (i > hi) i = hi;
  if (i < lo) i = lo;
  while (i > lo && !(val(U[i]) < val(U[i + 1]))) --i;      // step back over empty spans
  while (i < hi && !(val(U[i]) < val(U[i + 1]))) ++i;
  return i;
}

// Cox-de Boor recursion (The NURBS Book, Eq. 2.5); 0/0 := 0.  The degree-0
// functions are the indicator of the span chosen by find_span, which makes
// the right end of the domain belong to the last non-empty span.
template <class T>
T basis(const std::vector<T>& U, int i, int d, const T& u, int span) {
  if (d == 0) return T(i == span ? 1.0 : 0.0);
  T a(0.0), b(0.0);
  const T den1 = U[i + d] - U[i];
  if (val(den1) != 0.0) a = (u - U[i]) / den1 * basis(U, i, d - 1, u, span);
  const T den2 = U[i + d + 1] - U[i + 1];
  if (val(den2) != 0.0) b = (U[i + d + 1] - u) / den2 * basis(U, i + 1, d - 1, u, span);
  return a + b;
}

// Eq. 1 (and Eq. 4): C(u) = sum N w P / sum N w over (x, y, width).  Only
// N_{span-p..span} can be non-zero (every other N_{i,p} is built from
// degree-0 functions that vanish), so the sum runs over those; `full` sums
// over every control point instead, which tests use to check that claim.
template <class T>
void curve_point(const Curve<T>& cv, const T& u, int span, T out[3], bool full = false) {
  T Sx(0.0), Sy(0.0), Ss(0.0), Wt(0.0);
  const int i0 = full ? 0 : span - cv.p, i1 = full ? cv.ncp - 1 : span;
  for (int i = i0; i <= i1; ++i) {
    const T nw = basis(cv.U, i, cv.p, u, span) * cv.W[i];
    Sx += nw * cv.X[i];
    Sy += nw * cv.Y[i];
    Ss += nw * cv.S[i];
    Wt += nw;
  }
  out[0] = Sx / Wt;
  out[1] = Sy / Wt;
  out[2] = Ss / Wt;
}

// Eq. 2: C'(u) = (W sum N' w P - S sum N' w) / W^2, with N' the u-derivative
// of the Cox-de Boor recursion (taken with a dual number seeded on u).
void curve_deriv(const Curve<double>& cv, const std::vector<Dual>& U, double u, int span, double out[3],
                 bool full = false) {
  const Dual ud(u, 1.0);
  double S[3] = {0, 0, 0}, Sd[3] = {0, 0, 0}, Wt = 0, Wd = 0;
  const int i0 = full ? 0 : span - cv.p, i1 = full ? cv.ncp - 1 : span;
  for (int i = i0; i <= i1; ++i) {
    const Dual n = basis(U, i, cv.p, ud, span);
    const double P[3] = {cv.X[i], cv.Y[i], cv.S[i]};
    for (int k = 0; k < 3; ++k) {
      S[k] += n.v * cv.W[i] * P[k];
      Sd[k] += n.d * cv.W[i] * P[k];
    }
    Wt += n.v * cv.W[i];
    Wd += n.d * cv.W[i];
  }
  for (int k = 0; k < 3; ++k) out[k] = (Wt * Sd[k] - S[k] * Wd) / (Wt * Wt);
}

// Eq. 3 with N_L midpoint samples: L = sum_j ||C'(u_j)|| du.
double arc_length(const Curve<double>& cv, int n_L) {
  const double a = dom_lo(cv), b = dom_hi(cv);
  const double du = (b - a) / n_L;
  const std::vector<Dual> Ud(cv.U.begin(), cv.U.end());  // knots as constants for the u-derivative
  double L = 0.0;
  for (int j = 1; j <= n_L; ++j) {
    const double u = a + (j - 0.5) * du;
    double d[3];
    curve_deriv(cv, Ud, u, find_span(cv, u), d);
    L += std::sqrt(d[0] * d[0] + d[1] * d[1]) * du;
  }
  return L;
}

// Sample parameters, uniform in the domain [a, b].  Open: M values with both
// ends included (the last one is b exactly).  Closed: M values a + j (b-a)/M,
// the closure point b (= a on the curve) excluded.
template <class T>
T sample_u(const Curve<T>& cv, int j, int M, bool closed) {
  const T a = cv.U[cv.p], b = cv.U[cv.m - cv.p];
  if (!closed) {
    if (j >= M - 1) return b;
    const T step = (b - a) / T((double)(M - 1));
    return a + T((double)j) * step;
  }
  const T step = (b - a) / T((double)M);
  return a + T((double)j) * step;
}

// Sec. 3.1 fixes the value domain of a curve: rational weights w_i > 0 and
// knot intervals tau_j >= 0 (the knot vector is their cumulative sum) whose
// sum, the length of the parameter domain, is positive; a stroke's widths are
// the third coordinate of its control points and set sigma = s / rho > 0.  A
// curve outside that domain (or with a non-finite input) is rendered as
// absent.
bool values_in_domain(const or_curves* in, int c) {
  const bool filled = (in->flags[c] & F_FILLED) != 0;
  for (int k = in->key_off[c]; k < in->key_off[c + 1]; ++k) {
    if (!std::isfinite(in->key_xy[2 * k]) || !std::isfinite(in->key_xy[2 * k + 1])) return false;
    if (!(in->key_w[k] > 0.0) || !std::isfinite(in->key_w[k])) return false;
    if (!filled && (!(in->key_s[k] > 0.0) || !std::isfinite(in->key_s[k]))) return false;
  }
  double sum = 0.0;
  for (int t = in->tau_off[c]; t < in->tau_off[c + 1]; ++t) {
    if (!(in->tau[t] >= 0.0) || !std::isfinite(in->tau[t])) return false;
    sum += in->tau[t];
  }
  if (!(sum > 0.0)) return false;
  if (!std::isfinite(in->opacity[c])) return false;
  for (int ch = 0; ch < in->channels; ++ch)
    if (!std::isfinite(in->color[in->channels * c + ch])) return false;
  return true;
}

// Count rule of Sec. 3.2 / 3.3: ceil(delta L) with a floor (2 for open
// strokes, 3 for closed strokes and for fill boundaries).  Flags values that
// are within 1e-9 of an integer (two FP64 evaluations could round apart).
int count_rule(double delta, double L, int floor_min, int* flag) {
  const double x = delta * L;
  const double r = std::nearbyint(x);
  if (std::fabs(x - r) < 1e-9 && r >= floor_min) *flag = 1;
  const int M = (int)std::ceil(x);
  return M < floor_min ? floor_min : M;
}

// Suppl. S2, Eq. S1: distance from q to segment [a, b], projection clamped.
template <class T>
T seg_dist(const T& qx, const T& qy, const T& ax, const T& ay, const T& bx, const T& by) {
  const T ex = bx - ax, ey = by - ay;
  const T ee = ex * ex + ey * ey;
  T t(0.0);
  if (val(ee) > 0.0) t = ((qx - ax) * ex + (qy - ay) * ey) / ee;
  if (val(t) < 0.0) t = T(0.0);
  if (val(t) > 1.0) t = T(1.0);
  const T px = ax + t * ex - qx, py = ay + t * ey - qy;
  return sqrt(px * px + py * py);
}

// Suppl. S2, Eq. S2: winding number as the sum of signed angles / (2 pi).
double winding(double qx, double qy, const std::vector<double>& bx, const std::vector<double>& by) {
  const int n = (int)bx.size();
  double s = 0.0;
  for (int i = 0; i < n; ++i) {
    const int k = (i + 1) % n;
    const double ax = bx[i] - qx, ay = by[i] - qy, cx = bx[k] - qx, cy = by[k] - qy;
    s += std::atan2(ax * cy - ay * cx, ax * cx + ay * cy);
  }
  return s / (2.0 * M_PI);
}

// Eq. S1-S3: signed distance, positive inside.  The sign is a plain double
// (no derivative); the distance is the minimum over segments (strict <, so the
// lowest segment index wins a tie).
template <class T>
T sdf(double qx, double qy, const std::vector<T>& bx, const std::vector<T>& by) {
  const int n = (int)bx.size();
  T best(0.0);
  bool first = true;
  for (int i = 0; i < n; ++i) {
    const int k = (i + 1) % n;
    const T d = seg_dist(T(qx), T(qy), bx[i], by[i], bx[k], by[k]);
    if (first || val(d) < val(best)) { best = d; first = false; }
  }
  std::vector<double> vx(n), vy(n);
  for (int i = 0; i < n; ++i) { vx[i] = val(bx[i]); vy[i] = val(by[i]); }
  const double wn = winding(qx, qy, vx, vy);
  const double sgn = wn > 0.5 ? 1.0 : -1.0;
  return T(sgn) * best;
}

struct SceneGeom { int H, W, n_L; };

SceneGeom scene_geom(const or_scenes* sc, const or_params* pr, int s) {
  SceneGeom g;
  g.H = sc->hw[2 * s];
  g.W = sc->hw[2 * s + 1];
  g.n_L = (int)std::lround(pr->nl_factor * (double)std::max(g.H, g.W));
  return g;
}

// Boundary points of a filled curve (Sec. 3.3): N_b points, closed spacing.
template <class T>
void boundary_points(const Curve<T>& cv, int nb, std::vector<T>& bx, std::vector<T>& by) {
  bx.resize(nb);
  by.resize(nb);
  for (int j = 0; j < nb; ++j) {
    const T u = sample_u(cv, j, nb, true);
    T pt[3];
    curve_point(cv, u, find_span(cv, val(u)), pt);
    bx[j] = pt[0];
    by[j] = pt[1];
  }
}

// Fill lattice window: the global lattice q = ((i + 1/2) h, (j + 1/2) h)
// restricted to the boundary's AABB, padded on each side by fill_pad times
// its extent, clipped to the canvas [0, W] x [0, H].
void fill_window(const std::vector<double>& bx, const std::vector<double>& by, double pad,
                 double h, int W, int H, int win[4]) {
  const double x0 = *std::min_element(bx.begin(), bx.end());
  const double x1 = *std::max_element(bx.begin(), bx.end());
  const double y0 = *std::min_element(by.begin(), by.end());
  const double y1 = *std::max_element(by.begin(), by.end());
  const double px = pad * (x1 - x0), py = pad * (y1 - y0);
  const double bx0 = std::max(0.0, x0 - px), bx1 = std::min((double)W, x1 + px);
  const double by0 = std::max(0.0, y0 - py), by1 = std::min((double)H, y1 + py);
  const int ix0 = (int)std::ceil(bx0 / h - 0.5), ix1 = (int)std::floor(bx1 / h - 0.5);
  const int iy0 = (int)std::ceil(by0 / h - 0.5), iy1 = (int)std::floor(by1 / h - 0.5);
  win[0] = ix0;
  win[1] = iy0;
  win[2] = std::max(0, ix1 - ix0 + 1);
  win[3] = std::max(0, iy1 - iy0 + 1);
}

// One Gaussian: centre, sigma, opacity.
// One Gaussian: centre, sigma (the axis along the curve tangent for a
// tangent-aligned stroke Gaussian, else the isotropic sigma), opacity, and
// for a tangent-aligned one the axis across the curve and the tangent
// direction (isotropic: sp = sigma, t = (1, 0)).
template <class T>
struct Gauss { T mx, my, sigma, opacity, sp, tx, ty; };

// Gaussians of curve c for a given plan row, in emission order: open strokes
// [kappa copies of sample 0, samples 0..M-1, kappa copies of sample M-1];
// closed strokes samples 0..M-1; fills the lattice window row by row.
// If `need` is given, lattice Gaussians j with need[j] == false are left at
// zero (their terms of a sum that weights them by a zero adjoint vanish).
template <class T>
void curve_gaussians(const or_curves* in, const or_scenes* sc, const or_params* pr, int c,
                     const int32_t* plan_row, int seed_kind, int seed_index, std::vector<Gauss<T>>& out,
                     const std::vector<char>* need = nullptr) {
  out.clear();
  const int count = plan_row[P_COUNT], ns = plan_row[P_NSAMP];
  if (count <= 0 || ns <= 0) return;  // no Gaussians (e.g. a curve outside the value domain)
  const Curve<T> cv = build_curve<T>(in, c, seed_kind, seed_index);
  const T o = lift<T>(in->opacity[c], seed_kind == S_OPACITY);
  if (!cv.filled) {
    const int kap = cv.closed ? 0 : pr->kappa;
    const bool aniso = (in->flags[c] & F_ANISO) != 0;
    std::vector<Gauss<T>> smp(ns);
    for (int j = 0; j < ns; ++j) {
      const T u = sample_u(cv, j, ns, cv.closed);
      const int span = find_span(cv, val(u));
      T pt[3];
      curve_point(cv, u, span, pt);
      const T sg = pt[2] / T(pr->rho);
      smp[j] = Gauss<T>{pt[0], pt[1], sg, o, sg, T(1.0), T(0.0)};     // Eq. 5
      if (aniso) {
        // Tangent-aligned variant of Eq. 5 (the contour sampling of Bezier
        // Splatting that the paper contrasts with, Sec. 3.2): the axis across
        // the curve keeps s / rho, the axis along the tangent t = C' / |C'|
        // (Eq. 2) covers the local sample spacing |C'| du with the same
        // overlap ratio rho, and never falls below the axis across it.
        std::vector<T> Dx, Dy;
        curve_derivs(cv, u, span, 1, Dx, Dy);
        const T len = sqrt(Dx[1] * Dx[1] + Dy[1] * Dy[1]);
        const T a = cv.U[cv.p], b = cv.U[cv.m - cv.p];
        const T du = (b - a) / T((double)(cv.closed ? ns : ns - 1));
        if (val(len) > 0.0) {
          smp[j].tx = Dx[1] / len;
          smp[j].ty = Dy[1] / len;
          const T along = len * du / T(pr->rho);
          if (val(along) > val(sg)) smp[j].sigma = along;
        }
      }
    }
    for (int k = 0; k < kap; ++k) out.push_back(smp[0]);
    for (int j = 0; j < ns; ++j) out.push_back(smp[j]);
    for (int k = 0; k < kap; ++k) out.push_back(smp[ns - 1]);
  } else {
    std::vector<T> bx, by;
    boundary_points(cv, ns, bx, by);
    const double h = pr->h;
    const T sig = T(pr->eta * h / pr->rho);                         // Eq. 6
    for (int iy = 0; iy < plan_row[P_NY]; ++iy)
      for (int ix = 0; ix < plan_row[P_NX]; ++ix) {
        if (need && !(*need)[out.size()]) {
          out.push_back(Gauss<T>{T(0.0), T(0.0), T(0.0), T(0.0), T(0.0), T(1.0), T(0.0)});
          continue;
        }
        const double qx = (plan_row[P_IX0] + ix + 0.5) * h, qy = (plan_row[P_IY0] + iy + 0.5) * h;
        const T z = T(pr->gamma / h) * sdf(qx, qy, bx, by);
        out.push_back(Gauss<T>{T(qx), T(qy), sig, o * sigmoid(z), sig, T(1.0), T(0.0)});   // Eq. 7
      }
  }
  (void)sc;
}

// Scene ranges of the Gaussian array (curves are grouped by scene).
std::vector<int64_t> scene_ranges(const or_curves* in, const int32_t* plan, int n_scenes) {
  std::vector<int64_t> r(2 * n_scenes, 0);
  std::vector<bool> seen(n_scenes, false);
  for (int c = 0; c < in->n_curves; ++c) {
    const int s = in->scene[c];
    const int64_t a = plan[P_STRIDE * c + P_GOFF], b = a + plan[P_STRIDE * c + P_COUNT];
    if (!seen[s]) { r[2 * s] = a; r[2 * s + 1] = b; seen[s] = true; }
    else { r[2 * s] = std::min(r[2 * s], a); r[2 * s + 1] = std::max(r[2 * s + 1], b); }
  }
  return r;
}

// Eq. 8 and 9 at one pixel centre, every Gaussian of the scene in front-to-back
// order (descending index: later curves are drawn on top).  alpha is clamped to
// alpha_max; the pixel stops once T < eps_T; what transmittance remains goes to
// the background.  Terms with alpha < e^-75 are skipped: they are below FP64
// resolution of every quantity they would be added to.  If `up` is given the
// adjoint of sum_c up_c I_c is added into adj[g][0..6] =
// (d/dmx, d/dmy, d/dsigma, d/dopacity, d/dcolour[0..2]).
// One composited (pixel, Gaussian) pair: the Gaussian, its alpha and G, the
// offset from its centre, and for a tangent-aligned Gaussian the offsets
// along (dp) and across (dq) the tangent.
// Per-Gaussian adjoint slots: mx, my, sigma, opacity, colour (3), sp, theta.
constexpr int NADJ = 9;

struct Hit { int64_t g; double a, G, dx, dy, d2, T, dp, dq; bool an; };

void composite_pixel(const or_curves* in, const or_params* pr, int C, const double* bg,
                     const double* mx, const double* my, const double* sg, const double* op,
                     const double* sp, const double* tdir, const int32_t* gcurve, int64_t g0, int64_t g1,
                     double px, double py, double* img, double* Tout, const double* up, double* adj,
                     double* adjabs) {
  std::vector<Hit> hits;
  double T = 1.0;
  double acc[3] = {0, 0, 0};
  for (int64_t g = g1 - 1; g >= g0; --g) {
    const double dx = px - mx[g], dy = py - my[g];
    const double d2 = dx * dx + dy * dy;
    const double s2 = sg[g] * sg[g];
    const bool an = sp && (in->flags[gcurve[g]] & F_ANISO);
    double G, dp = 0.0, dq = 0.0;
    if (!an) {
      // Eq. 9
      if (pr->cutoff > 0.0 && d2 > pr->cutoff * pr->cutoff * s2) continue;
      if (d2 > 150.0 * s2) continue;  // exp(-75): below FP64 resolution
      G = std::exp(-d2 / (2.0 * s2));
    } else {
      // Eq. 9 with the covariance R diag(sigma^2, sp^2) R^T, R the rotation
      // to the tangent t: exp(-(dp^2 / sigma^2 + dq^2 / sp^2) / 2), dp and dq
      // the offsets along t and along the normal n = (-t_y, t_x)
      const double tx = tdir[2 * g], ty = tdir[2 * g + 1];
      dp = dx * tx + dy * ty;
      dq = dy * tx - dx * ty;
      const double m2 = dp * dp / s2 + dq * dq / (sp[g] * sp[g]);
      if (pr->cutoff > 0.0 && m2 > pr->cutoff * pr->cutoff) continue;
      if (m2 > 150.0) continue;
      G = std::exp(-0.5 * m2);
    }
    const double a = std::min(pr->alpha_max, op[g] * G);
    const double* col = in->color + (size_t)C * gcurve[g];
    for (int k = 0; k < C; ++k) acc[k] += col[k] * a * T;
    if (up) hits.push_back(Hit{g, a, G, dx, dy, d2, T, dp, dq, an});
    T = T * (1.0 - a);
    if (T < pr->eps_T) break;
  }
  for (int k = 0; k < C; ++k) img[k] = acc[k] + T * bg[k];
  *Tout = T;
  if (!up) return;
  // dI/dalpha_i = c_i T_i - R_i / (1 - alpha_i), R_i = everything behind i
  // (later hits plus T_final bg).  R is built by a backward pass over hits.
  double R[3];
  for (int k = 0; k < C; ++k) R[k] = T * bg[k];
  for (int h = (int)hits.size() - 1; h >= 0; --h) {
    const Hit& e = hits[h];
    const double* col = in->color + (size_t)C * gcurve[e.g];
    double dLda = 0.0, sabs = 0.0;
    for (int k = 0; k < C; ++k) {
      dLda += up[k] * (col[k] * e.T - R[k] / (1.0 - e.a));
      adj[NADJ * e.g + 4 + k] += up[k] * e.a * e.T;
      // the magnitude of the terms dL/dalpha is formed from: the scale of
      // its rounding error in any evaluation order
      sabs += std::fabs(up[k]) * (std::fabs(col[k]) * e.T + std::fabs(R[k]) / (1.0 - e.a));
      if (adjabs) adjabs[NADJ * e.g + 4 + k] += std::fabs(up[k]) * e.a * e.T;
    }
    for (int k = 0; k < C; ++k) R[k] += col[k] * e.a * e.T;
    if (op[e.g] * e.G < pr->alpha_max) {          // clamp inactive
      const double s = sg[e.g];
      const double dLdG = dLda * op[e.g];
      double* A = adj + NADJ * e.g;
      A[3] += dLda * e.G;
      // partials of G: w.r.t. (mx, my, sigma) and, tangent-aligned, sp and the
      // tangent angle theta (t = (cos theta, sin theta))
      double pg[5];
      if (!e.an) {
        pg[0] = e.dx / (s * s);           // dG/dmx = G (x - mx) / s^2
        pg[1] = e.dy / (s * s);
        pg[2] = e.d2 / (s * s * s);
        pg[3] = pg[4] = 0.0;
      } else {
        const double q = sp[e.g], tx = tdir[2 * e.g], ty = tdir[2 * e.g + 1];
        pg[0] = e.dp * tx / (s * s) - e.dq * ty / (q * q);
        pg[1] = e.dp * ty / (s * s) + e.dq * tx / (q * q);
        pg[2] = e.dp * e.dp / (s * s * s);
        pg[3] = e.dq * e.dq / (q * q * q);
        pg[4] = e.dp * e.dq * (1.0 / (q * q) - 1.0 / (s * s));
      }
      A[0] += dLdG * e.G * pg[0];
      A[1] += dLdG * e.G * pg[1];
      A[2] += dLdG * e.G * pg[2];
      A[7] += dLdG * e.G * pg[3];
      A[8] += dLdG * e.G * pg[4];
      if (adjabs) {
        // the magnitudes of the terms each partial is formed from (for the
        // tangent-aligned form: its two axes' terms, and both inverse squares)
        double ab[5] = {std::fabs(pg[0]), std::fabs(pg[1]), pg[2], pg[3], std::fabs(pg[4])};
        if (e.an) {
          const double q = sp[e.g], s = sg[e.g], tx = tdir[2 * e.g], ty = tdir[2 * e.g + 1];
          ab[0] = std::fabs(e.dp * tx) / (s * s) + std::fabs(e.dq * ty) / (q * q);
          ab[1] = std::fabs(e.dp * ty) / (s * s) + std::fabs(e.dq * tx) / (q * q);
          ab[4] = std::fabs(e.dp * e.dq) * (1.0 / (q * q) + 1.0 / (s * s));
        }
        const double sG = sabs * op[e.g] * e.G;
        double* B = adjabs + NADJ * e.g;
        B[3] += sabs * e.G;
        B[0] += sG * ab[0];
        B[1] += sG * ab[1];
        B[2] += sG * ab[2];
        B[7] += sG * ab[3];
        B[8] += sG * ab[4];
      }
    }
  }
}

}  // namespace

namespace {

// ---------------------------------------------------------------------------
// Sec. 3.5: geometric regularisers.
// ---------------------------------------------------------------------------

// k-th u-derivative of N_{i,d} (The NURBS Book, Eq. 2.9):
//   N^(k)_{i,d} = d (N^(k-1)_{i,d-1} / (u_{i+d} - u_i) - N^(k-1)_{i+1,d-1} / (u_{i+d+1} - u_{i+1})),
// with 0/0 := 0 and N^(0)_{i,d} = N_{i,d} (so the derivatives are those of the
// span chosen by find_span: one-sided at knots).
template <class T>
T basis_deriv(const std::vector<T>& U, int i, int d, int k, const T& u, int span) {
  if (k == 0) return basis(U, i, d, u, span);
  if (d == 0) return T(0.0);
  T a(0.0), b(0.0);
  const T den1 = U[i + d] - U[i];
  if (val(den1) != 0.0) a = basis_deriv(U, i, d - 1, k - 1, u, span) / den1;
  const T den2 = U[i + d + 1] - U[i + 1];
  if (val(den2) != 0.0) b = basis_deriv(U, i + 1, d - 1, k - 1, u, span) / den2;
  return T((double)d) * (a - b);
}

// u-derivatives C^(k)(u), k = 0..r, of the planar rational curve (x, y):
// A^(k) = sum_i N^(k)_{i,p} w_i P_i and W^(k) = sum_i N^(k)_{i,p} w_i, then the
// rational Leibniz rule (The NURBS Book, Eq. 4.8)
//   C^(k) = (A^(k) - sum_{i=1..k} binom(k, i) W^(i) C^(k-i)) / W.
template <class T>
void curve_derivs(const Curve<T>& cv, const T& u, int span, int r, std::vector<T>& Dx, std::vector<T>& Dy) {
  std::vector<T> Ax(r + 1, T(0.0)), Ay(r + 1, T(0.0)), Wk(r + 1, T(0.0));
  for (int k = 0; k <= r; ++k)
    for (int i = span - cv.p; i <= span; ++i) {
      const T nw = basis_deriv(cv.U, i, cv.p, k, u, span) * cv.W[i];
      Ax[k] += nw * cv.X[i];
      Ay[k] += nw * cv.Y[i];
      Wk[k] += nw;
    }
  Dx.assign(r + 1, T(0.0));
  Dy.assign(r + 1, T(0.0));
  for (int k = 0; k <= r; ++k) {
    T vx = Ax[k], vy = Ay[k];
    double bin = 1.0;  // binom(k, i), built up over i
    for (int i = 1; i <= k; ++i) {
      bin = bin * (double)(k - i + 1) / (double)i;
      vx = vx - T(bin) * Wk[i] * Dx[k - i];
      vy = vy - T(bin) * Wk[i] * Dy[k - i];
    }
    Dx[k] = vx / Wk[0];
    Dy[k] = vy / Wk[0];
  }
}

// Penalty of Eq. 12: ReLU (kind 0) or softplus (kind 1).
inline double penalty(double x, int kind) {
  if (kind == 0) return x > 0.0 ? x : 0.0;
  return x > 0.0 ? x + std::log1p(std::exp(-x)) : std::log1p(std::exp(x));
}
inline Dual penalty(const Dual& x, int kind) {
  if (kind == 0) return x.v > 0.0 ? x : Dual(0.0, 0.0);
  return Dual(penalty(x.v, 1), x.d / (1.0 + std::exp(-x.v)));
}

// Regularisers of curve c at the parameters of its own samples:
//   lambda_bbox * sum_j [phi(b_min - C(u_j)) + phi(C(u_j) - b_max)] (both axes)
// + lambda_deriv / n_scene * (1 / (u_max - u_min)) int ||C^(r)||^2 du,
// the integral by the trapezoid rule on the open samples (both ends
// included) or the periodic rectangle rule on closed ones, and n_scene the
// number of curves in the curve's scene (the average over curves).
template <class T>
T curve_reg(const or_curves* in, const or_scenes* sc, const int32_t* row, int c, const or_reg* rg,
            double n_scene, int seed_kind, int seed_index) {
  const int ns = row[P_NSAMP];
  if (ns <= 0) return T(0.0);
  const Curve<T> cv = build_curve<T>(in, c, seed_kind, seed_index);
  const int s = in->scene[c];
  double b0x = 0.0, b0y = 0.0, b1x = sc->hw[2 * s + 1], b1y = sc->hw[2 * s];
  if (rg->bbox) {
    b0x = rg->bbox[4 * s]; b0y = rg->bbox[4 * s + 1]; b1x = rg->bbox[4 * s + 2]; b1y = rg->bbox[4 * s + 3];
  }
  T loss(0.0);
  std::vector<T> Dx, Dy;
  for (int j = 0; j < ns; ++j) {
    const T u = sample_u(cv, j, ns, cv.closed);
    const int span = find_span(cv, val(u));
    if (rg->bbox_weight != 0.0) {
      T pt[3];
      curve_point(cv, u, span, pt);
      const T pen = penalty(T(b0x) - pt[0], rg->bbox_kind) + penalty(pt[0] - T(b1x), rg->bbox_kind) +
                    penalty(T(b0y) - pt[1], rg->bbox_kind) + penalty(pt[1] - T(b1y), rg->bbox_kind);
      loss += T(rg->bbox_weight) * pen;
    }
    if (rg->deriv_weight != 0.0) {
      double wq;
      if (cv.closed) wq = 1.0 / ns;
      else wq = (j == 0 || j == ns - 1) ? 0.5 / (ns - 1) : 1.0 / (ns - 1);
      curve_derivs(cv, u, span, rg->deriv_order, Dx, Dy);
      const int r = rg->deriv_order;
      loss += T(rg->deriv_weight / n_scene * wq) * (Dx[r] * Dx[r] + Dy[r] * Dy[r]);
    }
  }
  return loss;
}

std::vector<double> curves_per_scene(const or_curves* in, const or_scenes* sc) {
  std::vector<double> n(sc->n_scenes, 0.0);
  for (int c = 0; c < in->n_curves; ++c) n[in->scene[c]] += 1.0;
  return n;
}

}  // namespace

extern "C" {

// Plan: per curve {count, n_samples, ix0, iy0, nx, ny, g_offset, flags}
// (flags: 1 = delta L within 1e-9 of an integer, 2 = values outside the
// domain of Sec. 3.1, the curve then has no Gaussians) and the arc length L.
// Returns the total number of Gaussians.
int64_t or_plan(const or_curves* in, const or_scenes* sc, const or_params* pr, int32_t* plan, double* L) {
  const int N = in->n_curves;
#pragma omp parallel for schedule(dynamic, 1)
  for (int c = 0; c < N; ++c) {
    int32_t* row = plan + P_STRIDE * c;
    for (int k = 0; k < P_STRIDE; ++k) row[k] = 0;
    // values outside the domain of Sec. 3.1, or a tangent-aligned fill (the
    // variant concerns contour samples only): no Gaussians, flag 2
    if (!values_in_domain(in, c) || ((in->flags[c] & F_ANISO) && (in->flags[c] & F_FILLED))) {
      L[c] = 0.0;
      row[P_FLAG] = 2;
      continue;
    }
    const Curve<double> cv = build_curve<double>(in, c, S_NONE, 0);
    const SceneGeom geo = scene_geom(sc, pr, in->scene[c]);
    const double len = arc_length(cv, geo.n_L);
    L[c] = len;
    int flag = 0;
    if (!cv.filled) {
      const double delta = (in->flags[c] & F_ANISO) ? pr->delta_a : pr->delta_c;
      const int M = count_rule(delta, len, cv.closed ? 3 : 2, &flag);
      row[P_NSAMP] = M;
      row[P_COUNT] = cv.closed ? M : M + 2 * pr->kappa;
    } else {
      const int nb = count_rule(pr->delta_b, len, 3, &flag);
      row[P_NSAMP] = nb;
      std::vector<double> bx, by;
      boundary_points(cv, nb, bx, by);
      int win[4];
      fill_window(bx, by, pr->fill_pad, pr->h, geo.W, geo.H, win);
      row[P_IX0] = win[0]; row[P_IY0] = win[1]; row[P_NX] = win[2]; row[P_NY] = win[3];
      row[P_COUNT] = win[2] * win[3];
    }
    row[P_FLAG] = flag;
  }
  int64_t off = 0;
  for (int c = 0; c < N; ++c) {
    plan[P_STRIDE * c + P_GOFF] = (int32_t)off;
    off += plan[P_STRIDE * c + P_COUNT];
  }
  return off;
}

// Gaussians for a plan (frozen or fresh): centres, sigma, opacity, owning
// curve, index within the curve.
int64_t or_gaussians(const or_curves* in, const or_scenes* sc, const or_params* pr, const int32_t* plan,
                     double* mu, double* sigma, double* opacity, int32_t* curve, int32_t* local, double* sp,
                     double* tdir) {
  const int N = in->n_curves;
#pragma omp parallel for schedule(dynamic, 1)
  for (int c = 0; c < N; ++c) {
    std::vector<Gauss<double>> gs;
    curve_gaussians<double>(in, sc, pr, c, plan + P_STRIDE * c, S_NONE, 0, gs);
    const int64_t g0 = plan[P_STRIDE * c + P_GOFF];
    for (size_t j = 0; j < gs.size(); ++j) {
      mu[2 * (g0 + j)] = gs[j].mx;
      mu[2 * (g0 + j) + 1] = gs[j].my;
      sigma[g0 + j] = gs[j].sigma;
      opacity[g0 + j] = gs[j].opacity;
      curve[g0 + j] = c;
      local[g0 + j] = (int32_t)j;
      if (sp) sp[g0 + j] = gs[j].sp;
      if (tdir) {
        tdir[2 * (g0 + j)] = gs[j].tx;
        tdir[2 * (g0 + j) + 1] = gs[j].ty;
      }
    }
  }
  int64_t total = 0;
  for (int c = 0; c < N; ++c) total += plan[P_STRIDE * c + P_COUNT];
  return total;
}

// Sec. 3.4 tile binning, decided in FP32 exactly as the rasteriser decides it:
// centre m = fl32(mx), radius r = fl32(k_sigma) * fl32(sigma), conservative
// interval [(m - r) - 1, (m + r) + 1] per axis, tile = floor(x / tile),
// clamped to the scene's tile grid.  Pairs (global tile key, g) are emitted in
// ascending g and stably sorted by key.  ranges[2 t] .. ranges[2 t + 1] is
// tile t's slice of idx.  Returns the number of pairs (idx is written only if
// the capacity allows).
int64_t or_bin(int64_t G, const double* mu, const double* sigma, const int32_t* gscene,
               const or_scenes* sc, int32_t tile, float k_sigma, int32_t* ranges, int32_t* idx, int64_t cap) {
  std::vector<int64_t> tile_off(sc->n_scenes + 1, 0);
  std::vector<int> tiles_x(sc->n_scenes), tiles_y(sc->n_scenes);
  for (int s = 0; s < sc->n_scenes; ++s) {
    tiles_y[s] = (sc->hw[2 * s] + tile - 1) / tile;
    tiles_x[s] = (sc->hw[2 * s + 1] + tile - 1) / tile;
    tile_off[s + 1] = tile_off[s] + (int64_t)tiles_x[s] * tiles_y[s];
  }
  const float inv = 1.0f / (float)tile;
  std::vector<std::pair<int64_t, int64_t>> pairs;
  for (int64_t g = 0; g < G; ++g) {
    const int s = gscene[g];
    const float mx = (float)mu[2 * g], my = (float)mu[2 * g + 1];
    const float r = k_sigma * (float)sigma[g];
    const float xl = (mx - r) - 1.0f, xh = (mx + r) + 1.0f;
    const float yl = (my - r) - 1.0f, yh = (my + r) + 1.0f;
    if (!(xl == xl) || !(xh == xh) || !(yl == yl) || !(yh == yh)) continue;
    const float fx0 = std::max(0.0f, std::floor(xl * inv)), fx1 = std::min((float)(tiles_x[s] - 1), std::floor(xh * inv));
    const float fy0 = std::max(0.0f, std::floor(yl * inv)), fy1 = std::min((float)(tiles_y[s] - 1), std::floor(yh * inv));
    if (fx0 > fx1 || fy0 > fy1) continue;
    for (int ty = (int)fy0; ty <= (int)fy1; ++ty)
      for (int tx = (int)fx0; tx <= (int)fx1; ++tx)
        pairs.push_back({tile_off[s] + (int64_t)ty * tiles_x[s] + tx, g});
  }
  std::stable_sort(pairs.begin(), pairs.end(),
                   [](const std::pair<int64_t, int64_t>& a, const std::pair<int64_t, int64_t>& b) { return a.first < b.first; });
  const int64_t n_tiles = tile_off[sc->n_scenes];
  for (int64_t t = 0; t < 2 * n_tiles; ++t) ranges[t] = 0;
  const int64_t n = (int64_t)pairs.size();
  if (n <= cap) {
    for (int64_t i = 0; i < n; ++i) idx[i] = (int32_t)pairs[i].second;
    for (int64_t i = 0; i < n; ++i) {
      const int64_t t = pairs[i].first;
      if (i == 0 || pairs[i - 1].first != t) ranges[2 * t] = (int32_t)i;
      if (i == n - 1 || pairs[i + 1].first != t) ranges[2 * t + 1] = (int32_t)(i + 1);
    }
  }
  return n;
}

// Compositing (Eq. 8-9).  pix == NULL: every pixel of every scene; image
// layout per scene [C][H][W] concatenated, T_final [H][W] concatenated.
// Otherwise npix pixels given as (scene, y, x) triples, outputs [npix][C] and
// [npix].  If up != NULL (same layout as img), adj [G][9] receives the
// adjoint of sum(up * I) with respect to every Gaussian (mx, my, sigma,
// opacity, colour (3), sp, theta; it is zeroed first).  sp and tdir ([G],
// [G][2]) describe tangent-aligned Gaussians (NULL: every Gaussian isotropic).
int or_composite(const or_curves* in, const or_scenes* sc, const or_params* pr, const int32_t* plan,
                 const double* mu, const double* sigma, const double* opacity, const double* sp,
                 const double* tdir, const int32_t* gcurve, int64_t G, int64_t npix, const int32_t* pix,
                 double* img, double* Tfin, const double* up, double* adj, double* adjabs) {
  const int C = in->channels;
  const std::vector<int64_t> sr = scene_ranges(in, plan, sc->n_scenes);
  std::vector<double> mx(G), my(G);
  for (int64_t g = 0; g < G; ++g) { mx[g] = mu[2 * g]; my[g] = mu[2 * g + 1]; }
  // pixel list
  std::vector<int32_t> plist;
  std::vector<int64_t> img_off, t_off;
  if (!pix) {
    int64_t io = 0, to = 0;
    for (int s = 0; s < sc->n_scenes; ++s) {
      const int H = sc->hw[2 * s], W = sc->hw[2 * s + 1];
      for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
          plist.push_back(s); plist.push_back(y); plist.push_back(x);
          img_off.push_back(io + (int64_t)y * W + x);     // channel stride H*W
          t_off.push_back(to + (int64_t)y * W + x);
        }
      io += (int64_t)C * H * W;
      to += (int64_t)H * W;
    }
    npix = (int64_t)t_off.size();
    pix = plist.data();
  }
  int nthreads = 1;
#ifdef _OPENMP
#pragma omp parallel
  {
#pragma omp single
    nthreads = omp_get_num_threads();
  }
#endif
  std::vector<std::vector<double>> adj_t, abs_t;
  if (up) adj_t.assign(nthreads, std::vector<double>());
  if (up && adjabs) abs_t.assign(nthreads, std::vector<double>());
#pragma omp parallel
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    double* my_adj = nullptr;
    double* my_abs = nullptr;
    if (up) { adj_t[tid].assign((size_t)NADJ * G, 0.0); my_adj = adj_t[tid].data(); }
    if (up && adjabs) { abs_t[tid].assign((size_t)NADJ * G, 0.0); my_abs = abs_t[tid].data(); }
#pragma omp for schedule(dynamic, 16)
    for (int64_t q = 0; q < npix; ++q) {
      const int s = pix[3 * q], y = pix[3 * q + 1], x = pix[3 * q + 2];
      const int H = sc->hw[2 * s], W = sc->hw[2 * s + 1];
      double v[3], T, u[3] = {0, 0, 0};
      const bool full = !img_off.empty();
      if (up) {
        for (int k = 0; k < C; ++k)
          u[k] = full ? up[img_off[q] + (int64_t)k * H * W] : up[(int64_t)C * q + k];
      }
      composite_pixel(in, pr, C, sc->bg + (size_t)C * s, mx.data(), my.data(), sigma, opacity, sp, tdir, gcurve,
                      sr[2 * s], sr[2 * s + 1], x + 0.5, y + 0.5, v, &T, up ? u : nullptr, my_adj, my_abs);
      for (int k = 0; k < C; ++k) {
        if (full) img[img_off[q] + (int64_t)k * H * W] = v[k];
        else img[(int64_t)C * q + k] = v[k];
      }
      Tfin[full ? t_off[q] : q] = T;
    }
  }
  if (up) {
    for (int64_t i = 0; i < NADJ * G; ++i) {
      double s = 0.0, a = 0.0;
      for (int t = 0; t < nthreads; ++t) s += adj_t[t][i];
      adj[i] = s;
      if (adjabs) {
        for (int t = 0; t < nthreads; ++t) a += abs_t[t][i];
        adjabs[i] = a;
      }
    }
  }
  return 0;
}

// Gradient of the loss with respect to one curve parameter, from the
// per-Gaussian adjoints: sum_g adj_g . d(gaussian_g)/d(theta), with the
// derivative taken by forward-mode dual numbers over the frozen plan.
// kind: 1 key x, 2 key y, 3 key weight, 4 key width, 5 tau, 6 opacity,
// 7 + ch: colour channel ch.  index is local to the curve.
// With adjabs (the per-Gaussian sums of absolute terms from or_composite),
// *scale receives sum_g adjabs_g . |d(gaussian_g)/d(theta)|: the magnitude of
// the terms the gradient sums, which bounds the rounding error of any
// evaluation of it relative to FP32's unit roundoff.
static double param_grad_one(const or_curves* in, const or_scenes* sc, const or_params* pr, const int32_t* plan,
                             const double* adj, const double* adjabs, int c, int kind, int index, double* scale) {
  const int32_t* row = plan + P_STRIDE * c;
  const int64_t g0 = row[P_GOFF];
  if (kind >= 7) {
    double s = 0.0, sa = 0.0;
    for (int j = 0; j < row[P_COUNT]; ++j) {
      s += adj[NADJ * (g0 + j) + 4 + (kind - 7)];
      if (adjabs) sa += adjabs[NADJ * (g0 + j) + 4 + (kind - 7)];
    }
    if (scale) *scale = sa;
    return s;
  }
  std::vector<char> need(row[P_COUNT]);
  for (int j = 0; j < row[P_COUNT]; ++j) {
    const double* a = adj + NADJ * (g0 + j);
    need[j] = (a[0] != 0.0 || a[1] != 0.0 || a[2] != 0.0 || a[3] != 0.0 || a[7] != 0.0 || a[8] != 0.0);
  }
  std::vector<Gauss<Dual>> gs;
  curve_gaussians<Dual>(in, sc, pr, c, row, kind, index, gs, &need);
  double s = 0.0, sa = 0.0;
  for (size_t j = 0; j < gs.size(); ++j) {
    const double* a = adj + NADJ * (g0 + j);
    // d theta from the tangent's derivative: t = (cos theta, sin theta)
    const double dth = gs[j].tx.v * gs[j].ty.d - gs[j].ty.v * gs[j].tx.d;
    s += a[0] * gs[j].mx.d + a[1] * gs[j].my.d + a[2] * gs[j].sigma.d + a[3] * gs[j].opacity.d +
         a[7] * gs[j].sp.d + a[8] * dth;
    if (adjabs) {
      const double* b = adjabs + NADJ * (g0 + j);
      sa += b[0] * std::fabs(gs[j].mx.d) + b[1] * std::fabs(gs[j].my.d) + b[2] * std::fabs(gs[j].sigma.d) +
            b[3] * std::fabs(gs[j].opacity.d) + b[7] * std::fabs(gs[j].sp.d) + b[8] * std::fabs(dth);
    }
  }
  if (scale) *scale = sa;
  return s;
}

// Selected gradient components: seeds [n][3] = (curve, kind, index); with
// adjabs also their error scales (see param_grad_one) into scale [n].
int or_param_grad_seeds(const or_curves* in, const or_scenes* sc, const or_params* pr, const int32_t* plan,
                        const double* adj, int64_t n, const int32_t* seeds, double* out) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n; ++i)
    out[i] = param_grad_one(in, sc, pr, plan, adj, nullptr, seeds[3 * i], seeds[3 * i + 1], seeds[3 * i + 2],
                            nullptr);
  return 0;
}

int or_param_grad_seeds_scaled(const or_curves* in, const or_scenes* sc, const or_params* pr, const int32_t* plan,
                               const double* adj, const double* adjabs, int64_t n, const int32_t* seeds, double* out,
                               double* scale) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n; ++i)
    out[i] = param_grad_one(in, sc, pr, plan, adj, adjabs, seeds[3 * i], seeds[3 * i + 1], seeds[3 * i + 2],
                            scale + i);
  return 0;
}

// Every gradient component, written in the layout of the inputs.
int or_param_grad_full(const or_curves* in, const or_scenes* sc, const or_params* pr, const int32_t* plan,
                       const double* adj, double* g_key_xy, double* g_key_w, double* g_key_s, double* g_tau,
                       double* g_color, double* g_opacity, const double* adjabs, double* s_key_xy, double* s_key_w,
                       double* s_key_s, double* s_tau, double* s_color, double* s_opacity) {
  const int N = in->n_curves, C = in->channels;
  std::vector<int32_t> seeds;
  std::vector<int64_t> off;   // offset of each seed's output in its group
  std::vector<int> grp;       // group: 0 key_xy, 1 key_w, 2 key_s, 3 tau, 4 color, 5 opacity
  auto add = [&](int c, int kind, int idx, int g, int64_t o) {
    seeds.insert(seeds.end(), {c, kind, idx});
    grp.push_back(g);
    off.push_back(o);
  };
  for (int c = 0; c < N; ++c) {
    const int k0 = in->key_off[c], nk = in->key_off[c + 1] - k0;
    const int t0 = in->tau_off[c], nt = in->tau_off[c + 1] - t0;
    for (int k = 0; k < nk; ++k) {
      add(c, S_KEY_X, k, 0, 2 * (k0 + k));
      add(c, S_KEY_Y, k, 0, 2 * (k0 + k) + 1);
      add(c, S_KEY_W, k, 1, k0 + k);
      add(c, S_KEY_S, k, 2, k0 + k);
    }
    for (int t = 0; t < nt; ++t) add(c, S_TAU, t, 3, t0 + t);
    add(c, S_OPACITY, 0, 5, c);
    for (int ch = 0; ch < C; ++ch) add(c, 7 + ch, 0, 4, C * c + ch);
  }
  const int64_t n = (int64_t)grp.size();
  std::vector<double> out(n), sc_out(n);
  or_param_grad_seeds_scaled(in, sc, pr, plan, adj, adjabs, n, seeds.data(), out.data(), sc_out.data());
  double* gdst[6] = {g_key_xy, g_key_w, g_key_s, g_tau, g_color, g_opacity};
  double* sdst[6] = {s_key_xy, s_key_w, s_key_s, s_tau, s_color, s_opacity};
  for (int64_t i = 0; i < n; ++i) {
    gdst[grp[i]][off[i]] = out[i];
    if (adjabs && sdst[grp[i]]) sdst[grp[i]][off[i]] = sc_out[i];
  }
  return 0;
}

// Regularisers (Sec. 3.5, Eq. 11 and Eq. 12) summed over all curves for the
// given plan, and their derivative for each seed [n][3] = (curve, kind,
// index); colour and opacity do not enter them.
double or_reg_loss(const or_curves* in, const or_scenes* sc, const or_params* pr, const int32_t* plan,
                   const or_reg* rg, int64_t n, const int32_t* seeds, double* grad) {
  (void)pr;
  const std::vector<double> nsc = curves_per_scene(in, sc);
  double total = 0.0;
  for (int c = 0; c < in->n_curves; ++c)
    total += curve_reg<double>(in, sc, plan + P_STRIDE * c, c, rg, nsc[in->scene[c]], S_NONE, 0);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n; ++i) {
    const int c = seeds[3 * i], kind = seeds[3 * i + 1], idx = seeds[3 * i + 2];
    if (kind < S_KEY_X || kind > S_TAU) {
      grad[i] = 0.0;
      continue;
    }
    grad[i] = curve_reg<Dual>(in, sc, plan + P_STRIDE * c, c, rg, nsc[in->scene[c]], kind, idx).d;
  }
  return total;
}

// The regularisers' value and every gradient component in the layout of the
// inputs (zero for colour and opacity).
double or_reg_grad_full(const or_curves* in, const or_scenes* sc, const or_params* pr, const int32_t* plan,
                        const or_reg* rg, double* g_key_xy, double* g_key_w, double* g_key_s, double* g_tau) {
  std::vector<int32_t> seeds;
  std::vector<double*> dst;
  for (int c = 0; c < in->n_curves; ++c) {
    const int k0 = in->key_off[c], nk = in->key_off[c + 1] - k0;
    const int t0 = in->tau_off[c], nt = in->tau_off[c + 1] - t0;
    for (int k = 0; k < nk; ++k) {
      seeds.insert(seeds.end(), {c, S_KEY_X, k}); dst.push_back(g_key_xy + 2 * (k0 + k));
      seeds.insert(seeds.end(), {c, S_KEY_Y, k}); dst.push_back(g_key_xy + 2 * (k0 + k) + 1);
      seeds.insert(seeds.end(), {c, S_KEY_W, k}); dst.push_back(g_key_w + k0 + k);
      seeds.insert(seeds.end(), {c, S_KEY_S, k}); dst.push_back(g_key_s + k0 + k);
    }
    for (int t = 0; t < nt; ++t) { seeds.insert(seeds.end(), {c, S_TAU, t}); dst.push_back(g_tau + t0 + t); }
  }
  const int64_t n = (int64_t)dst.size();
  std::vector<double> out(n);
  const double total = or_reg_loss(in, sc, pr, plan, rg, n, seeds.data(), out.data());
  for (int64_t i = 0; i < n; ++i) *dst[i] = out[i];
  return total;
}

// Distance-weighted image loss (Sec. 4.2; the weights of LIVE, Ma et al.
// 2022): for every pixel centre q of a scene, d(q) = distance to the nearest
// boundary segment of the scene's selected filled curves (their N_b-point
// closed polylines of Sec. 3.3; sel == NULL selects every filled curve),
// w(q) = max(0, tau - d(q)), normalised to sum 1 over the scene (all zero if
// no pixel is within tau); L = sum_q w(q) (1/C) sum_c (I_c(q) - I*_c(q))^2,
// the weights held constant.  Writes dL/dI (image layout) and d (per pixel,
// +inf where no curve is selected) and returns L summed over the scenes.
double or_udf_loss(const or_curves* in, const or_scenes* sc, const or_params* pr, const int32_t* plan,
                   const int32_t* sel, double tau, const double* img, const double* tgt, double* dL, double* dist) {
  const int C = in->channels;
  std::vector<std::vector<double>> bxs(in->n_curves), bys(in->n_curves);
  std::vector<char> use(in->n_curves, 0);
  for (int c = 0; c < in->n_curves; ++c) {
    const int32_t* row = plan + P_STRIDE * c;
    if (!(in->flags[c] & F_FILLED) || row[P_NSAMP] <= 0 || (sel && !sel[c])) continue;
    use[c] = 1;
    boundary_points(build_curve<double>(in, c, S_NONE, 0), row[P_NSAMP], bxs[c], bys[c]);
  }
  double total = 0.0;
  int64_t pix_off = 0;
  for (int s = 0; s < sc->n_scenes; ++s) {
    const int H = sc->hw[2 * s], W = sc->hw[2 * s + 1];
    const int64_t plane = (int64_t)H * W;
    std::vector<double> wq(plane, 0.0);
#pragma omp parallel for schedule(dynamic, 4)
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        const double qx = x + 0.5, qy = y + 0.5;
        double d = INFINITY;
        for (int c = 0; c < in->n_curves; ++c) {
          if (!use[c] || in->scene[c] != s) continue;
          const std::vector<double>& bx = bxs[c];
          const std::vector<double>& by = bys[c];
          const size_t n = bx.size();
          for (size_t i = 0; i < n; ++i) {
            const size_t k = (i + 1) % n;
            d = std::min(d, seg_dist(qx, qy, bx[i], by[i], bx[k], by[k]));
          }
        }
        dist[pix_off + (int64_t)y * W + x] = d;
        wq[(int64_t)y * W + x] = std::max(0.0, tau - d);
      }
    double sum = 0.0;
    for (int64_t i = 0; i < plane; ++i) sum += wq[i];
    for (int64_t i = 0; i < plane; ++i) {
      const double wn = sum > 0.0 ? wq[i] / sum : 0.0;
      for (int ch = 0; ch < C; ++ch) {
        const int64_t k = pix_off * C + ch * plane + i;
        const double e = img[k] - tgt[k];
        total += wn * e * e / C;
        dL[k] = 2.0 * wn * e / C;
      }
    }
    pix_off += plane;
  }
  (void)pr;
  return total;
}

// ---------------------------------------------------------------------------
// Single-curve geometry, for the closed-form tests.
// ---------------------------------------------------------------------------
static or_curves one_curve(int p, int closed, int nk, int nt, const double* key_xy, const double* key_w,
                           const double* key_s, const double* tau, int32_t meta[6], double* dummy) {
  meta[0] = 0; meta[1] = p; meta[2] = closed ? F_CLOSED : 0; meta[3] = 0; meta[4] = nk; meta[5] = nt;
  or_curves c;
  c.n_curves = 1; c.channels = 1;
  c.scene = meta; c.degree = meta + 1; c.flags = meta + 2;
  static thread_local int32_t ko[2], to[2];
  ko[0] = 0; ko[1] = nk; to[0] = 0; to[1] = nt;
  c.key_off = ko; c.tau_off = to;
  c.key_xy = key_xy; c.key_w = key_w; c.key_s = key_s; c.tau = tau;
  c.color = dummy; c.opacity = dummy;
  return c;
}

// Knot vector of one curve; returns m + 1 (the number of knots).
int or_curve_knots(int p, int closed, int nk, int nt, const double* tau, double* U) {
  std::vector<double> xy(2 * nk, 0.0), w(nk, 1.0), s(nk, 1.0);
  int32_t meta[6];
  double dummy[4] = {0, 0, 0, 0};
  const or_curves c = one_curve(p, closed, nk, nt, xy.data(), w.data(), s.data(), tau, meta, dummy);
  const Curve<double> cv = build_curve<double>(&c, 0, S_NONE, 0);
  for (int k = 0; k <= cv.m; ++k) U[k] = cv.U[k];
  return cv.m + 1;
}

// Curve point and u-derivative at parameters u = a + t (b - a), t in [0, 1]
// (t = 1 gives b exactly): out [n][6] = (x, y, s, dx/du, dy/du, ds/du).
// full != 0 sums Eq. 1 over all control points instead of the span.
int or_curve_eval(int p, int closed, int nk, int nt, const double* key_xy, const double* key_w,
                  const double* key_s, const double* tau, int n, const double* t, int full, double* out) {
  int32_t meta[6];
  double dummy[4] = {0, 0, 0, 0};
  const or_curves c = one_curve(p, closed, nk, nt, key_xy, key_w, key_s, tau, meta, dummy);
  const Curve<double> cv = build_curve<double>(&c, 0, S_NONE, 0);
  const double a = dom_lo(cv), b = dom_hi(cv);
  for (int i = 0; i < n; ++i) {
    const double u = t[i] >= 1.0 ? b : a + t[i] * (b - a);
    const int span = find_span(cv, u);
    double pt[3], d[3];
    curve_point(cv, u, span, pt, full != 0);
    curve_deriv(cv, std::vector<Dual>(cv.U.begin(), cv.U.end()), u, span, d, full != 0);
    for (int k = 0; k < 3; ++k) { out[6 * i + k] = pt[k]; out[6 * i + 3 + k] = d[k]; }
  }
  return 0;
}

// All basis functions N_{i,p}(u), i = 0..m-p-1, and their u-derivatives, on
// an arbitrary non-decreasing knot vector U[0..m].
int or_basis_all(int m, int p, const double* Uin, double u, double* N, double* dN) {
  Curve<double> cv;
  cv.p = p; cv.m = m; cv.U.assign(Uin, Uin + m + 1);
  const int span = find_span(cv, u);
  std::vector<Dual> U(cv.U.begin(), cv.U.end());
  for (int i = 0; i < m - p; ++i) {
    const Dual n = basis(U, i, p, Dual(u, 1.0), span);
    N[i] = n.v;
    dN[i] = n.d;
  }
  return span;
}

double or_arc_length(int p, int closed, int nk, int nt, const double* key_xy, const double* key_w,
                     const double* key_s, const double* tau, int n_L) {
  int32_t meta[6];
  double dummy[4] = {0, 0, 0, 0};
  const or_curves c = one_curve(p, closed, nk, nt, key_xy, key_w, key_s, tau, meta, dummy);
  return arc_length(build_curve<double>(&c, 0, S_NONE, 0), n_L);
}

// u-derivatives of order 0..r of the planar curve at u = a + t (b - a):
// out [n][r + 1][2].
int or_curve_derivs(int p, int closed, int nk, int nt, const double* key_xy, const double* key_w,
                    const double* key_s, const double* tau, int n, const double* t, int r, double* out) {
  int32_t meta[6];
  double dummy[4] = {0, 0, 0, 0};
  const or_curves c = one_curve(p, closed, nk, nt, key_xy, key_w, key_s, tau, meta, dummy);
  const Curve<double> cv = build_curve<double>(&c, 0, S_NONE, 0);
  const double a = dom_lo(cv), b = dom_hi(cv);
  std::vector<double> Dx, Dy;
  for (int i = 0; i < n; ++i) {
    const double u = t[i] >= 1.0 ? b : a + t[i] * (b - a);
    curve_derivs(cv, u, find_span(cv, u), r, Dx, Dy);
    for (int k = 0; k <= r; ++k) {
      out[2 * ((r + 1) * i + k)] = Dx[k];
      out[2 * ((r + 1) * i + k) + 1] = Dy[k];
    }
  }
  return 0;
}

// Signed distance at q to the closed polyline b[n][2]: out = (d, wn, sdf).
int or_sdf(int n, const double* b, double qx, double qy, double* out) {
  std::vector<double> bx(n), by(n);
  for (int i = 0; i < n; ++i) { bx[i] = b[2 * i]; by[i] = b[2 * i + 1]; }
  const double s = sdf(qx, qy, bx, by);
  out[0] = std::fabs(s);
  out[1] = winding(qx, qy, bx, by);
  out[2] = s;
  return 0;
}

// Eq. 14: cosine grid-step annealing, clamped outside (t_b, t_e).
double or_anneal(double t, double T, double hmax, double hmin, double tb, double te) {
  double phi = (t / T - tb) / (te - tb);
  if (phi < 0.0) phi = 0.0;
  if (phi > 1.0) phi = 1.0;
  return hmax + (hmin - hmax) * (1.0 + std::cos(M_PI * (1.0 - phi))) / 2.0;
}

int or_num_threads(void) {
  int n = 1;
#ifdef _OPENMP
  n = omp_get_max_threads();
#endif
  return n;
}

}  // extern "C"
