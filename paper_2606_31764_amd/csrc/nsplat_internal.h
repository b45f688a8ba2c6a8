// Internal declarations of the gfx950 NURBS Splatting library: the Gaussian
// record, the workspace carve-out, scene table, and the device-side NURBS
// helpers (span search, Cox-de Boor basis with first derivative, curve point).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nsplat.h"

namespace nsp {

constexpr int MAXP = NSPLAT_MAX_DEGREE;
constexpr int KNOT_PAD = 2 * MAXP + 1;  // knots of curve c start at tau_off[c] + c * KNOT_PAD
constexpr int CP_PAD = MAXP;            // control points of curve c start at key_off[c] + c * CP_PAD
constexpr double LOG2E = 1.4426950408889634074;
constexpr double LN2 = 0.69314718055994530942;
constexpr int SCAN_ITEMS = 4096;        // elements per block in the device-wide scans
constexpr int SORT_ITEMS = 4096;        // elements per block in a radix pass
constexpr int RADIX_BITS_MAX = 10;      // widest radix digit
constexpr int RADIX_MAX = 1 << RADIX_BITS_MAX;
constexpr int FB_ITEMS = 4096;          // Gaussians per block of the one-digit binning (bin.hip)
constexpr int MAX_BATCH = 256;          // LDS depth limit of the blend kernels
constexpr int N_WS = 29;                // workspace entries

// One Gaussian (32 bytes).  The centre is kept in FP64 so that the blend can
// form exact tile-local FP32 coordinates (a fl32 absolute centre is off by up
// to half an ulp: 3e-5 px at 512 px, too coarse for a 1e-5 image tolerance).
struct __align__(16) Gauss {
  double mx, my;
  float sigma, opacity;
  int32_t curve, local;
};
static_assert(sizeof(Gauss) == 32, "Gaussian record must be 32 bytes");

struct SceneTab {
  int32_t H, W, tiles_x, tiles_y, tile_off, pix_off, n_L;
  int32_t fills;  // 1: a curve of the scene is filled (set by nsplat_bin at 32 x 32 tiles, see adj_blocks)
};

enum { P_COUNT = 0, P_NSAMP, P_IX0, P_IY0, P_NX, P_NY, P_GOFF, P_BOFF, P_FLAGS, P_STRIDE };

// Device pointers carved out of the caller's workspace.
struct Work {
  double* knots;       // [n_taus + n_curves * KNOT_PAD]
  double* L;           // [n_curves]
  int32_t* goff;       // [n_curves + 1]
  double2* bpts;       // [caps.boundary]
  SceneTab* scenes;    // [n_scenes + 1]
  uint32_t* gcnt;      // [caps.gauss + 1] pair counts, then their offsets
  uint32_t* keys0;     // [caps.pairs]
  uint32_t* keys1;     // [caps.pairs]
  uint32_t* vals1;     // [caps.pairs]
  uint32_t* hist;      // radix digit counts [RADIX_MAX][sort_blocks], or the one-digit binning's [RADIX_MAX + 1][blocks]
  uint32_t* scan_tmp;  // [scan_blocks + 1]
  float* ggrad;        // [caps.gauss][4] per-Gaussian adjoints (d/dmx, d/dmy, d/dsigma, d/dopacity)
  double* gcp;         // [(n_keys + n_curves * CP_PAD)][4] control-point adjoints (x, y, w, s)
  double* gknot;       // [n_taus + n_curves * KNOT_PAD]
  double* gcurve;      // [n_curves][4] (opacity, colour 0..2)
  double2* gb;         // [caps.boundary] boundary-point adjoints
  int32_t* queue;      // [64] work-queue counters of the persistent kernels (0-3), Gaussians by kind (Q_*)
  int32_t* aux;        // [caps.gauss] fill Gaussians: nearest boundary segment, sign in bit 31
  double4* cbox;       // [caps.boundary / SDF_CHUNK + 2 * n_curves + 2] fill SDF chunk boxes
  int32_t* order;      // [tiles at the smallest tile size] tiles by decreasing list length
  int32_t* obin;       // [64] list-length class counts, then their offsets
  double* sacc;        // [n_scenes + 1] per-scene sums (distance-weighted loss)
  int32_t* ck_off;     // [tiles at the smallest tile size + 1] first checkpoint of each tile (scan)
  int32_t* item_off;   // [tiles at the smallest tile size + 1] first adjoint item of each tile in blend order (scan)
  float* ckbuf;        // [caps.pairs / CK_MIN + 1][4][32 * 32] forward state at chunk boundaries: T, and
                       // the colour of everything behind the boundary (per channel)
  float4* gcol;        // [caps.gauss] colour of each Gaussian's curve, and its kind (Kind below)
  float4* gaux;        // [caps.gauss] tangent-aligned Gaussians: tangent (x, y), axis across the curve
  double* segs;        // [caps.boundary + (SDF_CHUNK - 1) * n_curves][SEG_WORDS] fill SDF segment records
  float* gop;          // [caps.gauss] fill Gaussians: the record's opacity, packed for the fill-run gathers
};

// The compositing lists are cut into chunks of CK = 2^ck_lg list positions,
// counted from each tile's front (list end): chunk k holds the positions
// [end - (k + 1) CK, end - k CK).  The forward stores every pixel's state at
// the chunk boundaries it passes, and the adjoint runs one work item per
// (tile, quadrant, chunk), so that a long list no longer sets the length of
// the adjoint pass.  CK is params.chunk, or chosen per launch by the
// binning (auto_chunk_log2); it is at least CK_MIN, for which the checkpoint
// store is sized.
constexpr int CK_MIN = 512, CK_MAX = 8192;
__host__ __device__ inline int n_chunks(int len, int ck_lg) { return (len + (1 << ck_lg) - 1) >> ck_lg; }
// About one adjoint item per two wavefront slots of the GPU: pairs x
// quadrants / (8 x compute units) positions per chunk, rounded to a power of
// two in [CK_MIN, CK_MAX].  Large launches keep whole lists together (fewer
// stored states and item set-ups); small ones split long lists across
// wavefronts.
__host__ __device__ inline int auto_chunk_log2(int64_t pairs, int quads, int n_cu) {
  const double v = (double)pairs * quads / (8.0 * (n_cu > 0 ? n_cu : 1));
  int lg = 9;
  while ((1 << lg) < CK_MAX && v >= 1.4142135623730951 * (double)(1 << lg)) ++lg;
  return lg;
}
// Adjoint work items per chunk of a tile list: the forward's quadrants (one
// at 8 x 8 tiles, four above), except for the tiles of scenes with fills at
// 32 x 32 tiles, which the adjoint takes as sixteen 8 x 8 pixel blocks with
// one pixel per lane (its fill-run walk is written for one pixel per lane).
__host__ __device__ constexpr int adj_blocks(int tile, bool fills) {
  return tile == 8 ? 1 : (tile == 32 && fills ? 16 : 4);
}

// Boundary segments per bounding box in the fill SDF.  Curve c (first
// boundary point boff) has a header at cbox_base(boff, c) holding the box
// (x0, x1, y0, y1) of its whole boundary, then one box per chunk of
// SDF_CHUNK segments.
constexpr int SDF_CHUNK = 8;
__host__ __device__ inline int64_t cbox_base(int64_t boff, int c) { return boff / SDF_CHUNK + 2 * (int64_t)c; }

// Segment records of the fill SDF, SEG_WORDS doubles each: for segment i of
// a filled curve (b_nb = b_0) the start point b_i, the edge e = b_{i+1} - b_i,
// 1 / |e|^2 (0 for a zero-length edge) and the end point's y.  Curve c's
// records start at seg_base(boff, c) and fill whole chunks of SDF_CHUNK:
// records past its nb segments are zero-length edges at SEG_FAR, which are
// never nearest (they follow a real segment of their chunk) and never cross.
constexpr int SEG_WORDS = 6;
constexpr double SEG_FAR = 1e100;
__host__ __device__ inline int64_t seg_base(int64_t boff, int c) { return boff + (int64_t)(SDF_CHUNK - 1) * c; }

// Floats per Gaussian in Work::ggrad: d/dmx, d/dmy, d/dsigma, then d/do_j for
// a fill Gaussian or d/dsigma_across for a tangent-aligned one (a stroke
// curve's opacity gradient is summed per curve), and d/dtheta of a
// tangent-aligned one's tangent t = (cos theta, sin theta).
constexpr int GG = 5;

// Kind of a Gaussian, in the w component of Work::gcol.
constexpr float KIND_STROKE = 0.0f, KIND_FILL = 1.0f, KIND_ANISO = 2.0f;

// Work::queue slots with the number of fill and of stroke Gaussians the
// sampling pass asked for (written with the Gaussian offsets), which lets the
// per-kind adjoint kernels return at once when there are none.
constexpr int Q_NFILL = 8, Q_NSTROKE = 9, Q_NANISO = 10;
// Work::queue slot with the log2 chunk length that the binning chose for the
// launch's lists when params.chunk is 0 (read by the blend kernels).
constexpr int Q_CKLG = 11;

struct Layout {
  size_t off[N_WS];
  size_t total;
  int64_t sort_blocks, scan_blocks;
};

Layout workspace_layout(const nsplat_curves* cv, const nsplat_scenes* sc, const nsplat_caps* caps);
Work carve(void* ws, const Layout& lay);

// ---------------------------------------------------------------------------
// Curve view: degree, sizes and where its knots live.
// ---------------------------------------------------------------------------
struct CurveView {
  int p, nk, nt, flags, m, ncp, k0, t0;
  int pmax;   // the batch's degree bound
  int fmask;  // the batch's declared flags
  int amask;  // the flags every curve of the batch declares it carries
  const double* U;
  __device__ bool closed() const { return (flags & NSPLAT_CLOSED) != 0; }
  __device__ bool filled() const { return (flags & NSPLAT_FILLED) != 0; }
  __device__ bool aniso() const { return (flags & NSPLAT_ANISO) != 0; }
  // Closed curves wrap the last ceil(p/2) key points in front (Sec. 3.1).
  __device__ int key_of_cp(int j) const {
    if (!closed()) return j;
    int k = j - (p + 1) / 2;
    k %= nk;
    return k < 0 ? k + nk : k;
  }
};

__device__ inline CurveView curve_view(const nsplat_curves& cv, const double* knots, int c) {
  CurveView v;
  v.p = cv.degree[c];
  v.pmax = (cv.max_degree >= 1 && cv.max_degree <= MAXP) ? cv.max_degree : MAXP;
  v.flags = cv.flags[c];
  v.fmask = cv.any_flags;
  v.amask = cv.all_flags;
  v.k0 = cv.key_off[c];
  v.nk = cv.key_off[c + 1] - v.k0;
  v.t0 = cv.tau_off[c];
  v.nt = cv.tau_off[c + 1] - v.t0;
  const bool closed = (v.flags & NSPLAT_CLOSED) != 0;
  v.ncp = closed ? v.nk + v.p : v.nk;
  v.m = v.nt + 2 * v.p;
  v.U = knots + v.t0 + (int64_t)c * KNOT_PAD;
  return v;
}

__device__ inline bool curve_valid(const CurveView& v) {
  if (v.p < 1 || v.p > v.pmax) return false;
  if (v.flags & ~v.fmask) return false;  // a flag the batch did not declare
  if ((v.flags & v.amask) != v.amask) return false;  // a flag all curves were declared to carry
  if (v.nk < v.p + 1) return false;
  if (v.nt != (v.closed() ? v.nk : v.nk - v.p)) return false;
  if (v.filled() && !v.closed()) return false;
  if (v.filled() && v.aniso()) return false;  // tangent alignment concerns contour samples only
  return true;
}

// Knot span of u: the largest i in [p, m-p-1] with U[i] <= u < U[i+1]; at or
// past the right end of the domain, the last non-empty span.
__device__ inline int find_span(const double* U, int p, int m, double u) {
  const int lo = p, hi = m - p - 1;
  if (u >= U[hi + 1]) {
    int i = hi;
    while (i > lo && !(U[i] < U[i + 1])) --i;
    return i;
  }
  int a = lo, b = hi + 1;  // U[a] <= u < U[b] once u >= U[lo]
  if (!(U[lo] <= u)) {
    int i = lo;
    while (i < hi && !(U[i] < U[i + 1])) ++i;
    return i;
  }
  while (b - a > 1) {
    const int mid = (a + b) >> 1;
    if (U[mid] <= u) a = mid;
    else b = mid;
  }
  return a;
}

// Non-zero B-spline basis functions on a non-empty span (Cox-de Boor in the
// triangular "left/right" form): N[r] = N_{span-p+r, p}(u), r = 0..p, and if
// dN != nullptr their u-derivatives from the degree p-1 functions,
// N'_{i,p} = p (N_{i,p-1} / (U_{i+p} - U_i) - N_{i+1,p-1} / (U_{i+p+1} - U_{i+1})).
// On a non-empty span no denominator can vanish.
__device__ inline void basis_funs(const double* U, int span, int p, double u, double (&N)[MAXP + 1],
                                  double* dN) {
  double left[MAXP + 1], right[MAXP + 1];
  N[0] = 1.0;
#pragma unroll
  for (int r = 1; r <= MAXP; ++r) N[r] = 0.0;
#pragma unroll
  for (int d = 1; d <= MAXP; ++d) {
    if (d > p) break;
    if (d == p && dN != nullptr) {
#pragma unroll
      for (int r = 0; r <= MAXP; ++r) {
        if (r > p) break;
        double v = 0.0;
        if (r >= 1) v += N[r - 1] / (U[span + r] - U[span - p + r]);
        if (r <= p - 1) v -= N[r] / (U[span + r + 1] - U[span - p + r + 1]);
        dN[r] = (double)p * v;
      }
    }
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
  }
}

// Rational curve point (x, y, width) at u on `span` (Eq. 1 / Eq. 4) and, if
// d != nullptr, its u-derivative by the quotient rule (Eq. 2).
__device__ inline void curve_point(const nsplat_curves& cv, const CurveView& v, double u, int span,
                                   double (&pt)[3], double* d) {
  double N[MAXP + 1], dN[MAXP + 1];
  basis_funs(v.U, span, v.p, u, N, d ? dN : nullptr);
  double S[3] = {0.0, 0.0, 0.0}, Sd[3] = {0.0, 0.0, 0.0}, W = 0.0, Wd = 0.0;
#pragma unroll
  for (int r = 0; r <= MAXP; ++r) {
    if (r > v.p) break;
    const int k = v.k0 + v.key_of_cp(span - v.p + r);
    const double w = (double)cv.key_w[k];
    const double P[3] = {(double)cv.key_xy[2 * k], (double)cv.key_xy[2 * k + 1], (double)cv.key_s[k]};
    const double nw = N[r] * w;
    W += nw;
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
  for (int q = 0; q < 3; ++q) pt[q] = S[q] / W;
  if (d) {
#pragma unroll
    for (int q = 0; q < 3; ++q) d[q] = (W * Sd[q] - S[q] * Wd) / (W * W);
  }
}

// Sample parameter j of `count` uniform samples in the domain [a, b]: open
// curves include both ends (the last sample is b exactly), closed curves
// exclude the closure point.  dt returns du/db (du/da = 1 - dt).
__device__ inline double sample_u(double a, double b, int j, int count, bool closed, double* dt) {
  if (!closed) {
    if (j >= count - 1) {
      if (dt) *dt = 1.0;
      return b;
    }
    const double step = (b - a) / (double)(count - 1);
    if (dt) *dt = (double)j / (double)(count - 1);
    return a + (double)j * step;
  }
  const double step = (b - a) / (double)count;
  if (dt) *dt = (double)j / (double)count;
  return a + (double)j * step;
}

__device__ inline float read_h(const nsplat_params& pr) { return pr.h_dev ? *pr.h_dev : pr.h; }

// One axis of a Gaussian's binning rectangle (Sec. 3.4): from m = fl32(mu)
// and r = k_sigma sigma in FP32, the interval [(m - r) - 1, (m + r) + 1] in
// tiles, floor(x / tile) clamped to [0, n - 1] (f0 > f1: no tile).  False for
// a NaN bound.
__device__ inline bool tile_axis(float m, float r, float inv_tile, int n, float* f0, float* f1) {
  const float lo = (m - r) - 1.0f, hi = (m + r) + 1.0f;
  if (!(lo == lo) || !(hi == hi)) return false;
  *f0 = fmaxf(0.0f, floorf(lo * inv_tile));
  *f1 = fminf((float)(n - 1), floorf(hi * inv_tile));
  return true;
}

// The last c with a[S c + O] <= x, for an ascending column of n entries
// (stride S, offset O) whose first entry is <= x.
template <int S, int O>
__device__ inline int last_le(const int32_t* a, int n, int64_t x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a[(int64_t)S * mid + O] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// A 64-bit value of the first active lane (wavefront-uniform).
__device__ inline int64_t first_lane_i64(int64_t v) {
  const uint32_t lo32 = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi32 = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi32 << 32) | lo32);
}

// last_le for a lane of a wavefront whose active lanes hold ascending x,
// given the answer c0 for the first active lane's x0: each lane steps
// forward from c0 over at most 8 entries; a lane that would need more, or
// holds a smaller x, searches alone.
template <int S, int O>
__device__ inline int last_le_walk(const int32_t* a, int n, int64_t x, int64_t x0, int c0) {
  if (x < x0) return last_le<S, O>(a, n, x);
  int c = c0;
  for (int k = 0; k < 8; ++k) {
    if (c + 1 >= n || a[(int64_t)S * (c + 1) + O] > x) return c;
    ++c;
  }
  return last_le<S, O>(a, n, x);
}

// The same with c0 found by one search for the first active lane's x
// (wavefront-uniform; the column is read through the constant address space,
// so the loads are scalar).  The column must not change during the kernel.
template <int S, int O>
__device__ inline int last_le_wave(const int32_t* a, int n, int64_t x) {
  typedef const __attribute__((address_space(4))) int32_t* const_i32;
  const const_i32 ca = (const_i32)a;
  const int64_t x0 = first_lane_i64(x);
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ca[(int64_t)S * mid + O] <= x0) lo = mid;
    else hi = mid - 1;
  }
  return last_le_walk<S, O>(a, n, x, x0, lo);
}

// The curve of Gaussian g: the last c with goff[c] <= g (goff ascending,
// goff[0] = 0), per lane, per wavefront, and from the curve c0 of the first
// active lane's g0.
__device__ inline int curve_search(const int32_t* goff, int n, int64_t g) { return last_le<1, 0>(goff, n, g); }
__device__ inline int curve_of_wave(const int32_t* goff, int n, int64_t g) { return last_le_wave<1, 0>(goff, n, g); }
__device__ inline int curve_walk(const int32_t* goff, int n, int64_t g, int64_t g0, int c0) {
  return last_le_walk<1, 0>(goff, n, g, g0, c0);
}

// Scene of a global tile index (binary search over the scene table).
__device__ inline int scene_of_tile(const SceneTab* st, int n_scenes, int tile) {
  int lo = 0, hi = n_scenes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (st[mid].tile_off <= tile) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// Launch helpers (host side), one per kernel family.
// ---------------------------------------------------------------------------
// Optional per-phase timing with HIP events (nsplat_timing): each phase is
// bracketed by two events on the launch stream; sums are read back on demand.
struct Timer {
  bool on = false;
  uint32_t mask = 0;  // phases recorded while on (bit NSPLAT_T_*)
  hipEvent_t* pool = nullptr;
  int cap = 0, used = 0;
  int span_id[4096];
  int span_ev[4096][2];
  int n_spans = 0;
  int open_ev[NSPLAT_NUM_TIMERS];
  double ms[NSPLAT_NUM_TIMERS];
  int64_t count[NSPLAT_NUM_TIMERS];
};
void timer_begin(Timer* t, int id, hipStream_t s);
void timer_end(Timer* t, int id, hipStream_t s);

struct Launch {
  Timer* tm = nullptr;
  const nsplat_curves* cv;
  const nsplat_scenes* sc;
  const nsplat_params* pr;
  const nsplat_buffers* bf;
  Work w;
  Layout lay;
  hipStream_t stream;
  int64_t n_tiles;
  int n_cu;
  int ck_lg;  // log2 of params.chunk, or -1: chosen by the binning (Q_CKLG)
};
// the adjoint's pixel blocks per chunk for this launch's tile side and curves
inline int adj_blocks_of(const Launch& L) { return adj_blocks(L.pr->tile, (L.cv->any_flags & NSPLAT_FILLED) != 0); }

// Scene table; also clears the NSPLAT_NUM_COUNTERS counters when given.
hipError_t launch_scene_setup(const Launch& L, int32_t* clear_counters);
// nsplat_udf_loss_noalloc's device scratch: UDF_SCRATCH_SLOTS doubles per
// device (per-scene sums, so at most UDF_SCRATCH_SLOTS - 1 scenes), its
// address taken once per device (with that device current) by
// udf_scratch_setup and read back by udf_scratch (nullptr before the setup).
constexpr int UDF_SCRATCH_SLOTS = 4096;
constexpr int MAX_DEVICES = 64;
hipError_t udf_scratch_setup(int device);
double* udf_scratch(int device);
hipError_t launch_sample(const Launch& L, int frozen);
hipError_t launch_bin(const Launch& L);
hipError_t launch_blend_fwd(const Launch& L, float* image, float* T_final, int32_t* n_last, int persistent);
hipError_t launch_blend_bwd(const Launch& L, const float* dL, const float* T_final, const int32_t* n_last,
                            int persistent);
hipError_t launch_adjoint(const Launch& L, const nsplat_grads* g);
hipError_t launch_reg(const Launch& L, const nsplat_reg* reg);
hipError_t launch_udf(const Launch& L, const int32_t* sel, float tau, const float* image, const float* target,
                      float* dL, float* loss, double* sacc = nullptr);
hipError_t launch_adam(const nsplat_adam* cfg, const nsplat_values* prm, const nsplat_grads* g, float* m, float* v,
                       int32_t* step_dev, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_scan(uint32_t* data, const int32_t* n_dev, int64_t n_cap, uint32_t* total_out, uint32_t* tmp,
                       hipStream_t s);
hipError_t launch_anneal(float* h_dev, int32_t* step_dev, int32_t step, int32_t total, float hmax, float hmin,
                         float tb, float te, hipStream_t s);
hipError_t launch_l2(const float* a, const float* b, float* out, float* loss, int64_t n, hipStream_t s);

struct Phase {
  Timer* t;
  int id;
  hipStream_t s;
  Phase(const Launch& L, int i) : t(L.tm && L.tm->on && ((L.tm->mask >> i) & 1u) ? L.tm : nullptr), id(i), s(L.stream) {
    if (t) timer_begin(t, id, s);
  }
  ~Phase() { if (t) timer_end(t, id, s); }
};

inline int grid_for(int64_t n, int threads, int max_blocks) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > max_blocks) b = max_blocks;
  return (int)b;
}

}  // namespace nsp
