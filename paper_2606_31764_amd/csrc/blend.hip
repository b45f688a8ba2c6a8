// nsplat_forward / the first half of nsplat_backward: per-tile alpha
// compositing (Sec. 3.4, Eq. 8-9) and its adjoint.
//
// The forward's unit of work is one wavefront per (tile, quadrant): see
// TileCfg below.  Centres become exact tile-local FP32 coordinates when an
// entry is loaded (FP64 centre minus the tile origin, rounded once).  The
// forward stops a pixel once T < eps_T and a wavefront once all its pixels
// have stopped, and stores each pixel's state at every chunk boundary (a
// chunk is 2^ck_lg list positions, chosen per launch) it passes.  The
// adjoint runs one wavefront per (tile, quadrant or 8x8 pixel block, chunk)
// (AdjCfg), back to front from the state stored at the chunk's back
// boundary, parks each Gaussian's per-lane gradient values in LDS and sums
// a dozen or more such rows at a time, with one atomic per value and
// wavefront.
#include "nsplat_internal.h"

namespace nsp {

namespace {

// Work decomposition: one wavefront per (tile, quadrant) item.  8x8 tiles are
// one quadrant; 16x16 and 32x32 tiles have four (8x8 or 16x16 pixels), and
// each lane owns a BLK x BLK block of its quadrant.  A wavefront walks the
// tile's list in steps of up to 64 E entries: every lane loads E entries (the
// next step's loads are issued before the current step is processed),
// entries whose support disc misses the quadrant are dropped, the rest are
// compacted in order into the wavefront's own LDS arrays and then composited
// one after another.  Wavefronts never wait for each other.
template <int TILE>
struct TileCfg {
  static constexpr int QUADS = TILE == 8 ? 1 : 4;
  static constexpr int SUB = TILE == 8 ? 8 : TILE / 2;
  static constexpr int BLK = SUB / 8;
  static constexpr int PPT = BLK * BLK;
};
constexpr int WPB = 4;                  // wavefronts per block
// Kernel forms (template KIND): with the tangent-aligned kind, with the
// fill-run walk (see FillRun).
constexpr int KIND_ANI = 1, KIND_FILL = 2;
constexpr int BLOCK = 64 * WPB;

template <int TILE>
__device__ inline void pixel_of(int quad, int lane, int q, int* lx, int* ly) {
  using Cfg = TileCfg<TILE>;
  *lx = (quad & 1) * Cfg::SUB + (lane & 7) * Cfg::BLK + q % Cfg::BLK;
  *ly = (quad >> 1) * Cfg::SUB + (lane >> 3) * Cfg::BLK + q / Cfg::BLK;
}

// The adjoint's pixel blocks (adj_blocks): the forward's quadrants, or, for
// the tiles of scenes with fills at 32 x 32 tiles, sixteen 8 x 8 blocks with
// one pixel per lane.  Block b sits at column b % COLS, row b / COLS of the
// tile; lane l owns the BLK x BLK pixels at column l & 7, row l >> 3 of it.
template <int TILE, bool SPLIT_>
struct AdjCfg {
  static constexpr bool SPLIT = SPLIT_;
  static constexpr int QUADS = SPLIT ? 16 : TileCfg<TILE>::QUADS;
  static constexpr int SUB = SPLIT ? 8 : TileCfg<TILE>::SUB;
  static constexpr int BLK = SUB / 8;
  static constexpr int PPT = BLK * BLK;
  static constexpr int COLS = TILE / SUB;
  static_assert(!SPLIT || TILE == 32, "8 x 8 blocks split 32 x 32 tiles only");
  static_assert(QUADS == adj_blocks(TILE, SPLIT), "adjoint blocks follow the binning's items");
};

template <class A>
__device__ inline void adj_pixel(int blk, int lane, int q, int* lx, int* ly) {
  *lx = (blk % A::COLS) * A::SUB + (lane & 7) * A::BLK + q % A::BLK;
  *ly = (blk / A::COLS) * A::SUB + (lane >> 3) * A::BLK + q / A::BLK;
}

// Slot of tile pixel (lx, ly) in a stored forward state: the forward's
// (quadrant x pixels per lane + pixel) x 64 + lane, as pixel_of lays it out.
template <int TILE>
__device__ inline int fwd_slot(int lx, int ly) {
  using F = TileCfg<TILE>;
  const int quad = lx / F::SUB + 2 * (ly / F::SUB);
  const int lane = (lx % F::SUB) / F::BLK + 8 * ((ly % F::SUB) / F::BLK);
  const int q = lx % F::BLK + F::BLK * (ly % F::BLK);
  return (quad * F::PPT + q) * 64 + lane;
}

// Next work item of this wavefront: the static assignment, or the next entry
// of the device work queue (persistent form).
__device__ inline int next_item(int it, int persistent, int32_t* queue) {
  if (!persistent)
    return __builtin_amdgcn_readfirstlane(it == 0 ? (int)(blockIdx.x * WPB + (threadIdx.x >> 6)) : 0x7fffffff);
  int v = 0;
  if (__lane_id() == 0) v = atomicAdd(queue, 1);
  return __builtin_amdgcn_readfirstlane(v);
}

// One list entry as loaded by a lane.
struct Entry {
  Gauss r;
  float c0, c1, c2;
  int g, kind;  // kind: 0 isotropic stroke, 1 fill, 2 tangent-aligned stroke
};

// Record and colour of Gaussian g.
__device__ inline void load_rec(const Gauss* __restrict__ gs, const float4* __restrict__ gcol, int g, Entry* e) {
  e->g = g;
  e->r = gs[g];
  const float4 cf = gcol[g];
  e->c0 = cf.x;
  e->c1 = cf.y;
  e->c2 = cf.z;
  e->kind = (int)cf.w;
}

// The entry's record and its curve's colour / fill tag (both by Gaussian
// index, so the two loads go out together once the index has arrived).
__device__ inline void load_entry(const int32_t* __restrict__ idx, const Gauss* __restrict__ gs,
                                  const float4* __restrict__ gcol, int pos, bool ok, Entry* e) {
  if (!ok) return;
  e->g = idx[pos];
  load_rec(gs, gcol, e->g, e);
}

// Rectangle of tile-local pixel centres: x in [x0, x1], y in [y0, y1].
struct Box {
  float x0, y0, x1, y1;
};

// The pixel centres held by the lanes with a set bit in `live` (lane l owns
// the BLK x BLK block at column l & 7, row l >> 3 of the quadrant): rows from
// the lowest and highest set bits, columns from the eight row bytes folded
// together.  Scalar work on a wavefront-uniform mask; `live` != 0.
template <class Cfg>
__device__ inline Box live_box_of(int qx, int qy, uint64_t live) {
  const int r0 = __builtin_ctzll(live) >> 3, r1 = (63 - __builtin_clzll(live)) >> 3;
  uint64_t f = live | (live >> 32);
  f |= f >> 16;
  f |= f >> 8;
  const uint32_t cols = (uint32_t)f & 0xffu;
  const int c0 = __builtin_ctz(cols), c1 = 31 - __builtin_clz(cols);
  Box b;
  b.x0 = (float)(qx + c0 * Cfg::BLK);
  b.x1 = (float)(qx + c1 * Cfg::BLK + Cfg::BLK - 1);
  b.y0 = (float)(qy + r0 * Cfg::BLK);
  b.y1 = (float)(qy + r1 * Cfg::BLK + Cfg::BLK - 1);
  return b;
}

template <int TILE>
__device__ inline Box live_box(int quad, uint64_t live) {
  using Cfg = TileCfg<TILE>;
  return live_box_of<Cfg>((quad & 1) * Cfg::SUB, (quad >> 1) * Cfg::SUB, live);
}

// All pixel centres of the quadrant.
template <int TILE>
__device__ inline Box quad_box(int quad) {
  using Cfg = TileCfg<TILE>;
  Box b;
  b.x0 = (float)((quad & 1) * Cfg::SUB);
  b.y0 = (float)((quad >> 1) * Cfg::SUB);
  b.x1 = b.x0 + (float)(Cfg::SUB - 1);
  b.y1 = b.y0 + (float)(Cfg::SUB - 1);
  return b;
}

// Tile-local centre (relative to the tile's first pixel centre), squared
// support radius, exp2 coefficient -log2(e) / (2 sigma^2), and whether the
// support disc reaches the rectangle `bx` of pixel centres (the quadrant's
// pixels that can still take part), with the radius enlarged by a relative
// 1e-4 so that the test is conservative under FP32 rounding.
__device__ inline bool entry_geometry(const Gauss& r, double ox, double oy, float ks, const Box& bx, float4* geo) {
  const double sg = (double)r.sigma;
  const float rr = ks * r.sigma;
  const float cx = (float)(r.mx - ox), cy = (float)(r.my - oy);
  *geo = make_float4(cx, cy, rr * rr, (float)(-0.5 * LOG2E / (sg * sg)));
  const float rc = rr * 1.0001f + 1e-4f;
  const float dx = fmaxf(fmaxf(bx.x0 - cx, cx - bx.x1), 0.0f);
  const float dy = fmaxf(fmaxf(bx.y0 - cy, cy - bx.y1), 0.0f);
  return dx * dx + dy * dy <= rc * rc;
}

// A tangent-aligned Gaussian (axis sigma along t, sp across it, sigma >= sp)
// is evaluated as exp2(-(a^2 + b^2)) with a = d . u and b = r (d x u), d the
// offset from the centre: u = t sqrt(ck) / sigma, r = sigma / sp, and
// ck = log2(e) / 2, so that a^2 + b^2 = ck (d_t^2 / sigma^2 + d_n^2 / sp^2).
// The support is a^2 + b^2 <= ck k_sigma^2, inside the disc of radius
// k_sigma sigma that binning and culling use.  Entries are staged like the
// others (exp2 coefficient -ck / sigma^2); after staging a step that holds
// such entries, the wavefront converts them, reading (t, sp, r) by Gaussian
// index, so that the other kinds carry no extra loads.  Where the two axes
// agree r is exactly 1 and the theta partial exactly 0.
constexpr float ANI_CK = (float)(0.5 * LOG2E);
constexpr float ANI_SQRT_CK = 0.8493218002880191f;  // sqrt(log2(e) / 2)
__device__ inline void aniso_axes(const float4& aux, float coef, float* ux, float* uy, float* r) {
  const float k = __builtin_sqrtf(-coef);  // sqrt(ck) / sigma
  *ux = aux.x * k;
  *uy = aux.y * k;
  *r = aux.w;  // sigma / sp, rounded once from FP64 (exactly 1 where the axes agree)
}

__device__ inline uint64_t lanes_below() {
  const int lane = __lane_id();
  return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// ---------------------------------------------------------------------------
// Fill runs.  A fill curve's Gaussians sit on the lattice ((i + 1/2) h,
// (j + 1/2) h) of its window and are emitted row by row (Sec. 3.3), all with
// one sigma.  Binning's test (tile_axis) is separable and monotone along each
// lattice axis, so the curve's points on a tile form a rectangle
// [i0, i1] x [j0, j1] of the window, and since a tile's list is in Gaussian
// order they occupy one run of consecutive positions, row by row.  At h = 1
// the lattice is the pixel grid: a pixel's in-support Gaussians of the run are
// its lattice neighbours at integer offsets (dx, dy) with dx^2 + dy^2 <=
// (k_sigma sigma)^2, so each lane walks those offsets (in list order) and
// gathers the opacities from LDS instead of visiting every entry of the run.
// ---------------------------------------------------------------------------
struct FillRun {
  int c, ix0, iy0, nx, goff;  // curve, window origin, window columns, first Gaussian
  int i0, i1, j0, j1, w;      // the run's rectangle (window-relative) and its width
  int p_lo, p_hi;             // its list positions
  int g_top;                  // the Gaussian at the run's entry point
  float sigma;                // the curve's fill sigma
};

// Window-relative lattice indices [k0, k1] (below n) whose binning interval
// covers tile t along one axis: each lane tests one candidate (the same
// arithmetic as binning).  False when the interval does not fit the 64
// candidates.
__device__ inline bool fill_axis(int org, int n, double h, float r, float inv, int n_tiles, int t, int tile, int* k0,
                                 int* k1) {
  const int base = (int)floor(((double)t * tile - (double)r - 2.0) / h - 0.5) - org - 1;
  const int k = base + (int)__lane_id();
  bool ok = false;
  if (k >= 0 && k < n) {
    const float m = (float)(((double)(org + k) + 0.5) * h);
    float f0, f1;
    ok = tile_axis(m, r, inv, n_tiles, &f0, &f1) && f0 <= (float)t && (float)t <= f1;
  }
  const uint64_t b = __ballot(ok);
  if (b == 0ull) return false;
  const int lo = __builtin_ctzll(b), hi = 63 - __builtin_clzll(b);
  if (__popcll(b) != hi - lo + 1) return false;           // not an interval
  if ((lo == 0 && base + lo > 0) || (hi == 63 && base + hi < n - 1)) return false;  // may extend past the candidates
  *k0 = base + lo;
  *k1 = base + hi;
  return true;
}

// The run of fill curve c that holds list position `at` (whose Gaussian has
// window index `local`): its rectangle and list positions, if they fit the
// list.  Wavefront-uniform.  Whether the list holds the whole rectangle there
// is for fill_corners_ok to say.
__device__ inline bool fill_run_at(const int32_t* __restrict__ plan, int c, int g, int local, float sigma, int at,
                                   int start, int end, double h, float ks, float inv, const SceneTab& st, int lt,
                                   int tile, FillRun* fr) {
  typedef const __attribute__((address_space(4))) int32_t* cip;
  const cip row = (cip)(plan + (int64_t)P_STRIDE * c);
  fr->c = c;
  fr->ix0 = row[P_IX0];
  fr->iy0 = row[P_IY0];
  fr->nx = row[P_NX];
  fr->goff = row[P_GOFF];
  const int ny = row[P_NY];
  fr->g_top = g;
  fr->sigma = sigma;
  if (fr->nx <= 0 || ny <= 0) return false;
  const float r = ks * sigma;
  const int tcol = lt % st.tiles_x, trow = lt / st.tiles_x;
  if (!fill_axis(fr->ix0, fr->nx, h, r, inv, st.tiles_x, tcol, tile, &fr->i0, &fr->i1)) return false;
  if (!fill_axis(fr->iy0, ny, h, r, inv, st.tiles_y, trow, tile, &fr->j0, &fr->j1)) return false;
  const int jt = local / fr->nx, it = local - jt * fr->nx;
  if (it < fr->i0 || it > fr->i1 || jt < fr->j0 || jt > fr->j1) return false;
  fr->w = fr->i1 - fr->i0 + 1;
  const int64_t n = (int64_t)fr->w * (fr->j1 - fr->j0 + 1);
  fr->p_lo = at - ((jt - fr->j0) * fr->w + (it - fr->i0));
  const int64_t p_hi = (int64_t)fr->p_lo + n - 1;
  if (fr->p_lo < start || p_hi >= end) return false;
  fr->p_hi = (int)p_hi;
  return true;
}

// The run's two corner entries are those of the rectangle: otherwise (a run
// cut short by a capacity overflow) it is left to the entry-by-entry path.
__device__ inline bool fill_corners_ok(const int32_t* __restrict__ idx, const FillRun& fr) {
  const int g_lo = __builtin_amdgcn_readfirstlane(idx[fr.p_lo]);
  const int g_hi = __builtin_amdgcn_readfirstlane(idx[fr.p_hi]);
  return g_lo == fr.goff + fr.j0 * fr.nx + fr.i0 && g_hi == fr.goff + fr.j1 * fr.nx + fr.i1;
}

// Opacities of the quadrant's lattice neighbourhood (NB x NB cells, window
// index (ib, jb) at cell 0; lane l gathers cells it * 64 + l): those of the
// run's Gaussians at list positions p0 .. p1, `none` elsewhere, read from the
// packed fill opacities (gop, the records' values).  Reads below the record
// capacity only, so that a rectangle still to be checked is safe.
template <int NB, int NIT>
__device__ inline void fill_gather(const float* __restrict__ gop, int64_t gcap, const FillRun& fr, int ib, int jb,
                                   int p0, int p1, float none, float (&og)[NIT]) {
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int sl = it * 64 + (int)__lane_id();
    const int j = jb + sl / NB, i = ib + sl % NB;
    float o = none;
    if (sl < NB * NB && i >= fr.i0 && i <= fr.i1 && j >= fr.j0 && j <= fr.j1) {
      const int pos = fr.p_lo + (j - fr.j0) * fr.w + (i - fr.i0);
      const int64_t g = (int64_t)fr.goff + (int64_t)j * fr.nx + i;
      if (pos >= p0 && pos <= p1 && g < gcap) o = gop[g];
    }
    og[it] = o;
  }
}

// Offsets (dx, dy) of a pixel's lattice neighbours inside the 6 sigma disc at
// h = 1 (sigma = eta / rho, so k_sigma sigma = 4.5 with the paper's
// constants): dx^2 + dy^2 <= R2, walked front to back (descending list
// position: rows from the bottom, each from the right).
constexpr int FR_R = 4;   // the largest |dx| the walk visits
constexpr int FR_R2 = 20;  // dx^2 + dy^2 bound for k_sigma sigma = 4.5
// LDS row stride of the adjoint's lattice cells: 24 floats puts the four
// lane rows of a half-wavefront in four different bank octets
constexpr int FR_NS = 24;

// LDS bytes per wavefront for a step of `depth` entries.
// A forward entry: what every composited pixel reads, in one 32-byte record
// (one LDS address per entry), and the colour, read where a run begins.
struct FwdRec {
  float4 geo;      // tile-local centre, squared support radius, exp2 coefficient
                   // (tangent-aligned: centre, scaled axis u)
  float op;           // opacity
  int pos, curve, g;  // list position, curve, Gaussian (tangent-aligned, once
                      // converted: the bits of the axis ratio r)
};
constexpr int FWD_ENTRY_BYTES = sizeof(FwdRec) + 16;
constexpr int BWD_ENTRY_BYTES = 48;   // geometry, opacity + colour, (g, curve, position, 1/sigma^3)
// The adjoint parks the per-lane gradient values it still has to sum over
// the wavefront in LDS rows of 64 floats, one row per value (three for a
// stroke Gaussian, one for a fill Gaussian), each with its (Gaussian, value
// index) target, and sums park_rows rows at a time (see flush_rows).  Rows
// are padded to 68 floats so that the flush's reads fall into different
// banks.  One-pixel-per-lane adjoints at depth 64 park 12 rows, which keeps a
// wavefront's LDS slice small enough for six wavefronts per SIMD; the others
// (held to fewer wavefronts by their registers) park 16.
constexpr int RB_ROW = 68;  // floats per parked row
__host__ __device__ constexpr bool bwd_six_waves(int tile, int E, int kind) {
  return tile <= 16 && E == 1 && !(kind & KIND_FILL);
}
__host__ __device__ constexpr int park_rows(int tile, int E, int kind) { return bwd_six_waves(tile, E, kind) ? 12 : 16; }
// wavefronts per SIMD the adjoint is built for: six without the fill-run
// walk at one pixel per lane and one entry per lane, four with it (or at
// several pixels per lane), one at several entries per lane
__host__ __device__ constexpr int bwd_waves(int tile, int E, int kind) {
  return bwd_six_waves(tile, E, kind) ? 6 : (E == 1 ? 4 : 1);
}
__host__ __device__ constexpr size_t bwd_wave_bytes(int tile, int E, int kind) {
  return ((size_t)64 * E * BWD_ENTRY_BYTES + (size_t)park_rows(tile, E, kind) * (RB_ROW * 4 + 8) + 15) / 16 * 16;
}

// Lower end of the step that starts at list position h (walking down from
// the list end): at most `depth` entries, not below `start`, and not across
// the boundary of h's chunk.
__device__ inline int step_floor(int h, int start, int depth, int end, int ck_lg) {
  const int k = (end - h) >> ck_lg;
  return max(max(start, h - depth), end - ((k + 1) << ck_lg));
}

template <int C, int TILE, int E, int KIND>
__global__ __launch_bounds__(BLOCK, E == 1 ? 4 : 1) void k_blend_fwd(
    nsplat_curves cv, nsplat_params pr, Work w, int n_scenes, int n_items, const Gauss* __restrict__ gs,
    const int32_t* __restrict__ ranges, const int32_t* __restrict__ idx, const float* __restrict__ bg,
    float* __restrict__ image, float* __restrict__ Tfin, int32_t* __restrict__ nlast, const int32_t* __restrict__ plan,
    int64_t gcap, int persistent, int ck_arg) {
  using Cfg = TileCfg<TILE>;
  constexpr int PPT = Cfg::PPT;
  extern __shared__ __align__(16) char smem[];
  typedef const __attribute__((address_space(4))) int32_t* const_i32;
  // the chunk length: the caller's, or the one the binning chose
  const int ck_lg = ck_arg >= 0 ? ck_arg : ((const_i32)w.queue)[Q_CKLG];
  const int depth = min(pr.batch, 64 * E);   // entries per step (E per lane; fewer lanes below 64)
  const float amax = pr.alpha_max, eps = pr.eps_T, ks = pr.k_sigma;
  const int lane = __lane_id(), wv = threadIdx.x >> 6;
  char* mine_lds = smem + (size_t)wv * (64 * E) * FWD_ENTRY_BYTES;
  FwdRec* wrec = (FwdRec*)mine_lds;
  float4* wcol = (float4*)(wrec + 64 * E);  // colour
  const uint64_t below = lanes_below();
  constexpr bool ANI = (KIND & KIND_ANI) != 0;
  // fill runs at h = 1 walk each pixel's lattice neighbours (see FillRun);
  // the support radius must be the 4.5 the offsets are laid out for
  const bool fill_lattice = (KIND & KIND_FILL) != 0 && read_h(pr) == 1.0f;
  const float inv_tile = 1.0f / (float)TILE;
  for (int it = 0;; ++it) {
    const int item = next_item(it, persistent, w.queue);
    if (item >= n_items) break;
    const int tq = item / Cfg::QUADS, quad = item - tq * Cfg::QUADS;
    const int tile = w.order[tq];
    const int s = scene_of_tile(w.scenes, n_scenes, tile);
    const SceneTab st = w.scenes[s];
    const int lt = tile - st.tile_off;
    const int x0 = (lt % st.tiles_x) * TILE, y0 = (lt / st.tiles_x) * TILE;
    // The colour is accumulated per run of entries of one curve (one
    // colour): over a run, sum alpha_j T_j = T at its start - T now
    // (alpha_j T_j = T_j - T_{j+1}), so each pixel keeps Tst, its T where the
    // run began, and adds col (Tst - T) where the run ends.  Runs end where
    // the curve changes between consecutive composited entries, at chunk
    // boundaries and at the end, all fixed by the list, so the result does not
    // depend on the batch depth.
    float px[PPT], py[PPT], T[PPT], Tst[PPT], acc[PPT][3];
    int stop[PPT];
    int run_curve = -1, run_kind = 0;
    float rc0 = 0.0f, rc1 = 0.0f, rc2 = 0.0f;  // the run's colour
    const int start = ranges[2 * tile], end = ranges[2 * tile + 1];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      int lx, ly;
      pixel_of<TILE>(quad, lane, q, &lx, &ly);
      px[q] = (float)lx;
      py[q] = (float)ly;
      // a pixel is live while T >= eps_T (0 <= eps_T <= 1): T only falls,
      // and it falls below eps_T exactly at the entry where the pixel stops;
      // pixels outside the image start at T = 0
      T[q] = (x0 + lx < st.W && y0 + ly < st.H) ? 1.0f : 0.0f;
      Tst[q] = T[q];
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[q][c] = 0.0f;
      stop[q] = start;
    }
    const double ox = (double)x0 + 0.5, oy = (double)y0 + 0.5;
    const Box qbox = quad_box<TILE>(quad);
    // front to back: list positions end-1 down to start, at most `depth` per
    // step and never across a chunk boundary, where the state is stored
    const int ck0 = w.ck_off[tile];
    int n_ck = 0;  // chunk boundaries passed (state stored)
    // loads run two steps ahead for the list indices and one step ahead for
    // the records, so a step waits for one round trip, issued a step earlier
    Entry e[E];
    int gnext[E];  // Gaussian indices of the next step
    int hi = end, lo_s = step_floor(hi, start, depth, end, ck_lg);
    int nhi = lo_s, nlo = step_floor(nhi, start, depth, end, ck_lg);
#pragma unroll
    for (int u = 0; u < E; ++u) {
      const int k = u * 64 + lane;
      load_entry(idx, gs, w.gcol, hi - 1 - k, k < hi - lo_s, &e[u]);
      gnext[u] = k < nhi - nlo ? idx[nhi - 1 - k] : 0;
    }
    // One fill run's positions fr.p_lo .. top at h = 1, front to back for each
    // pixel: the colour run, the chunk boundaries and the per-pixel
    // arithmetic are those of the entry-by-entry path, entry for entry.
    constexpr int FNB = Cfg::SUB + 2 * FR_R;  // lattice neighbourhood of the quadrant, per axis
    constexpr int FNIT = (FNB * FNB + 63) / 64;
    auto fill_run_fwd = [&](const FillRun& fr, int top, const float (&og)[FNIT]) {
      constexpr int NB = FNB;
      float* ol = (float*)mine_lds;            // [NB][NB] opacities (0: no Gaussian of the run waits there)
      if (run_curve != fr.c) {                 // a run of this curve already open goes on
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
          const float a = Tst[q] - T[q];
          acc[q][0] = __builtin_fmaf(rc0, a, acc[q][0]);
          if (C == 3) {
            acc[q][1] = __builtin_fmaf(rc1, a, acc[q][1]);
            acc[q][2] = __builtin_fmaf(rc2, a, acc[q][2]);
          }
          Tst[q] = T[q];
        }
        const float4 pc = w.gcol[fr.g_top];
        rc0 = pc.x;
        rc1 = pc.y;
        rc2 = pc.z;
        run_curve = fr.c;
      }
      const int qx = (quad & 1) * Cfg::SUB, qy = (quad >> 1) * Cfg::SUB;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int it = 0; it < FNIT; ++it)
        if (it * 64 + lane < NB * NB) ol[it * 64 + lane] = og[it];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const double sgd = (double)fr.sigma;
      const float coef = (float)(-0.5 * LOG2E / (sgd * sgd));  // as entry_geometry
      // lane k holds G at squared lattice distance k, as the entry path forms it
      const int gtab = __float_as_int(__builtin_amdgcn_exp2f(coef * (float)lane));
      bool neg = false;
#pragma unroll
      for (int it = 0; it < FNIT; ++it) neg = neg || !(og[it] >= 0.0f);
      const bool nonneg = __ballot(neg) == 0ull;  // no negative (or NaN) opacity in the run
      int nb[PPT];
      const int nb0 = end - ((n_ck + 1) << ck_lg);  // the next chunk boundary still to store
#pragma unroll
      for (int q = 0; q < PPT; ++q) nb[q] = nb0;
      // pixel q's LDS cell and the list position of its own lattice point:
      // those of the lane's first pixel plus q's offset in the lane's block
      int lx0, ly0;
      pixel_of<TILE>(quad, lane, 0, &lx0, &ly0);
      const int cell0 = (ly0 - qy + FR_R) * NB + (lx0 - qx + FR_R);
      const int pb0 = fr.p_lo + (y0 + ly0 - fr.iy0 - fr.j0) * fr.w + (x0 + lx0 - fr.ix0 - fr.i0);
      // the state of pixel q at chunk boundary nb[q] (all positions >= it done)
      auto store_boundary = [&](int q) {
        const float a = Tst[q] - T[q];
        acc[q][0] = __builtin_fmaf(rc0, a, acc[q][0]);
        if (C == 3) {
          acc[q][1] = __builtin_fmaf(rc1, a, acc[q][1]);
          acc[q][2] = __builtin_fmaf(rc2, a, acc[q][2]);
        }
        Tst[q] = T[q];
        float* ckp = w.ckbuf + (int64_t)(ck0 + ((end - nb[q]) >> ck_lg) - 1) * (4 * TILE * TILE);
        const int slot = (quad * PPT + q) * 64 + lane;
        ckp[slot] = T[q];
#pragma unroll
        for (int ch = 0; ch < C; ++ch) {
          ckp[(1 + ch) * TILE * TILE + slot] = acc[q][ch];
          acc[q][ch] = 0.0f;
        }
        nb[q] -= 1 << ck_lg;
      };
      // pixels are independent here: one pixel's whole walk at a time
#pragma unroll
      for (int q = 0; q < PPT; ++q) {
#pragma unroll 1
        for (int dy = FR_R; dy >= -FR_R; --dy) {
          const int dxm = dy * dy <= 4 ? 4 : (dy * dy == 9 ? 3 : 2);  // dx^2 + dy^2 <= FR_R2
          const int roff = cell0 + (q / Cfg::BLK + dy) * NB + q % Cfg::BLK;
          const int rpos = pb0 + (q / Cfg::BLK + dy) * fr.w + q % Cfg::BLK;
          {
            // a row with no Gaussian still to composite for any live pixel
            // changes nothing (chunk boundaries it crosses are stored with
            // the unchanged state at the end)
            const int jr = y0 + ly0 + q / Cfg::BLK + dy - fr.iy0, ir = x0 + lx0 + q % Cfg::BLK - fr.ix0;
            const bool any = T[q] >= eps && jr >= fr.j0 && jr <= fr.j1 && ir + dxm >= fr.i0 && ir - dxm <= fr.i1 &&
                             rpos - dxm <= top;
            if (__ballot(any) == 0ull) continue;
          }
          // the row's opacities first, one LDS wait per row, and its five
          // Gaussian factors (|dx| = 0 .. 4) from the table
          float orow[2 * FR_R + 1], Gr[FR_R + 1];
#pragma unroll
          for (int dx = -FR_R; dx <= FR_R; ++dx) orow[dx + FR_R] = ol[roff + dx];
#pragma unroll
          for (int a = 0; a <= FR_R; ++a) Gr[a] = __int_as_float(__builtin_amdgcn_readlane(gtab, a * a + dy * dy));
          auto cell = [&](int dx, bool check) {
            const float G = Gr[dx < 0 ? -dx : dx];
            const float o = orow[dx + FR_R];
            const int pos = rpos + dx;
            if (check && o != 0.0f)
              while (pos < nb[q]) store_boundary(q);
            const float Tn = T[q] * (1.0f - fminf(amax, o * G));
            const bool live = T[q] >= eps;
            stop[q] = (live && Tn < eps) ? pos : stop[q];
            T[q] = live ? Tn : T[q];
          };
          // a chunk boundary falls in the row of some lane only now and then
          if (__ballot(rpos - dxm < nb[q]) == 0ull) {
            // With no negative opacity in the run T does not grow along the
            // row, so a pixel live at its start whose T ends it at or above
            // eps_T was live at every cell: the row's product, with no stop
            // test, is then the cell-by-cell result.  Only where some pixel
            // stops inside the row is the row taken cell by cell.
            float Tr = T[q];
#pragma unroll
            for (int dx = FR_R; dx >= -FR_R; --dx)
              if (dx <= dxm && dx >= -dxm) Tr = Tr * (1.0f - fminf(amax, orow[dx + FR_R] * Gr[dx < 0 ? -dx : dx]));
            const bool live = T[q] >= eps;
            if (nonneg && __ballot(live && !(Tr >= eps)) == 0ull) {
              T[q] = live ? Tr : T[q];
            } else {
#pragma unroll
              for (int dx = FR_R; dx >= -FR_R; --dx)
                if (dx <= dxm && dx >= -dxm) cell(dx, false);
            }
          } else {
#pragma unroll
            for (int dx = FR_R; dx >= -FR_R; --dx)
              if (dx <= dxm && dx >= -dxm) cell(dx, true);
          }
        }
      }
      // boundaries at or above the run's bottom (none at or below start)
      const int bl = max(fr.p_lo, start + 1);
#pragma unroll
      for (int q = 0; q < PPT; ++q)
        while (nb[q] >= bl) store_boundary(q);
      n_ck = (end - bl) >> ck_lg;
    };
    while (hi > start) {
      if (fill_lattice && __builtin_amdgcn_readfirstlane(e[0].kind) == 1) {
        // the next entry (position hi - 1, lane 0's first) is a fill
        // Gaussian: take its run's remaining positions pixel by pixel
        FillRun fr;
        const int c = __builtin_amdgcn_readfirstlane(e[0].r.curve);
        const float sg = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, e[0].r.sigma)));
        const float rr = ks * sg;
        float og[FNIT];
        bool take = false;
        if (rr * rr >= (float)FR_R2 && rr * rr < (float)(FR_R2 + 5) &&
            fill_run_at(plan, c, __builtin_amdgcn_readfirstlane(e[0].g), __builtin_amdgcn_readfirstlane(e[0].r.local),
                        sg, hi - 1, start, end, 1.0, ks, inv_tile, st, lt, TILE, &fr)) {
          // the opacities and the corner check in flight together
          const int ib = x0 + (quad & 1) * Cfg::SUB - fr.ix0 - FR_R, jb = y0 + (quad >> 1) * Cfg::SUB - fr.iy0 - FR_R;
          fill_gather<FNB, FNIT>(w.gop, gcap, fr, ib, jb, fr.p_lo, hi - 1, 0.0f, og);
          take = fill_corners_ok(idx, fr);
        }
        if (take) {
          const int top = hi - 1;
          hi = fr.p_lo;
          // the next step's loads (as at the start of the list), in flight
          // during the walk
          lo_s = step_floor(hi, start, depth, end, ck_lg);
          nhi = lo_s;
          nlo = step_floor(nhi, start, depth, end, ck_lg);
#pragma unroll
          for (int u = 0; u < E; ++u) {
            const int k = u * 64 + lane;
            load_entry(idx, gs, w.gcol, hi - 1 - k, k < hi - lo_s, &e[u]);
            gnext[u] = k < nhi - nlo ? idx[nhi - 1 - k] : 0;
          }
          fill_run_fwd(fr, top, og);
          bool done = true;
#pragma unroll
          for (int q = 0; q < PPT; ++q) done = done && !(T[q] >= eps);
          if (__ballot(!done) == 0ull) break;  // every pixel of the quadrant has stopped
          continue;
        }
      }
      int cnt = 0;
      bool step_aniso = false;
#pragma unroll
      for (int u = 0; u < E; ++u) {
        const int k = u * 64 + lane;
        const int mypos = hi - 1 - k;
        const bool ok = k < hi - lo_s;
        float4 geo;
        const bool keep = ok && entry_geometry(e[u].r, ox, oy, ks, qbox, &geo);
        const uint64_t m = __ballot(keep);
        if (ANI) step_aniso = step_aniso || __ballot(keep && e[u].kind == 2) != 0ull;
        if (keep) {
          const int dst = cnt + __popcll(m & below);
          FwdRec rec;
          rec.geo = geo;
          rec.op = e[u].r.opacity;
          rec.pos = mypos;
          rec.curve = e[u].r.curve;
          rec.g = e[u].g;
          wrec[dst] = rec;
          wcol[dst] = make_float4(e[u].c0, e[u].c1, e[u].c2, ANI ? (float)e[u].kind : 0.0f);
        }
        cnt += __popcll(m);
      }
      // next step's records (their indices arrived during this step's
      // predecessor) and the indices of the step after, in flight while
      // this step is composited
      const int n2hi = nlo, n2lo = step_floor(n2hi, start, depth, end, ck_lg);
#pragma unroll
      for (int u = 0; u < E; ++u) {
        const int k = u * 64 + lane;
        if (k < nhi - nlo) load_rec(gs, w.gcol, gnext[u], &e[u]);
        gnext[u] = k < n2hi - n2lo ? idx[n2hi - 1 - k] : 0;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (ANI && step_aniso) {
        // tangent-aligned entries of the step take their axis u and ratio r
        for (int i = lane; i < cnt; i += 64) {
          if (wcol[i].w != 2.0f) continue;
          const float4 ax = w.gaux[wrec[i].g];
          float ux, uy, rq;
          aniso_axes(ax, wrec[i].geo.w, &ux, &uy, &rq);
          wrec[i].geo.z = ux;
          wrec[i].geo.w = uy;
          wrec[i].g = __float_as_int(rq);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
      // composited entries that begin a run (their curve differs from the
      // entry before, the first one compared with the previous step's run)
      uint64_t rs[E];
#pragma unroll
      for (int g = 0; g < E; ++g) {
        const int i = 64 * g + lane;
        const int prev = i == 0 ? run_curve : wrec[i > 0 ? i - 1 : 0].curve;
        rs[g] = __ballot(i < cnt && wrec[i < cnt ? i : 0].curve != prev);
      }
      for (int j = 0; j < cnt;) {
        // this segment: j up to the next run start (or the step's end)
        int jend = cnt;
#pragma unroll
        for (int g = E - 1; g >= 0; --g) {
          const int b = j + 1 - 64 * g;  // first bit of group g after j
          const uint64_t m = b <= 0 ? rs[g] : (b < 64 ? rs[g] & (~0ull << b) : 0ull);
          if (m) jend = 64 * g + __builtin_ctzll(m);
        }
        if ((rs[j >> 6] >> (j & 63)) & 1ull) {  // a new run: close the previous one
#pragma unroll
          for (int q = 0; q < PPT; ++q) {
            const float a = Tst[q] - T[q];
            acc[q][0] = __builtin_fmaf(rc0, a, acc[q][0]);
            if (C == 3) {
              acc[q][1] = __builtin_fmaf(rc1, a, acc[q][1]);
              acc[q][2] = __builtin_fmaf(rc2, a, acc[q][2]);
            }
            Tst[q] = T[q];
          }
          const float4 pc = wcol[j];
          rc0 = pc.x;
          rc1 = pc.y;
          rc2 = pc.z;
          run_curve = wrec[j].curve;
          if (ANI) run_kind = __builtin_amdgcn_readfirstlane((int)pc.w);
        }
        if (ANI && run_kind == 2) {
          // tangent-aligned strokes (elliptical Eq. 9)
          const float lim = ANI_CK * ks * ks;
          for (; j < jend; ++j) {
            const float4 gm = wrec[j].geo;
            const float op = wrec[j].op, rq = __int_as_float(wrec[j].g);
            const int pos = wrec[j].pos;
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
              const float dx = px[q] - gm.x, dy = py[q] - gm.y;
              const float a = __builtin_fmaf(dx, gm.z, dy * gm.w);
              const float b = rq * __builtin_fmaf(dy, gm.z, -(dx * gm.w));
              const float m = __builtin_fmaf(a, a, b * b);
              const float G = __builtin_amdgcn_exp2f(-m);
              const bool in = (m <= lim) && (T[q] >= eps);
              const float Tn = T[q] * (1.0f - fminf(amax, op * G));
              stop[q] = (in && Tn < eps) ? pos : stop[q];
              T[q] = in ? Tn : T[q];
            }
          }
        }
#pragma unroll 8
        for (; j < jend; ++j) {
          const float4 gm = wrec[j].geo;
          const float op = wrec[j].op;
          const int pos = wrec[j].pos;
#pragma unroll
          for (int q = 0; q < PPT; ++q) {
            const float dx = px[q] - gm.x, dy = py[q] - gm.y;
            const float d2 = __builtin_fmaf(dx, dx, dy * dy);
            const float G = __builtin_amdgcn_exp2f(gm.w * d2);
            const bool in = (d2 <= gm.z) && (T[q] >= eps);
            const float Tn = T[q] * (1.0f - fminf(amax, op * G));
            stop[q] = (in && Tn < eps) ? pos : stop[q];  // the pixel's last composited position
            T[q] = in ? Tn : T[q];
          }
        }
      }
      bool mine = true;
#pragma unroll
      for (int q = 0; q < PPT; ++q) mine = mine && !(T[q] >= eps);
      hi = nhi;
      lo_s = nlo;
      nhi = n2hi;
      nlo = n2lo;
      if (hi > start && ((end - hi) & ((1 << ck_lg) - 1)) == 0) {
        // at the front of chunk k = (end - hi) / CK: T, and the colour the
        // chunk just finished contributed (the current run closed at the
        // boundary; the sum restarts for the next chunk)
        float* ckp = w.ckbuf + (int64_t)(ck0 + ((end - hi) >> ck_lg) - 1) * (4 * TILE * TILE);
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
          const float a = Tst[q] - T[q];
          acc[q][0] = __builtin_fmaf(rc0, a, acc[q][0]);
          if (C == 3) {
            acc[q][1] = __builtin_fmaf(rc1, a, acc[q][1]);
            acc[q][2] = __builtin_fmaf(rc2, a, acc[q][2]);
          }
          Tst[q] = T[q];
        }
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
          const int slot = (quad * PPT + q) * 64 + lane;
          ckp[slot] = T[q];
#pragma unroll
          for (int c = 0; c < C; ++c) {
            ckp[(1 + c) * TILE * TILE + slot] = acc[q][c];
            acc[q][c] = 0.0f;
          }
        }
        ++n_ck;
      }
      __builtin_amdgcn_wave_barrier();
      if (__ballot(!mine) == 0ull) break;  // every pixel of the quadrant has stopped
    }
#pragma unroll
    for (int q = 0; q < PPT; ++q) {  // close the last run
      const float a = Tst[q] - T[q];
      acc[q][0] = __builtin_fmaf(rc0, a, acc[q][0]);
      if (C == 3) {
        acc[q][1] = __builtin_fmaf(rc1, a, acc[q][1]);
        acc[q][2] = __builtin_fmaf(rc2, a, acc[q][2]);
      }
    }
    // Suffix sums over the chunks, back to front: each boundary's slot
    // receives the colour of everything behind it (the chunks after it; the
    // background is added by the adjoint), a sum of the chunks' own
    // contributions with no cancellation, and the total is the pixel's
    // colour.  Each lane rereads only the slots it wrote itself.
    const int64_t ck_first = (int64_t)ck0 * (4 * TILE * TILE);
    for (int k = n_ck; k >= 1; --k) {
      float* ckp = w.ckbuf + ck_first + (int64_t)(k - 1) * (4 * TILE * TILE);
#pragma unroll
      for (int q = 0; q < PPT; ++q) {
        const int slot = (quad * PPT + q) * 64 + lane;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const float ch = ckp[(1 + c) * TILE * TILE + slot];
          ckp[(1 + c) * TILE * TILE + slot] = acc[q][c];
          acc[q][c] += ch;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      int lx, ly;
      pixel_of<TILE>(quad, lane, q, &lx, &ly);
      const int x = x0 + lx, y = y0 + ly;
      if (x < st.W && y < st.H) {
        const int64_t pix = (int64_t)st.pix_off + (int64_t)y * st.W + x;
        const int64_t plane = (int64_t)st.H * st.W;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const int64_t o = (int64_t)st.pix_off * C + c * plane + (int64_t)y * st.W + x;
          image[o] = __builtin_fmaf(T[q], bg[s * C + c], acc[q][c]);
        }
        Tfin[pix] = T[q];
        nlast[pix] = stop[q];
      }
    }
  }
}

// Totals over the 64 lanes of a wavefront of N per-lane values at once, with
// DPP row shifts and row broadcasts (no LDS traffic): inclusive sums inside
// each row of 16 lanes, then row 0 into row 1, row 2 into row 3, and rows 0-1
// into row 3, so that lane 63 ends with the total.  The N chains are
// interleaved so that each fills the others' data-hazard slots.  Lane i < N
// of the result holds the total of value i (0 elsewhere), ready for one
// N-lane atomic.
template <int N>
__device__ inline float wave_totals_to_lanes(const float (&v)[N]) {
  int x[N];
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = __float_as_int(v[i]);
#define NSP_DPP_STEP(ctrl, rmask, bc)                                                                          \
  _Pragma("unroll") for (int i = 0; i < N; ++i) x[i] = __float_as_int(                                        \
      __int_as_float(x[i]) + __int_as_float(__builtin_amdgcn_update_dpp(0, x[i], ctrl, rmask, 0xf, bc)));
  NSP_DPP_STEP(0x111, 0xf, true)
  NSP_DPP_STEP(0x112, 0xf, true)
  NSP_DPP_STEP(0x114, 0xf, true)
  NSP_DPP_STEP(0x118, 0xf, true)
  NSP_DPP_STEP(0x142, 0xa, false)
  NSP_DPP_STEP(0x143, 0xc, false)
#undef NSP_DPP_STEP
  const int lane = __lane_id();
  float out = 0.0f;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const float t = __int_as_float(__builtin_amdgcn_readlane(x[i], 63));
    out = lane == i ? t : out;
  }
  return out;
}

// Minimum over the wavefront: running minima inside each row of 16 lanes by
// DPP row shifts (a lane with no source keeps its own value), then the four
// rows' last lanes.  Needs no per-lane shuffle addresses.
__device__ inline int wave_min(int v) {
  v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x111, 0xf, 0xf, false));  // row_shr:1
  v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x112, 0xf, 0xf, false));  // row_shr:2
  v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x114, 0xf, 0xf, false));  // row_shr:4
  v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x118, 0xf, 0xf, false));  // row_shr:8
  return min(min(__builtin_amdgcn_readlane(v, 15), __builtin_amdgcn_readlane(v, 31)),
             min(__builtin_amdgcn_readlane(v, 47), __builtin_amdgcn_readlane(v, 63)));
}

// Flushes one wavefront's running per-curve sums into the FP64 per-curve
// accumulators: the colour gradient sum_q dL/dI_c(q) sum(alpha T) of each
// channel (aT: each pixel's sum of alpha T over the run, reset here), and the
// opacity gradient of a stroke curve.
template <int C, int PPT>
__device__ inline void flush_curve(double* gcurve, int c, bool fill, const float (&gI)[PPT][3], float (&aT)[PPT],
                                   float& accO) {
  float v[C + 1];
  v[0] = fill ? 0.0f : accO;
#pragma unroll
  for (int ch = 0; ch < C; ++ch) {
    float a = 0.0f;
#pragma unroll
    for (int q = 0; q < PPT; ++q) a = __builtin_fmaf(gI[q][ch], aT[q], a);
    v[1 + ch] = a;
  }
#pragma unroll
  for (int q = 0; q < PPT; ++q) aT[q] = 0.0f;
  accO = 0.0f;
  const float t = wave_totals_to_lanes<C + 1>(v);
  const int lane = __lane_id();
  if (lane <= C && t != 0.0f) unsafeAtomicAdd(gcurve + 4 * (int64_t)c + lane, (double)t);
}

// Sums the first n (<= RB) parked rows over the 64 lanes and adds each total
// to its target ggrad[g * GG + value] (tgt[row] = (g, value)).  Lane (r, part)
// = (lane / 4, lane % 4) adds up floats part, part + 4, ..., part + 60 of row
// r (lanes of rows past RB add nothing); two DPP row shifts finish the sum in
// the quad's last lane, which issues the atomic.  Every lane of the wavefront
// must call it.
template <int RB>
__device__ inline void flush_rows(const float* park, const int2* tgt, int n, float* __restrict__ ggrad) {
  static_assert(RB <= 16, "four lanes per parked row");
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int lane = __lane_id(), r = lane >> 2, part = lane & 3;
  const float* row = park + r * RB_ROW + part;
  float t = 0.0f;
  if (r < RB) {
#pragma unroll
    for (int j = 0; j < 16; ++j) t += row[4 * j];
  }
  t += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(t), 0x111, 0xf, 0xf, true));  // row_shr:1
  t += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(t), 0x112, 0xf, 0xf, true));  // row_shr:2
  if (part == 3 && r < n && t != 0.0f) {
    const int2 tg = tgt[r];
    unsafeAtomicAdd(ggrad + (int64_t)tg.x * GG + tg.y, t);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Adjoint of the forward blend, one work item per (tile, quadrant, chunk).
// Inside its chunk an item walks back to front, starting from the state the
// forward stored at the chunk's back end (T there, and the colour of
// everything behind it), or from T_final for a pixel that stopped inside the
// chunk.  With K = sum_c dL/dI_c col_c of an entry and B the loss-weighted
// colour behind it, Eq. 8 gives
//   dL/dalpha = T K - B / (1 - alpha),   T the transmittance in front of it.
// Walking back to front, B grows by K alpha T = K (T - T') from each entry
// (T' = T (1 - alpha), the transmittance behind it), and T is recovered as
// T = T' / (1 - alpha).  Over a run of one curve's entries K is fixed, so
// W = B - K T' does not change, and dL/dalpha = -W / (1 - alpha); W is
// re-expressed where K changes.  B is built from the back, a sum of the terms
// behind the entry, so its rounding stays relative to the colour actually
// behind (a front-to-back form B = R - U loses it where T is small).  Per
// Gaussian it accumulates dL/dmu and dL/dsigma for stroke Gaussians and
// dL/do_j for fill Gaussians (whose own opacity carries the SDF); colour
// gradients (and a stroke curve's opacity gradient, its o_j all being o)
// belong to the curve, so each lane keeps running per-curve sums that are
// flushed when the curve changes along the list (and for strokes every FLUSH
// entries).  The entries of a step are cut into runs of one curve with one
// ballot, and each run is composited by a loop for its kind, with no
// per-entry curve test.  Occupancy: six wavefronts per SIMD for one pixel per
// lane at depth 64, four for 32 x 32 tiles at depth 64 (128 VGPRs, unspilled);
// elsewhere the registers decide.
template <int C, int TILE, int E, int KIND>
__global__ __launch_bounds__(BLOCK, bwd_waves(TILE, E, KIND)) void k_blend_bwd(
    nsplat_curves cv, nsplat_params pr, Work w, int n_scenes, int n_tiles, const Gauss* __restrict__ gs,
    const int32_t* __restrict__ ranges, const int32_t* __restrict__ idx, const float* __restrict__ bg,
    const float* __restrict__ dL, const float* __restrict__ Tfin, const int32_t* __restrict__ nlast,
    const int32_t* __restrict__ plan, int64_t gcap, int persistent, int ck_arg) {
  // both block forms in one kernel where a launch can hold both (32 x 32
  // tiles with fills): scenes with fills in 8 x 8 blocks, the others in
  // quadrants
  constexpr bool DUAL = TILE == 32 && (KIND & KIND_FILL) != 0;
  constexpr int FLUSH = 32;
  extern __shared__ __align__(16) char smem[];
  typedef const __attribute__((address_space(4))) int32_t* const_i32;
  const int ck_lg = ck_arg >= 0 ? ck_arg : ((const_i32)w.queue)[Q_CKLG];
  const int depth = min(pr.batch, 64 * E);
  const float amax = pr.alpha_max, ks = pr.k_sigma;
  const float ln2 = (float)LN2;
  constexpr bool ANI = (KIND & KIND_ANI) != 0;
  // fill runs pixel by pixel (see FillRun), in blocks of one pixel per lane
  const bool fill_h1 = (KIND & KIND_FILL) != 0 && read_h(pr) == 1.0f;
  const float inv_tile = 1.0f / (float)TILE;
  const int lane = __lane_id(), wv = threadIdx.x >> 6;
  constexpr int RB = park_rows(TILE, E, KIND);
  char* mine_lds = smem + (size_t)wv * bwd_wave_bytes(TILE, E, KIND);
  float4* wgeo = (float4*)mine_lds;
  float4* wpc = wgeo + 64 * E;
  int4* wmeta = (int4*)(wpc + 64 * E);  // (g, or ~g for fills), curve, list position, 1/sigma^3 bits
  float* park = (float*)(wmeta + 64 * E);  // [RB][RB_ROW] parked gradient values
  int2* ptgt = (int2*)(park + RB * RB_ROW);  // [RB] their (Gaussian, value index) targets
  int n_rows = 0;                          // parked rows (wavefront-uniform)
  const uint64_t below = lanes_below();
  float* __restrict__ ggrad = w.ggrad;
  const const_i32 item_off = (const_i32)w.item_off;  // not written during the kernel: scalar loads
  const int n_items = item_off[n_tiles];
  for (int it = 0;; ++it) {
    const int item = next_item(it, persistent, w.queue);
    if (item >= n_items) break;
    // blend-order position of the item's tile: the last i with item_off[i] <= item
    int tq = 0;
    {
      int lo_t = 0, hi_t = n_tiles - 1;
      while (lo_t < hi_t) {
        const int mid = (lo_t + hi_t + 1) >> 1;
        if (item_off[mid] <= item) lo_t = mid;
        else hi_t = mid - 1;
      }
      tq = lo_t;
    }
    const int r_it = item - item_off[tq];
    const int tile = w.order[tq];
    const int s = scene_of_tile(w.scenes, n_scenes, tile);
    const SceneTab st = w.scenes[s];
    auto item_body = [&](auto cfg) {
    using Cfg = decltype(cfg);
    constexpr int PPT = Cfg::PPT;
    const bool fill_lattice = fill_h1 && PPT == 1;
    const int quad = r_it % Cfg::QUADS, kc = r_it / Cfg::QUADS;
    const int qx = (quad % Cfg::COLS) * Cfg::SUB, qy = (quad / Cfg::COLS) * Cfg::SUB;  // the block's first pixel
    const int lt = tile - st.tile_off;
    const int x0 = (lt % st.tiles_x) * TILE, y0 = (lt / st.tiles_x) * TILE;
    const int start = ranges[2 * tile], end = ranges[2 * tile + 1];
    const int c_hi = end - (kc << ck_lg), c_lo = max(start, end - ((kc + 1) << ck_lg));  // the chunk's positions
    const int64_t plane = (int64_t)st.H * st.W;
    // the forward's state at the chunk's back end (the front of chunk kc + 1),
    // stored when a chunk follows
    const float* ckn = c_lo > start ? w.ckbuf + (int64_t)(w.ck_off[tile] + kc) * (4 * TILE * TILE) : nullptr;
    float px[PPT], py[PPT], T[PPT], Wc[PPT], gI[PPT][3];
    int stop[PPT];
    int my_lo = end;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      int lx, ly;
      adj_pixel<Cfg>(quad, lane, q, &lx, &ly);
      px[q] = (float)lx;
      py[q] = (float)ly;
      T[q] = 1.0f;
      Wc[q] = 0.0f;
      stop[q] = end;  // invalid pixels never take part
#pragma unroll
      for (int c = 0; c < 3; ++c) gI[q][c] = 0.0f;
      if (x0 + lx < st.W && y0 + ly < st.H) {
        const int64_t pix = (int64_t)st.pix_off + (int64_t)(y0 + ly) * st.W + (x0 + lx);
        const float tf = Tfin[pix];
        stop[q] = nlast[pix];
        // a pixel still live behind this chunk starts from the stored state,
        // one that stopped inside it from T_final with only the background
        // behind it (no chunk is stored after a pixel's stop is passed)
        const int slot = Cfg::SPLIT ? fwd_slot<TILE>(lx, ly) : (quad * PPT + q) * 64 + lane;
        float behind[3] = {0.0f, 0.0f, 0.0f};
        T[q] = tf;
        if (stop[q] < c_lo) {  // then c_lo > start, so a chunk follows and ckn is set
          T[q] = ckn[slot];
#pragma unroll
          for (int c = 0; c < C; ++c) behind[c] = ckn[(1 + c) * TILE * TILE + slot];
        }
        float B = 0.0f;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const int64_t o = (int64_t)st.pix_off * C + c * plane + (int64_t)(y0 + ly) * st.W + (x0 + lx);
          gI[q][c] = dL[o];
          B = __builtin_fmaf(gI[q][c], __builtin_fmaf(tf, bg[s * C + c], behind[c]), B);
        }
        Wc[q] = B;  // W = B - K T' with no curve yet (K = 0)
        my_lo = min(my_lo, stop[q]);
      }
    }
    // positions below every pixel's stopping position take no part
    const int lo = max(wave_min(my_lo), c_lo);
    if (c_hi <= lo) return;
    int cur = -1, since = 0;
    bool cur_fill = false, cur_aniso = false;
    // per pixel: K of the current curve, W (fixed over a run of one curve),
    // and the run's sum of alpha T (the curve's colour gradient is dL/dI_c
    // times it)
    float Kc[PPT], aT[PPT], accO = 0.0f;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      Kc[q] = 0.0f;
      aT[q] = 0.0f;
    }
    const double ox = (double)x0 + 0.5, oy = (double)y0 + 0.5;
    // back to front over the chunk's positions lo up to c_hi - 1, in steps
    // of `depth` (each lane loads one entry per 64 of a step)
    Entry e[E];
    int s_lo = lo, s_hi = min(c_hi, lo + depth);
#pragma unroll
    for (int u = 0; u < E; ++u) {
      const int k = u * 64 + lane;
      load_entry(idx, gs, w.gcol, s_lo + k, k < s_hi - s_lo, &e[u]);
    }
    // One fill run's positions p0 .. p1 at h = 1, back to front for each
    // pixel over its in-disc lattice neighbours (the reverse of the forward's
    // walk), with the per-pixel arithmetic of the entry-by-entry path; each
    // Gaussian's dL/do_j is summed over the lanes in LDS and added with one
    // atomic.
    constexpr int BNB = Cfg::SUB + 2 * FR_R;  // lattice neighbourhood of the pixel block, per axis
    constexpr int BNIT = (BNB * BNB + 63) / 64;
    auto fill_run_bwd = [&](const FillRun& fr, int p0, int p1, const float (&og)[BNIT]) {
      // (one pixel per lane: lane (l & 7, l >> 3) of the 8 x 8 pixel
      // block; fill_lattice is false otherwise)
      constexpr int NB = BNB;                  // 16 cells per axis
      constexpr int NS = FR_NS;                // LDS row stride (conflict-free rows)
      float* ol = (float*)mine_lds;  // [NB][NS] opacities (0: no Gaussian at p0 .. p1 there)
      float* gl = park;              // [NB][NS] dL/do_j
      if (n_rows > 0) {
        flush_rows<RB>(park, ptgt, n_rows, ggrad);
        n_rows = 0;
      }
      if (cur != fr.c) {  // a new curve: close the previous one, W for the new K
        if (cur >= 0) flush_curve<C, PPT>(w.gcurve, cur, cur_fill, gI, aT, accO);
        const float4 pc = w.gcol[fr.g_top];
        const float col[3] = {pc.x, pc.y, pc.z};
        float K = 0.0f;
#pragma unroll
        for (int ch = 0; ch < C; ++ch) K = __builtin_fmaf(gI[0][ch], col[ch], K);
        Wc[0] = __builtin_fmaf(-K, T[0], __builtin_fmaf(Kc[0], T[0], Wc[0]));
        Kc[0] = K;
        cur = fr.c;
        cur_fill = true;
        cur_aniso = false;
        since = 0;
      }
      const int ib = x0 + qx - fr.ix0 - FR_R, jb = y0 + qy - fr.iy0 - FR_R;  // window index of cell (0, 0)
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // an absent cell composites as a zero opacity (alpha 0, T unchanged);
      // its dL/do_j sum is dropped by the presence bits
      int pm = 0;
#pragma unroll
      for (int it = 0; it < BNIT; ++it) {
        const int sl = it * 64 + lane;
        if (sl < NB * NB) {
          const bool pres = og[it] == og[it];
          ol[(sl / NB) * NS + sl % NB] = pres ? og[it] : 0.0f;
          gl[(sl / NB) * NS + sl % NB] = 0.0f;
          pm |= (int)pres << it;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const double sgd = (double)fr.sigma;
      const float coef = (float)(-0.5 * LOG2E / (sgd * sgd));  // as entry_geometry
      // lane k holds G at squared lattice distance k, as the entry path forms it
      const int gtab = __float_as_int(__builtin_amdgcn_exp2f(coef * (float)lane));
      const float nW = -Wc[0];  // dL/dalpha (1 - alpha) over the run
      const int lx = lane & 7, ly = lane >> 3;
      const bool col0 = lx == 0, col7 = lx == 7;
      const int pb0 = fr.p_lo + (y0 + qy + ly - fr.iy0 - fr.j0) * fr.w + (x0 + qx + lx - fr.ix0 - fr.i0);
#pragma unroll 1
      for (int dy = -FR_R; dy <= FR_R; ++dy) {
        const int dxm = dy * dy <= 4 ? 4 : (dy * dy == 9 ? 3 : 2);  // dx^2 + dy^2 <= FR_R2
        const int roff = (ly + dy + FR_R) * NS + lx + FR_R;         // this pixel's cell in row dy
        const int rpos = pb0 + dy * fr.w;
        {
          // a row with no Gaussian of p0 .. p1 at or in front of any pixel's
          // stop adds nothing
          const int jr = y0 + qy + ly + dy - fr.iy0, ir = x0 + qx + lx - fr.ix0;
          const bool any = jr >= fr.j0 && jr <= fr.j1 && ir + dxm >= fr.i0 && ir - dxm <= fr.i1 &&
                           rpos + dxm >= max(p0, stop[0]) && rpos - dxm <= p1;
          if (__ballot(any) == 0ull) continue;
        }
        // the row's opacities first, one LDS wait per row (each becomes the
        // cell's dL/do_j in place), and its five Gaussian factors
        float v[2 * FR_R + 1], Gr[FR_R + 1];
#pragma unroll
        for (int dx = -FR_R; dx <= FR_R; ++dx) v[dx + FR_R] = ol[roff + dx];
#pragma unroll
        for (int a = 0; a <= FR_R; ++a) Gr[a] = __int_as_float(__builtin_amdgcn_readlane(gtab, a * a + dy * dy));
        const int sd = stop[0] - rpos;  // cells at dx >= sd lie at or behind the pixel's stop
#pragma unroll
        for (int dx = -FR_R; dx <= FR_R; ++dx) {
          const float o = v[dx + FR_R];
          v[dx + FR_R] = 0.0f;
          if (dx > dxm || dx < -dxm) continue;
          // a cell in front of the stop takes part with G = 0: alpha 0, T
          // and alpha T unchanged, no gradient
          const float G = dx >= sd ? Gr[dx < 0 ? -dx : dx] : 0.0f;
          const float oG = o * G;
          const bool lt = oG < amax;
          const float alpha = fminf(oG, amax);  // lt ? oG : amax, also for a NaN oG
          const float r = __builtin_amdgcn_rcpf(1.0f - alpha);
          T[0] *= r;
          aT[0] = __builtin_fmaf(alpha, T[0], aT[0]);
          v[dx + FR_R] = lt ? nW * r * G : 0.0f;  // dL/do_j of the cell at dx
        }
        // the row's cells get their sums over the pixels of each lane row
        // by two sliding sums along the row (DPP shifts by one lane, 8-lane
        // groups kept apart): P ends with cell lx - 4, Q with cell lx + 4
        float P = v[2 * FR_R], Q = v[0];
#pragma unroll
        for (int k = 1; k <= 2 * FR_R; ++k) {
          const float ps = col7 ? 0.0f : P, qs = col0 ? 0.0f : Q;
          P = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(ps), 0x111, 0xf, 0xf, true)) +
              v[2 * FR_R - k];  // row_shr:1
          Q = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(qs), 0x101, 0xf, 0xf, true)) +
              v[k];  // row_shl:1
        }
        const int crow = (ly + dy + FR_R) * NS;  // cell row of this lane row
        gl[crow + lx] += P;                      // cell column lx - 4
        gl[crow + lx + 2 * FR_R] += Q;           // cell column lx + 4
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int it = 0; it < (NB * NB + 63) / 64; ++it) {
        const int sl = it * 64 + lane;
        if (sl >= NB * NB) continue;
        const float val = gl[(sl / NB) * NS + sl % NB];
        if (((pm >> it) & 1) && val != 0.0f) {
          const int j = jb + sl / NB, i = ib + sl % NB;
          unsafeAtomicAdd(ggrad + ((int64_t)fr.goff + (int64_t)j * fr.nx + i) * GG + 3, val);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    while (s_lo < c_hi) {
      if (fill_lattice && __builtin_amdgcn_readfirstlane(e[0].kind) == 1) {
        // the next entry (position s_lo, lane 0's first) is a fill Gaussian:
        // take its run's positions in this chunk pixel by pixel
        FillRun fr;
        const int c = __builtin_amdgcn_readfirstlane(e[0].r.curve);
        const float sg = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, e[0].r.sigma)));
        const float rr = ks * sg;
        float og[BNIT];
        bool take = false;
        const int p0 = s_lo;
        int p1 = 0;
        if (rr * rr >= (float)FR_R2 && rr * rr < (float)(FR_R2 + 5) &&
            fill_run_at(plan, c, __builtin_amdgcn_readfirstlane(e[0].g), __builtin_amdgcn_readfirstlane(e[0].r.local),
                        sg, s_lo, start, end, 1.0, ks, inv_tile, st, lt, TILE, &fr)) {
          // the opacities and the corner check in flight together
          p1 = min(fr.p_hi, c_hi - 1);
          const int ib = x0 + qx - fr.ix0 - FR_R, jb = y0 + qy - fr.iy0 - FR_R;
          fill_gather<BNB, BNIT>(w.gop, gcap, fr, ib, jb, s_lo, p1, __builtin_nanf(""), og);
          take = fill_corners_ok(idx, fr);
        }
        if (take) {
          // the next step's loads in flight during the walk
          s_lo = p1 + 1;
          s_hi = min(c_hi, s_lo + depth);
#pragma unroll
          for (int u = 0; u < E; ++u) {
            const int k = u * 64 + lane;
            load_entry(idx, gs, w.gcol, s_lo + k, k < s_hi - s_lo, &e[u]);
          }
          fill_run_bwd(fr, p0, p1, og);
          continue;
        }
      }
      int cnt = 0;
      // pixels that take part somewhere in this step (their stop lies below
      // its top); walking back to front the set only grows.  Entries that
      // reach none of them are dropped.
      bool lv = false, step_aniso = false;
#pragma unroll
      for (int q = 0; q < PPT; ++q) lv = lv || (stop[q] < s_hi);
      const Box box = live_box_of<Cfg>(qx, qy, __ballot(lv));
#pragma unroll
      for (int u = 0; u < E; ++u) {
        const int k = u * 64 + lane;
        const int mypos = s_lo + k;
        const bool ok = k < s_hi - s_lo;
        float4 geo;
        const bool keep = ok && entry_geometry(e[u].r, ox, oy, ks, box, &geo);
        const uint64_t m = __ballot(keep);
        if (ANI) step_aniso = step_aniso || __ballot(keep && e[u].kind == 2) != 0ull;
        if (keep) {
          const int dst = cnt + __popcll(m & below);
          const double sg = (double)e[u].r.sigma;
          // tangent-aligned entries: -1 (negative: the kind) in place of 1 / sigma^3
          const float wbits = (ANI && e[u].kind == 2) ? -1.0f : (float)(1.0 / (sg * sg * sg));
          wgeo[dst] = geo;
          wpc[dst] = make_float4(e[u].r.opacity, e[u].c0, e[u].c1, e[u].c2);
          wmeta[dst] = make_int4(e[u].kind == 1 ? ~e[u].g : e[u].g, e[u].r.curve, mypos, __float_as_int(wbits));
        }
        cnt += __popcll(m);
      }
      const int n_lo = s_hi, n_hi = min(c_hi, s_hi + depth);
#pragma unroll
      for (int u = 0; u < E; ++u) {  // next step, in flight while this one is processed
        const int k = u * 64 + lane;
        load_entry(idx, gs, w.gcol, n_lo + k, k < n_hi - n_lo, &e[u]);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (ANI && step_aniso) {
        // tangent-aligned entries of the step take their axis u (in place of
        // the support radius and coefficient) and -r (in place of the kind)
        for (int i = lane; i < cnt; i += 64) {
          const int4 mt = wmeta[i];
          if (mt.x < 0 || mt.w >= 0) continue;
          const float4 ax = w.gaux[mt.x];
          float ux, uy, rq;
          aniso_axes(ax, wgeo[i].w, &ux, &uy, &rq);
          wgeo[i].z = ux;
          wgeo[i].w = uy;
          wmeta[i].w = __float_as_int(-rq);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
      // entries that begin a run (their curve differs from the entry processed
      // before them, the first one compared with the previous step's curve)
      uint64_t rs[E];
#pragma unroll
      for (int g = 0; g < E; ++g) {
        const int i = 64 * g + lane;
        const int prev = i == 0 ? cur : wmeta[i > 0 ? i - 1 : 0].y;
        rs[g] = __ballot(i < cnt && wmeta[i < cnt ? i : 0].y != prev);
      }
      const float* wop = (const float*)wpc;  // opacities
      for (int j = 0; j < cnt;) {
        // this segment: j up to the next run start (or the step's end)
        int jend = cnt;
#pragma unroll
        for (int g = E - 1; g >= 0; --g) {
          const int b = j + 1 - 64 * g;  // first bit of group g after j
          const uint64_t m = b <= 0 ? rs[g] : (b < 64 ? rs[g] & (~0ull << b) : 0ull);
          if (m) jend = 64 * g + __builtin_ctzll(m);
        }
        if ((rs[j >> 6] >> (j & 63)) & 1ull) {  // a new curve: close the previous one
          if (cur >= 0) flush_curve<C, PPT>(w.gcurve, cur, cur_fill, gI, aT, accO);
          const int4 mt = wmeta[j];
          const float4 pc = wpc[j];
          const float col[3] = {pc.y, pc.z, pc.w};
#pragma unroll
          for (int q = 0; q < PPT; ++q) {
            float K = 0.0f;
#pragma unroll
            for (int c = 0; c < C; ++c) K = __builtin_fmaf(gI[q][c], col[c], K);
            // B = W + K_old T' is unchanged; W re-expressed with the new K
            Wc[q] = __builtin_fmaf(-K, T[q], __builtin_fmaf(Kc[q], T[q], Wc[q]));
            Kc[q] = K;
          }
          cur = __builtin_amdgcn_readfirstlane(mt.y);
          cur_fill = __builtin_amdgcn_readfirstlane(mt.x) < 0;
          cur_aniso = ANI && !cur_fill && __builtin_amdgcn_readfirstlane(mt.w) < 0;
          since = 0;
        }
        if (ANI && cur_aniso) {
          // tangent-aligned stroke Gaussians: dL/dmu (2), dL/dsigma, dL/dsp
          // and dL/dtheta (t = (cos theta, sin theta)) parked in five rows.
          // With h = dL/dG G / ck: dG/dmu = (a u - b r u^perp) 2 ln 2 G, and so
          // on (the partials of exp(-(d_t^2 / sigma^2 + d_n^2 / sp^2) / 2)
          // rewritten in a, b).
          const float lim = ANI_CK * ks * ks;
          const float two_ln2 = 2.0f * ln2;
          for (; j < jend; ++j) {
            if (since >= FLUSH) {
              flush_curve<C, PPT>(w.gcurve, cur, false, gI, aT, accO);
              since = 0;
            }
            ++since;
            const float4 gm = wgeo[j];
            const float op = wop[4 * j];
            const int4 mt = wmeta[j];
            const float rq = -__int_as_float(mt.w);
            const float isg = __builtin_sqrtf(__builtin_fmaf(gm.z, gm.z, gm.w * gm.w)) * (1.0f / ANI_SQRT_CK);
            const float isp = isg * rq;           // 1 / sp
            const float rr = rq - 1.0f / rq;      // sigma / sp - sp / sigma
            const float rux = rq * gm.z, ruy = rq * gm.w;
            float v[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
            bool act = false;
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
              const float dx = px[q] - gm.x, dy = py[q] - gm.y;
              const float a = __builtin_fmaf(dx, gm.z, dy * gm.w);
              const float b = rq * __builtin_fmaf(dy, gm.z, -(dx * gm.w));
              const float m = __builtin_fmaf(a, a, b * b);
              const bool in = (mt.z >= stop[q]) && (m <= lim);
              act = act || in;
              const float G = __builtin_amdgcn_exp2f(-m);
              const float oG = op * G;
              const bool lt = oG < amax;
              const float alpha = in ? fminf(oG, amax) : 0.0f;  // = lt ? oG : amax
              const float r = __builtin_amdgcn_rcpf(1.0f - alpha);
              const float dLda = (in && lt) ? -Wc[q] * r : 0.0f;
              T[q] = in ? T[q] * r : T[q];
              aT[q] = __builtin_fmaf(alpha, T[q], aT[q]);
              v[5] = __builtin_fmaf(dLda, G, v[5]);  // dL/do_j
              const float h = dLda * op * G * two_ln2;
              v[0] = __builtin_fmaf(h, __builtin_fmaf(a, gm.z, -(b * ruy)), v[0]);
              v[1] = __builtin_fmaf(h, __builtin_fmaf(a, gm.w, b * rux), v[1]);
              v[2] = __builtin_fmaf(h * a, a * isg, v[2]);
              v[3] = __builtin_fmaf(h * b, b * isp, v[3]);
              v[4] = __builtin_fmaf(h * a, b * rr, v[4]);
            }
            if (__ballot(act) == 0ull) continue;
            if (n_rows + 5 > RB) {
              flush_rows<RB>(park, ptgt, n_rows, ggrad);
              n_rows = 0;
            }
            accO += v[5];
#pragma unroll
            for (int i = 0; i < 5; ++i) park[(n_rows + i) * RB_ROW + lane] = v[i];
            if (lane < 5) ptgt[n_rows + lane] = make_int2(mt.x, lane);
            n_rows = __builtin_amdgcn_readfirstlane(n_rows + 5);
          }
        } else if (cur_fill) {
          // fill Gaussians: one value each (dL/do_j), parked in one row;
          // entries are evaluated two at a time (independent work of the
          // pair overlaps) and parked in order
          auto fill_eval = [&](int jj, float& v3, bool& act, int& gneg) {
            const float4 gm = wgeo[jj];
            const float op = wop[4 * jj];
            const int4 mt = wmeta[jj];
            gneg = mt.x;
            v3 = 0.0f;
            act = false;
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
              const float dx = px[q] - gm.x, dy = py[q] - gm.y;
              const float d2 = __builtin_fmaf(dx, dx, dy * dy);
              const bool in = (mt.z >= stop[q]) && (d2 <= gm.z);
              act = act || in;
              const float G = __builtin_amdgcn_exp2f(gm.w * d2);
              const float oG = op * G;
              const bool lt = oG < amax;
              const float alpha = in ? fminf(oG, amax) : 0.0f;  // = lt ? oG : amax
              const float r = __builtin_amdgcn_rcpf(1.0f - alpha);
              // dL/dalpha = (T' K - B) / (1 - alpha) = -W / (1 - alpha)
              const float dLda = (in && lt) ? -Wc[q] * r : 0.0f;
              T[q] = in ? T[q] * r : T[q];  // the transmittance in front of the entry
              aT[q] = __builtin_fmaf(alpha, T[q], aT[q]);
              v3 = __builtin_fmaf(dLda, G, v3);  // dL/do_j
            }
          };
          auto fill_park = [&](float v3, bool act, int gneg) {
            if (__ballot(act) == 0ull) return;
            if (n_rows + 1 > RB) {
              flush_rows<RB>(park, ptgt, n_rows, ggrad);
              n_rows = 0;
            }
            park[n_rows * RB_ROW + lane] = v3;
            if (lane == 0) ptgt[n_rows] = make_int2(~gneg, 3);
            n_rows = __builtin_amdgcn_readfirstlane(n_rows + 1);
          };
          for (; j + 1 < jend; j += 2) {
            float va, vb;
            bool aa, ab;
            int ga, gb;
            fill_eval(j, va, aa, ga);
            fill_eval(j + 1, vb, ab, gb);
            fill_park(va, aa, ga);
            fill_park(vb, ab, gb);
          }
          if (j < jend) {
            float va;
            bool aa;
            int ga;
            fill_eval(j, va, aa, ga);
            fill_park(va, aa, ga);
            ++j;
          }
        } else {
          // stroke Gaussians: dL/dmu (2) and dL/dsigma parked in three rows;
          // dL/do_j summed per lane into the curve's opacity gradient, which
          // is flushed every FLUSH entries to keep that FP32 sum short
          for (; j < jend; ++j) {
            if (since >= FLUSH) {
              flush_curve<C, PPT>(w.gcurve, cur, false, gI, aT, accO);
              since = 0;
            }
            ++since;
            const float4 gm = wgeo[j];
            const float op = wop[4 * j];
            const int4 mt = wmeta[j];
            const float is3 = __int_as_float(mt.w);
            float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            bool act = false;
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
              const float dx = px[q] - gm.x, dy = py[q] - gm.y;
              const float d2 = __builtin_fmaf(dx, dx, dy * dy);
              const bool in = (mt.z >= stop[q]) && (d2 <= gm.z);
              act = act || in;
              const float G = __builtin_amdgcn_exp2f(gm.w * d2);
              const float oG = op * G;
              const bool lt = oG < amax;
              const float alpha = in ? fminf(oG, amax) : 0.0f;  // = lt ? oG : amax
              const float r = __builtin_amdgcn_rcpf(1.0f - alpha);
              const float dLda = (in && lt) ? -Wc[q] * r : 0.0f;
              T[q] = in ? T[q] * r : T[q];
              aT[q] = __builtin_fmaf(alpha, T[q], aT[q]);
              v[3] = __builtin_fmaf(dLda, G, v[3]);  // dL/do_j
              const float dG = dLda * op;
              const float dd2 = dG * G * gm.w * ln2;  // d exp2(a d2) / d d2 = G a ln 2
              v[0] = __builtin_fmaf(-2.0f * dx, dd2, v[0]);
              v[1] = __builtin_fmaf(-2.0f * dy, dd2, v[1]);
              v[2] = __builtin_fmaf(dG * G, d2 * is3, v[2]);
            }
            if (__ballot(act) == 0ull) continue;
            if (n_rows + 3 > RB) {
              flush_rows<RB>(park, ptgt, n_rows, ggrad);
              n_rows = 0;
            }
            accO += v[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) park[(n_rows + i) * RB_ROW + lane] = v[i];
            if (lane < 3) ptgt[n_rows + lane] = make_int2(mt.x, lane);
            n_rows = __builtin_amdgcn_readfirstlane(n_rows + 3);
          }
        }
      }
      __builtin_amdgcn_wave_barrier();
      s_lo = n_lo;
      s_hi = n_hi;
    }
    if (n_rows > 0) {
      flush_rows<RB>(park, ptgt, n_rows, ggrad);
      n_rows = 0;
    }
    if (cur >= 0) flush_curve<C, PPT>(w.gcurve, cur, cur_fill, gI, aT, accO);
    };
    if constexpr (DUAL) {
      if (st.fills) item_body(AdjCfg<TILE, true>{});
      else item_body(AdjCfg<TILE, false>{});
    } else {
      item_body(AdjCfg<TILE, false>{});
    }
  }
}

__global__ void k_reset_queue(int32_t* q) {
  if (threadIdx.x < 4 && blockIdx.x == 0) q[threadIdx.x] = 0;
}

template <class K>
int resident_grid(K kernel, int n_blocks, int n_cu, size_t lds) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, BLOCK, lds) != hipSuccess || per_cu < 1)
    per_cu = 1;
  const int g = per_cu * n_cu;
  return g < n_blocks ? g : n_blocks;
}

inline int depth_factor(int batch) { return batch <= 64 ? 1 : (batch <= 128 ? 2 : 4); }

template <int C, int TILE, int E, int KIND>
hipError_t fwd_t(const Launch& L, float* image, float* T_final, int32_t* n_last, int persistent) {
  const int n_items = (int)L.n_tiles * TileCfg<TILE>::QUADS;
  if (n_items <= 0) return hipSuccess;
  const size_t lds = (size_t)WPB * 64 * E * FWD_ENTRY_BYTES;
  int grid = (n_items + WPB - 1) / WPB;
  if (persistent) {
    grid = resident_grid(k_blend_fwd<C, TILE, E, KIND>, grid, L.n_cu, lds);
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, L.stream, L.w.queue);
  }
  Phase ph(L, NSPLAT_T_BLEND_FWD);
  hipLaunchKernelGGL((k_blend_fwd<C, TILE, E, KIND>), dim3(grid), dim3(BLOCK), lds, L.stream, *L.cv, *L.pr, L.w,
                     L.sc->n_scenes, n_items, (const Gauss*)L.bf->gauss, L.bf->ranges, L.bf->idx, L.sc->bg, image,
                     T_final, n_last, L.bf->plan, (int64_t)L.bf->caps.gauss, persistent, L.ck_lg);
  return hipGetLastError();
}

template <int C, int TILE, int E, int KIND>
hipError_t bwd_t(const Launch& L, const float* dL, const float* T_final, const int32_t* n_last, int persistent) {
  if (L.n_tiles <= 0) return hipSuccess;
  // the item count lives on the device; the grid covers its bound
  // sum over tiles of QUADS * ceil(len / CK) <= QUADS * (pairs / CK + tiles)
  const int64_t max_items =
      (int64_t)adj_blocks(TILE, (KIND & KIND_FILL) != 0) * ((L.bf->caps.pairs >> (L.ck_lg >= 0 ? L.ck_lg : 9)) +
                                                             L.n_tiles);
  const size_t lds = (size_t)WPB * bwd_wave_bytes(TILE, E, KIND);
  int grid = (int)((max_items + WPB - 1) / WPB);
  if (persistent) {
    grid = resident_grid(k_blend_bwd<C, TILE, E, KIND>, grid, L.n_cu, lds);
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, L.stream, L.w.queue);
  }
  Phase ph(L, NSPLAT_T_BLEND_BWD);
  hipLaunchKernelGGL((k_blend_bwd<C, TILE, E, KIND>), dim3(grid), dim3(BLOCK), lds, L.stream, *L.cv, *L.pr, L.w,
                     L.sc->n_scenes, (int)L.n_tiles, (const Gauss*)L.bf->gauss, L.bf->ranges, L.bf->idx, L.sc->bg,
                     dL, T_final, n_last, L.bf->plan, (int64_t)L.bf->caps.gauss, persistent, L.ck_lg);
  return hipGetLastError();
}

// The tangent-aligned kind and the fill-run walk are compiled in only for
// batches that declare such curves (nsplat_curves.any_flags), so that the
// other batches run without their branches and registers.
inline int kinds_of(const Launch& L) {
  return ((L.cv->any_flags & NSPLAT_ANISO) ? KIND_ANI : 0) | ((L.cv->any_flags & NSPLAT_FILLED) ? KIND_FILL : 0);
}

template <int C, int TILE, int E>
hipError_t fwd_k(const Launch& L, float* image, float* T_final, int32_t* n_last, int persistent) {
  switch (kinds_of(L)) {
    case 0: return fwd_t<C, TILE, E, 0>(L, image, T_final, n_last, persistent);
    case KIND_ANI: return fwd_t<C, TILE, E, KIND_ANI>(L, image, T_final, n_last, persistent);
    case KIND_FILL: return fwd_t<C, TILE, E, KIND_FILL>(L, image, T_final, n_last, persistent);
    default: return fwd_t<C, TILE, E, KIND_ANI | KIND_FILL>(L, image, T_final, n_last, persistent);
  }
}

template <int C, int TILE>
hipError_t fwd_d(const Launch& L, float* image, float* T_final, int32_t* n_last, int persistent) {
  switch (depth_factor(L.pr->batch)) {
    case 1: return fwd_k<C, TILE, 1>(L, image, T_final, n_last, persistent);
    case 2: return fwd_k<C, TILE, 2>(L, image, T_final, n_last, persistent);
    default: return fwd_k<C, TILE, 4>(L, image, T_final, n_last, persistent);
  }
}

template <int C, int TILE, int E>
hipError_t bwd_k(const Launch& L, const float* dL, const float* T_final, const int32_t* n_last, int persistent) {
  switch (kinds_of(L)) {
    case 0: return bwd_t<C, TILE, E, 0>(L, dL, T_final, n_last, persistent);
    case KIND_ANI: return bwd_t<C, TILE, E, KIND_ANI>(L, dL, T_final, n_last, persistent);
    case KIND_FILL: return bwd_t<C, TILE, E, KIND_FILL>(L, dL, T_final, n_last, persistent);
    default: return bwd_t<C, TILE, E, KIND_ANI | KIND_FILL>(L, dL, T_final, n_last, persistent);
  }
}

template <int C, int TILE>
hipError_t bwd_d(const Launch& L, const float* dL, const float* T_final, const int32_t* n_last, int persistent) {
  switch (depth_factor(L.pr->batch)) {
    case 1: return bwd_k<C, TILE, 1>(L, dL, T_final, n_last, persistent);
    case 2: return bwd_k<C, TILE, 2>(L, dL, T_final, n_last, persistent);
    default: return bwd_k<C, TILE, 4>(L, dL, T_final, n_last, persistent);
  }
}

}  // namespace

hipError_t launch_blend_fwd(const Launch& L, float* image, float* T_final, int32_t* n_last, int persistent) {
  const int C = L.cv->channels, t = L.pr->tile;
  if (C == 1) {
    if (t == 8) return fwd_d<1, 8>(L, image, T_final, n_last, persistent);
    if (t == 16) return fwd_d<1, 16>(L, image, T_final, n_last, persistent);
    return fwd_d<1, 32>(L, image, T_final, n_last, persistent);
  }
  if (t == 8) return fwd_d<3, 8>(L, image, T_final, n_last, persistent);
  if (t == 16) return fwd_d<3, 16>(L, image, T_final, n_last, persistent);
  return fwd_d<3, 32>(L, image, T_final, n_last, persistent);
}

hipError_t launch_blend_bwd(const Launch& L, const float* dL, const float* T_final, const int32_t* n_last,
                            int persistent) {
  const int C = L.cv->channels, t = L.pr->tile;
  if (C == 1) {
    if (t == 8) return bwd_d<1, 8>(L, dL, T_final, n_last, persistent);
    if (t == 16) return bwd_d<1, 16>(L, dL, T_final, n_last, persistent);
    return bwd_d<1, 32>(L, dL, T_final, n_last, persistent);
  }
  if (t == 8) return bwd_d<3, 8>(L, dL, T_final, n_last, persistent);
  if (t == 16) return bwd_d<3, 16>(L, dL, T_final, n_last, persistent);
  return bwd_d<3, 32>(L, dL, T_final, n_last, persistent);
}

}  // namespace nsp
