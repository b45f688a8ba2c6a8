// C ABI of the library (declared in include/nsplat.h): context, host-side
// argument checks, workspace carve-out, the four render-path entry points,
// the annealing / loss helpers and the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "nsplat_internal.h"

struct nsplat_ctx {
  int device = 0;
  int n_cu = 256;
  std::string err;
  nsp::Timer timer;
  // tile side, chunk length and adjoint pixel blocks per chunk of the last
  // nsplat_bin on each workspace (the tile lists, checkpoint offsets and
  // adjoint items in it are laid out for them)
  struct BinState {
    const void* ws;
    int tile, chunk, blocks;
  };
  std::vector<BinState> bin_tile;
  // what the scene table of each workspace was last built for (tile side,
  // N_L factor, scene sizes), so that nsplat_bin need not rebuild it
  struct SceneSig {
    const void* ws;
    int tile;
    float nl_factor;
    std::vector<int32_t> hw;
  };
  std::vector<SceneSig> scene_sig;
};

namespace nsp {
hipError_t launch_zero_grads(const Launch& L);

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

Layout workspace_layout(const nsplat_curves* cv, const nsplat_scenes* sc, const nsplat_caps* caps) {
  Layout lay;
  const int64_t N = cv->n_curves, K = cv->n_keys, T = cv->n_taus, S = sc->n_scenes;
  const int64_t gcap = caps->gauss, pcap = caps->pairs, bcap = caps->boundary;
  lay.sort_blocks = (pcap + SORT_ITEMS - 1) / SORT_ITEMS;
  const int64_t tiles8 = nsplat_num_tiles(sc, 8);
  // the one-digit binning's per-block tile counts: RADIX_MAX rows and a row
  // of block totals, one column per FB_ITEMS Gaussians
  const int64_t fb_hist = (int64_t)(RADIX_MAX + 1) * std::max<int64_t>((gcap + FB_ITEMS - 1) / FB_ITEMS, 1);
  const int64_t hist_n = std::max<int64_t>((int64_t)RADIX_MAX * std::max<int64_t>(lay.sort_blocks, 1), fb_hist);
  const int64_t scan_n = std::max<int64_t>({gcap, hist_n, tiles8 + 1, 1});
  lay.scan_blocks = (scan_n + SCAN_ITEMS - 1) / SCAN_ITEMS;
  const size_t sizes[N_WS] = {
      sizeof(double) * (size_t)(T + N * KNOT_PAD),         // knots
      sizeof(double) * (size_t)N,                          // L
      sizeof(int32_t) * (size_t)(N + 1),                   // goff
      sizeof(double2) * (size_t)std::max<int64_t>(bcap, 1),  // bpts
      sizeof(SceneTab) * (size_t)(S + 1),                  // scenes
      sizeof(uint32_t) * (size_t)(gcap + 1),               // gcnt
      sizeof(uint32_t) * (size_t)std::max<int64_t>(pcap, 1),  // keys0
      sizeof(uint32_t) * (size_t)std::max<int64_t>(pcap, 1),  // keys1
      sizeof(uint32_t) * (size_t)std::max<int64_t>(pcap, 1),  // vals1
      sizeof(uint32_t) * (size_t)hist_n,                   // hist
      sizeof(uint32_t) * (size_t)(lay.scan_blocks + 1),    // scan_tmp
      sizeof(float) * GG * (size_t)std::max<int64_t>(gcap, 1),  // ggrad
      sizeof(double) * 4 * (size_t)(K + N * CP_PAD),       // gcp
      sizeof(double) * (size_t)(T + N * KNOT_PAD),         // gknot
      sizeof(double) * 4 * (size_t)N,                      // gcurve
      sizeof(double2) * (size_t)std::max<int64_t>(bcap, 1),  // gb
      sizeof(int32_t) * 64,                                // queue
      sizeof(int32_t) * (size_t)std::max<int64_t>(gcap, 1),  // aux
      sizeof(double4) * (size_t)(bcap / SDF_CHUNK + 2 * N + 2),  // cbox
      sizeof(int32_t) * (size_t)std::max<int64_t>(tiles8, 1),  // order
      sizeof(int32_t) * 64,                                // obin
      sizeof(double) * (size_t)(S + 1),                    // sacc
      sizeof(int32_t) * (size_t)(tiles8 + 1),              // ck_off
      sizeof(int32_t) * (size_t)(tiles8 + 1),              // item_off
      sizeof(float) * 4 * 32 * 32 * (size_t)(pcap / CK_MIN + 1),  // ckbuf
      sizeof(float4) * (size_t)std::max<int64_t>(gcap, 1),  // gcol
      sizeof(double) * SEG_WORDS * (size_t)(bcap + (SDF_CHUNK - 1) * N + 1),  // segs
      sizeof(float4) * (size_t)std::max<int64_t>(gcap, 1),  // gaux
      sizeof(float) * (size_t)std::max<int64_t>(gcap, 1),   // gop
  };
  size_t off = 0;
  for (int i = 0; i < N_WS; ++i) {
    lay.off[i] = off;
    off += align256(sizes[i]);
  }
  lay.total = off;
  return lay;
}

Work carve(void* ws, const Layout& lay) {
  char* b = (char*)ws;
  Work w;
  w.knots = (double*)(b + lay.off[0]);
  w.L = (double*)(b + lay.off[1]);
  w.goff = (int32_t*)(b + lay.off[2]);
  w.bpts = (double2*)(b + lay.off[3]);
  w.scenes = (SceneTab*)(b + lay.off[4]);
  w.gcnt = (uint32_t*)(b + lay.off[5]);
  w.keys0 = (uint32_t*)(b + lay.off[6]);
  w.keys1 = (uint32_t*)(b + lay.off[7]);
  w.vals1 = (uint32_t*)(b + lay.off[8]);
  w.hist = (uint32_t*)(b + lay.off[9]);
  w.scan_tmp = (uint32_t*)(b + lay.off[10]);
  w.ggrad = (float*)(b + lay.off[11]);
  w.gcp = (double*)(b + lay.off[12]);
  w.gknot = (double*)(b + lay.off[13]);
  w.gcurve = (double*)(b + lay.off[14]);
  w.gb = (double2*)(b + lay.off[15]);
  w.queue = (int32_t*)(b + lay.off[16]);
  w.aux = (int32_t*)(b + lay.off[17]);
  w.cbox = (double4*)(b + lay.off[18]);
  w.order = (int32_t*)(b + lay.off[19]);
  w.obin = (int32_t*)(b + lay.off[20]);
  w.sacc = (double*)(b + lay.off[21]);
  w.ck_off = (int32_t*)(b + lay.off[22]);
  w.item_off = (int32_t*)(b + lay.off[23]);
  w.ckbuf = (float*)(b + lay.off[24]);
  w.gcol = (float4*)(b + lay.off[25]);
  w.segs = (double*)(b + lay.off[26]);
  w.gaux = (float4*)(b + lay.off[27]);
  w.gop = (float*)(b + lay.off[28]);
  return w;
}

static hipEvent_t timer_event(Timer* t) {
  if (t->used == t->cap) {
    const int ncap = t->cap ? 2 * t->cap : 256;
    hipEvent_t* np = new hipEvent_t[ncap];
    for (int i = 0; i < t->cap; ++i) np[i] = t->pool[i];
    // timing-only events: no system-scope fence (cache write-back) when they
    // are recorded, so that the phases they bracket run as they would without
    for (int i = t->cap; i < ncap; ++i)
      if (hipEventCreateWithFlags(&np[i], hipEventDisableSystemFence) != hipSuccess) np[i] = nullptr;
    delete[] t->pool;
    t->pool = np;
    t->cap = ncap;
  }
  return t->pool[t->used++];
}

void timer_begin(Timer* t, int id, hipStream_t s) {
  if (t->n_spans >= 4096) return;
  const int e = t->used;
  hipEvent_t ev = timer_event(t);
  if (ev && hipEventRecord(ev, s) == hipSuccess) t->open_ev[id] = e;
  else t->open_ev[id] = -1;
}

void timer_end(Timer* t, int id, hipStream_t s) {
  if (t->open_ev[id] < 0 || t->n_spans >= 4096) return;
  const int e = t->used;
  hipEvent_t ev = timer_event(t);
  if (!ev || hipEventRecord(ev, s) != hipSuccess) return;
  t->span_id[t->n_spans] = id;
  t->span_ev[t->n_spans][0] = t->open_ev[id];
  t->span_ev[t->n_spans][1] = e;
  ++t->n_spans;
  t->open_ev[id] = -1;
}

}  // namespace nsp

using namespace nsp;

namespace {

int fail(nsplat_ctx* ctx, int code, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return code;
}

int hip_fail(nsplat_ctx* ctx, hipError_t e, const char* where) {
  return fail(ctx, NSPLAT_EHIP, "%s: %s", where, hipGetErrorString(e));
}

int check_curves(nsplat_ctx* ctx, const nsplat_curves* cv) {
  if (!cv) return fail(ctx, NSPLAT_EINVAL, "curves is NULL");
  if (cv->n_curves < 0 || cv->n_keys < 0 || cv->n_taus < 0)
    return fail(ctx, NSPLAT_EINVAL, "negative size in curves (n_curves=%d n_keys=%d n_taus=%d)", cv->n_curves,
                cv->n_keys, cv->n_taus);
  if (cv->channels != 1 && cv->channels != 3)
    return fail(ctx, NSPLAT_EINVAL, "channels must be 1 or 3 (got %d)", cv->channels);
  if (cv->n_curves > 0) {
    const void* ptrs[11] = {cv->scene, cv->degree, cv->flags, cv->key_off, cv->tau_off, cv->key_xy,
                            cv->key_w, cv->key_s, cv->color, cv->opacity, cv->n_taus > 0 ? (const void*)cv->tau
                                                                                         : (const void*)cv};
    const char* names[11] = {"scene", "degree", "flags", "key_off", "tau_off", "key_xy",
                             "key_w", "key_s", "color", "opacity", "tau"};
    for (int i = 0; i < 11; ++i)
      if (!ptrs[i]) return fail(ctx, NSPLAT_EINVAL, "curves.%s is NULL", names[i]);
  }
  return NSPLAT_OK;
}

int check_scenes(nsplat_ctx* ctx, const nsplat_scenes* sc) {
  if (!sc) return fail(ctx, NSPLAT_EINVAL, "scenes is NULL");
  if (sc->n_scenes < 1) return fail(ctx, NSPLAT_EINVAL, "n_scenes must be >= 1 (got %d)", sc->n_scenes);
  if (!sc->hw_host || !sc->hw || !sc->bg) return fail(ctx, NSPLAT_EINVAL, "scenes.hw_host / hw / bg is NULL");
  int64_t pix = 0;
  for (int s = 0; s < sc->n_scenes; ++s) {
    const int H = sc->hw_host[2 * s], W = sc->hw_host[2 * s + 1];
    if (H < 1 || W < 1 || H > 32767 || W > 32767)
      return fail(ctx, NSPLAT_EINVAL, "scene %d has invalid size %dx%d", s, H, W);
    pix += (int64_t)H * W;
  }
  if (pix > 0x7fffffffLL / 3) return fail(ctx, NSPLAT_EINVAL, "too many pixels over all scenes");
  return NSPLAT_OK;
}

int check_params(nsplat_ctx* ctx, const nsplat_params* pr) {
  if (!pr) return fail(ctx, NSPLAT_EINVAL, "params is NULL");
  if (pr->tile != 8 && pr->tile != 16 && pr->tile != 32)
    return fail(ctx, NSPLAT_EINVAL, "tile must be 8, 16 or 32 (got %d)", pr->tile);
  if (pr->batch < 1 || pr->batch > MAX_BATCH)
    return fail(ctx, NSPLAT_EINVAL, "batch must be in [1, %d] (got %d)", MAX_BATCH, pr->batch);
  if (!(pr->rho > 0.f) || !(pr->delta_c > 0.f) || !(pr->delta_b > 0.f) || !(pr->eta > 0.f) ||
      !(pr->nl_factor > 0.f) || !(pr->delta_a > 0.f))
    return fail(ctx, NSPLAT_EINVAL, "rho, delta_c, delta_b, delta_a, eta and nl_factor must be > 0");
  if (!(pr->h > 0.f) && !pr->h_dev) return fail(ctx, NSPLAT_EINVAL, "h must be > 0");
  if (!(pr->alpha_max > 0.f && pr->alpha_max < 1.f))
    return fail(ctx, NSPLAT_EINVAL, "alpha_max must be in (0, 1) (got %g)", (double)pr->alpha_max);
  if (!(pr->k_sigma > 0.f)) return fail(ctx, NSPLAT_EINVAL, "k_sigma must be > 0");
  if (!(pr->eps_T >= 0.f && pr->eps_T <= 1.f))
    return fail(ctx, NSPLAT_EINVAL, "eps_T must be in [0, 1] (got %g)", (double)pr->eps_T);
  if (pr->kappa < 0) return fail(ctx, NSPLAT_EINVAL, "kappa must be >= 0");
  if (!(pr->fill_pad >= 0.f)) return fail(ctx, NSPLAT_EINVAL, "fill_pad must be >= 0");
  if (pr->chunk != 0 && (pr->chunk < CK_MIN || pr->chunk > CK_MAX || (pr->chunk & (pr->chunk - 1)) != 0))
    return fail(ctx, NSPLAT_EINVAL, "chunk must be 0 or a power of two in [%d, %d] (got %d)", CK_MIN, CK_MAX,
                pr->chunk);
  return NSPLAT_OK;
}

// log2 of params.chunk; when it is 0, 512 for batches without fills and -1
// (the binning chooses on the device, auto_chunk_log2) for batches with them:
// the fill-run walks cost mostly per run and per item set-up, which longer
// chunks save, while entry-by-entry stroke compositing gains more from
// splitting long lists across wavefronts.
int chunk_log2(const nsplat_curves* cv, const nsplat_params* pr) {
  if (pr->chunk == 0) return (cv->any_flags & NSPLAT_FILLED) ? -1 : 9;
  int lg = 0;
  while ((1 << lg) < pr->chunk) ++lg;
  return lg;
}

int check_bufs(nsplat_ctx* ctx, const nsplat_curves* cv, const nsplat_scenes* sc, const nsplat_buffers* bf) {
  if (!bf) return fail(ctx, NSPLAT_EINVAL, "buffers is NULL");
  if (bf->caps.gauss < 0 || bf->caps.pairs < 0 || bf->caps.boundary < 0)
    return fail(ctx, NSPLAT_EINVAL, "negative capacity");
  if (bf->caps.gauss > 0x7fffffffLL || bf->caps.pairs > 0x7fffffffLL || bf->caps.boundary > 0x7fffffffLL)
    return fail(ctx, NSPLAT_EINVAL, "capacity above 2^31 - 1");
  if (!bf->plan || !bf->gauss || !bf->ranges || !bf->idx || !bf->counters || !bf->ws)
    return fail(ctx, NSPLAT_EINVAL, "a buffer pointer is NULL");
  if (((uintptr_t)bf->ws & 255) != 0) return fail(ctx, NSPLAT_EINVAL, "workspace must be 256-byte aligned");
  const Layout lay = workspace_layout(cv, sc, &bf->caps);
  if (bf->ws_bytes < lay.total)
    return fail(ctx, NSPLAT_ECAPACITY, "workspace has %zu bytes, %zu required", bf->ws_bytes, lay.total);
  return NSPLAT_OK;
}

void record_scene_table(nsplat_ctx* ctx, const void* ws, const nsplat_scenes* sc, const nsplat_params* pr) {
  std::vector<int32_t> hw(sc->hw_host, sc->hw_host + 2 * (size_t)sc->n_scenes);
  for (auto& e : ctx->scene_sig)
    if (e.ws == ws) {
      e.tile = pr->tile;
      e.nl_factor = pr->nl_factor;
      e.hw.swap(hw);
      return;
    }
  ctx->scene_sig.push_back({ws, pr->tile, pr->nl_factor, std::move(hw)});
}

bool scene_table_current(nsplat_ctx* ctx, const void* ws, const nsplat_scenes* sc, const nsplat_params* pr) {
  for (const auto& e : ctx->scene_sig)
    if (e.ws == ws)
      return e.tile == pr->tile && e.nl_factor == pr->nl_factor && e.hw.size() == 2 * (size_t)sc->n_scenes &&
             std::equal(e.hw.begin(), e.hw.end(), sc->hw_host);
  return false;
}

void record_bin_tile(nsplat_ctx* ctx, const void* ws, int tile, int chunk, int blocks) {
  for (auto& e : ctx->bin_tile)
    if (e.ws == ws) {
      e.tile = tile;
      e.chunk = chunk;
      e.blocks = blocks;
      return;
    }
  ctx->bin_tile.push_back({ws, tile, chunk, blocks});
}

// NSPLAT_EINVAL when the workspace's tile lists were built (by this context)
// for another tile side or params.chunk than this launch's, or (blocks > 0,
// the adjoint) with adjoint items for another pixel-block split: at 32 x 32
// tiles the split follows whether the curves declare fills.
int check_bin_tile(nsplat_ctx* ctx, const void* ws, int tile, int chunk, int blocks = 0) {
  for (const auto& e : ctx->bin_tile) {
    if (e.ws != ws) continue;
    if (e.tile != tile)
      return fail(ctx, NSPLAT_EINVAL, "the tile lists of this workspace were built by nsplat_bin with tile %d, "
                  "but params.tile is %d", e.tile, tile);
    if (e.chunk != chunk)
      return fail(ctx, NSPLAT_EINVAL, "the tile lists of this workspace were built by nsplat_bin with chunk %d, "
                  "but params.chunk is %d", e.chunk, chunk);
    if (blocks > 0 && e.blocks != blocks)
      return fail(ctx, NSPLAT_EINVAL, "the adjoint items of this workspace were built by nsplat_bin for %d pixel "
                  "blocks per chunk, but these curves need %d (any_flags differs in NSPLAT_FILLED)", e.blocks,
                  blocks);
  }
  return NSPLAT_OK;
}

int prepare(nsplat_ctx* ctx, const nsplat_curves* cv, const nsplat_scenes* sc, const nsplat_params* pr,
            const nsplat_buffers* bf, void* stream, Launch* L) {
  if (!ctx) return NSPLAT_EINVAL;
  int e;
  if ((e = check_curves(ctx, cv)) || (e = check_scenes(ctx, sc)) || (e = check_params(ctx, pr)) ||
      (e = check_bufs(ctx, cv, sc, bf)))
    return e;
  L->cv = cv;
  L->sc = sc;
  L->pr = pr;
  L->bf = bf;
  L->lay = workspace_layout(cv, sc, &bf->caps);
  L->w = carve(bf->ws, L->lay);
  L->stream = (hipStream_t)stream;
  L->n_tiles = nsplat_num_tiles(sc, pr->tile);
  L->n_cu = ctx->n_cu;
  L->ck_lg = chunk_log2(cv, pr);
  L->tm = ctx->timer.on ? &ctx->timer : nullptr;
  return NSPLAT_OK;
}

}  // namespace

extern "C" {

int nsplat_abi_version(void) { return NSPLAT_ABI_VERSION; }

int nsplat_create(nsplat_ctx** out, int device) {
  if (!out) return NSPLAT_EINVAL;
  *out = nullptr;
  nsplat_ctx* c = new nsplat_ctx();
  c->device = device;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    c->err = "no such HIP device";
    *out = c;
    return NSPLAT_EHIP;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    c->n_cu = prop.multiProcessorCount;
  // the device address of nsplat_udf_loss_noalloc's static scratch, taken
  // once per device with that device current
  int prev = 0;
  hipError_t h = hipGetDevice(&prev);
  if (h == hipSuccess) h = hipSetDevice(device);
  if (h == hipSuccess) {
    h = udf_scratch_setup(device);
    const hipError_t r = hipSetDevice(prev);
    if (h == hipSuccess) h = r;
  }
  *out = c;
  if (h != hipSuccess) return hip_fail(c, h, "nsplat_create: device scratch");
  return NSPLAT_OK;
}

int nsplat_destroy(nsplat_ctx* ctx) {
  delete ctx;
  return NSPLAT_OK;
}

const char* nsplat_last_error(const nsplat_ctx* ctx) { return ctx ? ctx->err.c_str() : "no context"; }

int64_t nsplat_num_tiles(const nsplat_scenes* sc, int32_t tile) {
  if (!sc || !sc->hw_host || tile <= 0) return 0;
  int64_t n = 0;
  for (int s = 0; s < sc->n_scenes; ++s)
    n += (int64_t)((sc->hw_host[2 * s] + tile - 1) / tile) * ((sc->hw_host[2 * s + 1] + tile - 1) / tile);
  return n;
}

size_t nsplat_workspace_size(const nsplat_curves* cv, const nsplat_scenes* sc, const nsplat_params* pr,
                             const nsplat_caps* caps) {
  (void)pr;
  if (!cv || !sc || !caps) return 0;
  return workspace_layout(cv, sc, caps).total;
}

int nsplat_sample(nsplat_ctx* ctx, const nsplat_curves* cv, const nsplat_scenes* sc, const nsplat_params* pr,
                  const nsplat_buffers* bf, int frozen, void* stream) {
  Launch L;
  int e = prepare(ctx, cv, sc, pr, bf, stream, &L);
  if (e) return e;
  hipError_t h = launch_scene_setup(L, bf->counters);
  record_scene_table(ctx, bf->ws, sc, pr);
  if (h == hipSuccess && cv->n_curves > 0) h = launch_sample(L, frozen);
  if (h == hipSuccess && cv->n_curves == 0) h = launch_fill_u32((uint32_t*)L.w.goff, 0u, 1, L.stream);
  if (h != hipSuccess) return hip_fail(ctx, h, "nsplat_sample");
  return NSPLAT_OK;
}

int nsplat_bin(nsplat_ctx* ctx, const nsplat_curves* cv, const nsplat_scenes* sc, const nsplat_params* pr,
               const nsplat_buffers* bf, void* stream) {
  Launch L;
  int e = prepare(ctx, cv, sc, pr, bf, stream, &L);
  if (e) return e;
  // the table is rebuilt unless the last build on this workspace (in stream
  // order, e.g. the nsplat_sample of the same step) used the same tile side,
  // N_L factor and scene sizes
  hipError_t h = hipSuccess;
  if (!scene_table_current(ctx, bf->ws, sc, pr)) {
    h = launch_scene_setup(L, nullptr);
    record_scene_table(ctx, bf->ws, sc, pr);
  }
  if (h == hipSuccess) h = launch_bin(L);
  if (h != hipSuccess) return hip_fail(ctx, h, "nsplat_bin");
  record_bin_tile(ctx, bf->ws, pr->tile, pr->chunk, nsp::adj_blocks_of(L));
  return NSPLAT_OK;
}

int nsplat_forward(nsplat_ctx* ctx, const nsplat_curves* cv, const nsplat_scenes* sc, const nsplat_params* pr,
                   const nsplat_buffers* bf, float* image, float* T_final, int32_t* n_last, int persistent,
                   void* stream) {
  Launch L;
  int e = prepare(ctx, cv, sc, pr, bf, stream, &L);
  if (e) return e;
  if (!image || !T_final || !n_last) return fail(ctx, NSPLAT_EINVAL, "image / T_final / n_last is NULL");
  if ((e = check_bin_tile(ctx, bf->ws, pr->tile, pr->chunk))) return e;
  hipError_t h = launch_blend_fwd(L, image, T_final, n_last, persistent);
  if (h != hipSuccess) return hip_fail(ctx, h, "nsplat_forward");
  return NSPLAT_OK;
}

int nsplat_backward_reg(nsplat_ctx* ctx, const nsplat_curves* cv, const nsplat_scenes* sc, const nsplat_params* pr,
                        const nsplat_buffers* bf, const float* dL, const float* T_final, const int32_t* n_last,
                        const nsplat_reg* reg, const nsplat_grads* gr, int persistent, void* stream) {
  Launch L;
  int e = prepare(ctx, cv, sc, pr, bf, stream, &L);
  if (e) return e;
  if (!dL || !T_final || !n_last || !gr) return fail(ctx, NSPLAT_EINVAL, "dL_dimage / T_final / n_last / grads is NULL");
  if ((e = check_bin_tile(ctx, bf->ws, pr->tile, pr->chunk, nsp::adj_blocks_of(L)))) return e;
  const bool use_reg = reg && (reg->bbox_weight != 0.0f || reg->deriv_weight != 0.0f);
  if (use_reg) {
    if (reg->deriv_weight != 0.0f && (reg->deriv_order < 1 || reg->deriv_order > 3))
      return fail(ctx, NSPLAT_EINVAL, "deriv_order must be in 1..3 (got %d)", reg->deriv_order);
    if (reg->bbox_kind != 0 && reg->bbox_kind != 1)
      return fail(ctx, NSPLAT_EINVAL, "bbox_kind must be 0 (ReLU) or 1 (softplus) (got %d)", reg->bbox_kind);
  }
  hipError_t h = launch_zero_grads(L);
  if (h == hipSuccess) h = launch_blend_bwd(L, dL, T_final, n_last, persistent);
  if (h == hipSuccess && use_reg && cv->n_curves > 0) h = launch_reg(L, reg);
  if (h == hipSuccess && cv->n_curves > 0) h = launch_adjoint(L, gr);
  if (h != hipSuccess) return hip_fail(ctx, h, "nsplat_backward");
  return NSPLAT_OK;
}

int nsplat_backward(nsplat_ctx* ctx, const nsplat_curves* cv, const nsplat_scenes* sc, const nsplat_params* pr,
                    const nsplat_buffers* bf, const float* dL, const float* T_final, const int32_t* n_last,
                    const nsplat_grads* gr, int persistent, void* stream) {
  return nsplat_backward_reg(ctx, cv, sc, pr, bf, dL, T_final, n_last, nullptr, gr, persistent, stream);
}

int nsplat_udf_loss(nsplat_ctx* ctx, const nsplat_curves* cv, const nsplat_scenes* sc, const nsplat_params* pr,
                    const nsplat_buffers* bf, const int32_t* sel, float tau, const float* image, const float* target,
                    float* dL, float* loss, void* stream) {
  Launch L;
  int e = prepare(ctx, cv, sc, pr, bf, stream, &L);
  if (e) return e;
  if (!image || !target || !dL) return fail(ctx, NSPLAT_EINVAL, "image / target / dL_dimage is NULL");
  if (!(tau > 0.0f)) return fail(ctx, NSPLAT_EINVAL, "tau must be positive (got %g)", (double)tau);
  hipError_t h = launch_udf(L, sel, tau, image, target, dL, loss);
  if (h != hipSuccess) return hip_fail(ctx, h, "nsplat_udf_loss");
  return NSPLAT_OK;
}

int nsplat_udf_loss_noalloc(nsplat_ctx* ctx, const nsplat_curves* cv, const nsplat_scenes* sc,
                            const nsplat_params* pr, const nsplat_buffers* bf, const int32_t* sel, float tau,
                            const float* image, const float* target, float* dL, float* loss, void* stream) {
  Launch L;
  int e = prepare(ctx, cv, sc, pr, bf, stream, &L);
  if (e) return e;
  if (!image || !target || !dL) return fail(ctx, NSPLAT_EINVAL, "image / target / dL_dimage is NULL");
  if (!(tau > 0.0f)) return fail(ctx, NSPLAT_EINVAL, "tau must be positive (got %g)", (double)tau);
  if (sc->n_scenes > UDF_SCRATCH_SLOTS - 1)
    return fail(ctx, NSPLAT_EINVAL, "nsplat_udf_loss_noalloc takes at most %d scenes (got %d)",
                UDF_SCRATCH_SLOTS - 1, sc->n_scenes);
  double* sacc = udf_scratch(ctx->device);
  if (!sacc) return fail(ctx, NSPLAT_EHIP, "nsplat_udf_loss_noalloc: device scratch was not set up");
  hipError_t h = launch_udf(L, sel, tau, image, target, dL, loss, sacc);
  if (h != hipSuccess) return hip_fail(ctx, h, "nsplat_udf_loss_noalloc");
  return NSPLAT_OK;
}

int nsplat_adam_step(nsplat_ctx* ctx, const nsplat_adam* cfg, const nsplat_values* prm, const nsplat_grads* gr,
                     float* m, float* v, int32_t* step_dev, void* stream) {
  if (!ctx) return NSPLAT_EINVAL;
  if (!cfg || !prm || !gr || !step_dev) return fail(ctx, NSPLAT_EINVAL, "cfg / params / grads / step is NULL");
  if (prm->n_curves < 0 || prm->n_keys < 0 || prm->n_taus < 0 || (prm->channels != 1 && prm->channels != 3))
    return fail(ctx, NSPLAT_EINVAL, "bad parameter sizes");
  const int64_t n = 4 * (int64_t)prm->n_keys + prm->n_taus + (int64_t)prm->n_curves * (prm->channels + 1);
  if (n > 0 && (!m || !v)) return fail(ctx, NSPLAT_EINVAL, "moment buffers are NULL");
  if ((prm->n_keys > 0 && (!prm->key_xy || !prm->key_w || !prm->key_s || !gr->key_xy || !gr->key_w ||
                           !gr->key_s)) ||
      (prm->n_taus > 0 && (!prm->tau || !gr->tau)) ||
      (prm->n_curves > 0 && (!prm->color || !prm->opacity || !gr->color || !gr->opacity)))
    return fail(ctx, NSPLAT_EINVAL, "a parameter or gradient pointer is NULL");
  if (!(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) || !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) ||
      !(cfg->eps > 0.0f) || !(cfg->w_min <= cfg->w_max) || !(cfg->tau_min <= cfg->tau_max))
    return fail(ctx, NSPLAT_EINVAL, "bad Adam settings");
  hipError_t h = launch_adam(cfg, prm, gr, m, v, step_dev, (hipStream_t)stream);
  if (h != hipSuccess) return hip_fail(ctx, h, "nsplat_adam_step");
  return NSPLAT_OK;
}

int nsplat_anneal_h(nsplat_ctx* ctx, float* h_dev, int32_t* step_dev, int32_t step, int32_t total, float hmax,
                    float hmin, float tb, float te, void* stream) {
  if (!ctx) return NSPLAT_EINVAL;
  if (!h_dev) return fail(ctx, NSPLAT_EINVAL, "h_dev is NULL");
  if (total <= 0 || !(te > tb)) return fail(ctx, NSPLAT_EINVAL, "need total_steps > 0 and t_e > t_b");
  hipError_t h = launch_anneal(h_dev, step_dev, step, total, hmax, hmin, tb, te, (hipStream_t)stream);
  if (h != hipSuccess) return hip_fail(ctx, h, "nsplat_anneal_h");
  return NSPLAT_OK;
}

int nsplat_l2_grad(nsplat_ctx* ctx, const float* a, const float* b, float* out, float* loss, int64_t n,
                   void* stream) {
  if (!ctx) return NSPLAT_EINVAL;
  if (n < 0 || (n > 0 && (!a || !b || !out))) return fail(ctx, NSPLAT_EINVAL, "bad arguments to nsplat_l2_grad");
  hipError_t h = launch_l2(a, b, out, loss, n, (hipStream_t)stream);
  if (h != hipSuccess) return hip_fail(ctx, h, "nsplat_l2_grad");
  return NSPLAT_OK;
}

int nsplat_timing(nsplat_ctx* ctx, int enable) {
  if (!ctx) return NSPLAT_EINVAL;
  Timer& t = ctx->timer;
  t.on = enable != 0;
  t.mask = (enable & NSPLAT_TIMING_ONLY) ? (uint32_t)enable & ((1u << NSPLAT_NUM_TIMERS) - 1u)
                                         : (1u << NSPLAT_NUM_TIMERS) - 1u;
  t.used = 0;
  t.n_spans = 0;
  for (int i = 0; i < NSPLAT_NUM_TIMERS; ++i) {
    t.ms[i] = 0.0;
    t.count[i] = 0;
    t.open_ev[i] = -1;
  }
  return NSPLAT_OK;
}

int nsplat_timing_read(nsplat_ctx* ctx, double* ms, int64_t* count) {
  if (!ctx) return NSPLAT_EINVAL;
  Timer& t = ctx->timer;
  for (int k = 0; k < t.n_spans; ++k) {
    float x = 0.f;
    hipEvent_t b = t.pool[t.span_ev[k][1]];
    if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&x, t.pool[t.span_ev[k][0]], b) != hipSuccess)
      return fail(ctx, NSPLAT_EHIP, "nsplat_timing_read: event query failed");
    t.ms[t.span_id[k]] += (double)x;
    t.count[t.span_id[k]] += 1;
  }
  t.n_spans = 0;
  t.used = 0;
  for (int i = 0; i < NSPLAT_NUM_TIMERS; ++i) {
    if (ms) ms[i] = t.ms[i];
    if (count) count[i] = t.count[i];
  }
  return NSPLAT_OK;
}

int nsplat_read_counters(nsplat_ctx* ctx, const nsplat_buffers* bf, int32_t* host_out, void* stream) {
  if (!ctx) return NSPLAT_EINVAL;
  if (!bf || !bf->counters || !host_out) return fail(ctx, NSPLAT_EINVAL, "bad arguments to nsplat_read_counters");
  hipError_t h = hipMemcpyAsync(host_out, bf->counters, sizeof(int32_t) * NSPLAT_NUM_COUNTERS,
                                hipMemcpyDeviceToHost, (hipStream_t)stream);
  if (h == hipSuccess) h = hipStreamSynchronize((hipStream_t)stream);
  if (h != hipSuccess) return hip_fail(ctx, h, "nsplat_read_counters");
  return NSPLAT_OK;
}

int nsplat_gauss_frame(nsplat_ctx* ctx, const nsplat_curves* cv, const nsplat_scenes* sc, const nsplat_buffers* bf,
                       float* out, int64_t n, void* stream) {
  if (!ctx) return NSPLAT_EINVAL;
  int e;
  if ((e = check_curves(ctx, cv)) || (e = check_scenes(ctx, sc)) || (e = check_bufs(ctx, cv, sc, bf))) return e;
  if (n < 0 || n > bf->caps.gauss)
    return fail(ctx, NSPLAT_EINVAL, "n = %lld outside [0, caps.gauss = %lld]", (long long)n,
                (long long)bf->caps.gauss);
  if (n == 0) return NSPLAT_OK;
  if (!out) return fail(ctx, NSPLAT_EINVAL, "out is NULL");
  const Layout lay = workspace_layout(cv, sc, &bf->caps);
  const Work w = carve(bf->ws, lay);
  const hipError_t h = hipMemcpyAsync(out, w.gaux, sizeof(float4) * (size_t)n, hipMemcpyDeviceToDevice,
                                      (hipStream_t)stream);
  if (h != hipSuccess) return hip_fail(ctx, h, "nsplat_gauss_frame");
  return NSPLAT_OK;
}

int nsplat_autotune(nsplat_ctx* ctx, const nsplat_curves* cv, const nsplat_scenes* sc, const nsplat_params* pr,
                    const nsplat_buffers* bf, float* image, float* T_final, int32_t* n_last, const float* dL,
                    const nsplat_grads* gr, int persistent, int32_t* best_tile, int32_t* best_batch,
                    float* times_ms, void* stream) {
  if (!ctx) return NSPLAT_EINVAL;
  if (!best_tile || !best_batch) return fail(ctx, NSPLAT_EINVAL, "best_tile / best_batch is NULL");
  static const int tiles[3] = {8, 16, 32};
  static const int batches[4] = {32, 64, 128, 256};
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(ctx, NSPLAT_EHIP, "hipEventCreate failed");
  float best = 1e30f;
  int rc = NSPLAT_OK;
  *best_tile = pr->tile;
  *best_batch = pr->batch;
  for (int ti = 0; ti < 3 && rc == NSPLAT_OK; ++ti)
    for (int bi = 0; bi < 4 && rc == NSPLAT_OK; ++bi) {
      nsplat_params p = *pr;
      p.tile = tiles[ti];
      p.batch = batches[bi];
      float ms = 0.f;
      for (int rep = 0; rep < 2 && rc == NSPLAT_OK; ++rep) {
        if (rep == 1 && hipEventRecord(e0, s) != hipSuccess) rc = NSPLAT_EHIP;
        if (rc == NSPLAT_OK) rc = nsplat_bin(ctx, cv, sc, &p, bf, stream);
        if (rc == NSPLAT_OK) rc = nsplat_forward(ctx, cv, sc, &p, bf, image, T_final, n_last, persistent, stream);
        if (rc == NSPLAT_OK)
          rc = nsplat_backward(ctx, cv, sc, &p, bf, dL, T_final, n_last, gr, persistent, stream);
        if (rep == 1 && rc == NSPLAT_OK) {
          if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
              hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            rc = NSPLAT_EHIP;
        }
      }
      if (rc != NSPLAT_OK) break;
      int32_t cnt[NSPLAT_NUM_COUNTERS];
      rc = nsplat_read_counters(ctx, bf, cnt, stream);
      if (rc == NSPLAT_OK && (cnt[NSPLAT_CNT_STATUS] & NSPLAT_STATUS_PAIR_CAP)) ms = 1e30f;  // did not fit
      if (times_ms) times_ms[ti * 4 + bi] = ms;
      if (ms < best) {
        best = ms;
        *best_tile = tiles[ti];
        *best_batch = batches[bi];
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == NSPLAT_EHIP && ctx->err.empty()) ctx->err = "autotune: HIP event error";
  if (rc == NSPLAT_OK) {
    // leave the buffers and outputs in the state of the chosen setting
    nsplat_params p = *pr;
    p.tile = *best_tile;
    p.batch = *best_batch;
    rc = nsplat_bin(ctx, cv, sc, &p, bf, stream);
    if (rc == NSPLAT_OK) rc = nsplat_forward(ctx, cv, sc, &p, bf, image, T_final, n_last, persistent, stream);
    if (rc == NSPLAT_OK) rc = nsplat_backward(ctx, cv, sc, &p, bf, dL, T_final, n_last, gr, persistent, stream);
  }
  return rc;
}

}  // extern "C"
