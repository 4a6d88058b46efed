// Host runtime of libddpinn: argument validation, workspace layout, work
// partitioning, hipGraph capture and the C ABI declared in include/ddpinn.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ddpinn.h"
#include "ddpinn_internal.h"

namespace ddp {
hipError_t set_lds_limits(int bytes);
}

using namespace ddp;

namespace {

thread_local std::string g_err;

pinn_status fail(pinn_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
pinn_status fail(pinn_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHECK(expr)                                                              \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return fail(PINN_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));    \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Device address of the library-held query scratch, one per device, resolved
// at the first pinn_create on that device (with the device current).
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};

hipError_t resolve_noalloc_scratch(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = noalloc_scratch_address(&p);
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_noalloc_ptr[device] = p;
  }
  *out = g_noalloc_ptr[device];
  return hipSuccess;
}

int64_t nparams(int dim, int W, int H) {
  const int64_t D = dim + 1;
  return W * D + W + (int64_t)(H - 1) * ((int64_t)W * W + W) + D * W + D;
}

Shape make_shape(int dim, int W, int H) {
  Shape sh{};
  sh.dim = dim;
  sh.D = dim + 1;
  sh.W = W;
  sh.H = H;
  sh.Wp = (W + 15) / 16 * 16;
  sh.NW = sh.Wp / 16;
  sh.NWV = std::min(sh.NW, kMaxWaves);
  sh.Kq = (W + 3) / 4;
  sh.P = (int32_t)nparams(dim, W, H);
  const int64_t Wp = sh.Wp, D = sh.D;
  // packed offsets
  int64_t o = 0;
  for (int l = 1; l <= H + 1; ++l) {
    const int64_t fi = (l == 1) ? D : W, fo = (l == H + 1) ? D : W;
    sh.p_w[l] = o;
    o += fo * fi;
    sh.p_b[l] = o;
    o += fo;
  }
  // fragment buffer
  o = 0;
  sh.f_hid = o; o += 2 * (int64_t)(H - 1) * Wp * Wp;
  sh.f_w1 = o;  o += Wp * D;
  sh.f_b = o;   o += (int64_t)H * Wp;
  sh.f_wo = o;  o += D * Wp;
  sh.f_bo = o;  o += 4;
  sh.frag_floats = (o + 63) / 64 * 64;
  // slab
  o = 0;
  sh.s_hid = o; o += (int64_t)(H - 1) * Wp * Wp;
  sh.s_b = o;   o += (int64_t)H * Wp;
  sh.s_w1 = o;  o += Wp * D;
  sh.s_wo = o;  o += D * Wp;
  sh.s_bo = o;  o += 4;
  sh.s_loss = o; o += 8;
  sh.slab_floats = (o + 63) / 64 * 64;
  return sh;
}

// Tiles of one subdomain: collocation tiles, and value tiles over the
// concatenated [observation | ghost | anchor] list, the value tiles spread
// evenly among the collocation tiles.  A value tile costs more than a
// collocation tile (an activation per column instead of per point), so
// spreading them keeps every workgroup's mix, and time, the same.
void tiles_of(const pinn_subdomain& s, int sub, int tp, int tv, std::vector<Item>& out) {
  const int64_t np = (s.n_pde + tp - 1) / tp;
  const int64_t nv = s.n_obs + s.n_gh + s.n_anc;
  const int64_t nvt = (nv + tv - 1) / tv;
  int64_t ip = 0, iv = 0;
  for (int64_t k = 0; k < np + nvt; ++k) {
    // value tile iv goes at position floor((iv + 1/2) (np + nvt) / nvt)
    const bool value = iv < nvt && (ip >= np || 2 * k + 1 >= (2 * iv + 1) * (np + nvt) / nvt);
    if (value) {
      const int64_t st = iv * tv;
      out.push_back(Item{sub, ITEM_VALUE, (int32_t)st, (int32_t)std::min<int64_t>(tv, nv - st), -1, 0, {0, 0}});
      ++iv;
    } else {
      const int64_t st = ip * tp;
      out.push_back(Item{sub, ITEM_PDE, (int32_t)st, (int32_t)std::min<int64_t>(tp, s.n_pde - st), -1, 0, {0, 0}});
      ++ip;
    }
  }
}

// Relative cost of a value tile: the GEMM work of both kinds is the same,
// the extra activation work of a value tile is per wave (independent of the
// width) while the GEMM work per wave grows with it.
double value_tile_cost(const Shape& sh) { return 1.0 + 21.0 / sh.Wp; }

// Split a sorted item list into n_wg contiguous ranges of equal estimated
// cost and mark segments (maximal runs of one subdomain inside one
// workgroup); slabs are numbered from slab0.
void partition(std::vector<Item>& items, int n_wg, double vcost, int slab0, std::vector<int32_t>& wg_begin,
               int* n_seg) {
  const int64_t n = (int64_t)items.size();
  std::vector<double> cum(n + 1, 0.0);
  for (int64_t i = 0; i < n; ++i) cum[i + 1] = cum[i] + (items[i].kind == ITEM_VALUE ? vcost : 1.0);
  wg_begin.assign(n_wg + 1, 0);
  wg_begin[n_wg] = (int32_t)n;
  int64_t i = 0;
  for (int b = 1; b < n_wg; ++b) {
    const double target = cum[n] * b / n_wg;
    while (i < n && cum[i] + 0.5 * (cum[i + 1] - cum[i]) < target) ++i;
    // every workgroup keeps at least one item when there are enough
    const int64_t lo = wg_begin[b - 1] + 1, hi = n - (n_wg - b);
    wg_begin[b] = (int32_t)std::max<int64_t>(std::min<int64_t>(std::max<int64_t>(i, lo), hi), wg_begin[b - 1]);
  }
  int seg = slab0 - 1;
  for (int b = 0; b < n_wg; ++b) {
    for (int i = wg_begin[b]; i < wg_begin[b + 1]; ++i) {
      const bool first = (i == wg_begin[b]) || items[i].sub != items[i - 1].sub;
      const bool last = (i + 1 == wg_begin[b + 1]) || items[i].sub != items[i + 1].sub;
      if (first) ++seg;
      items[i].slab = seg;
      items[i].flags = (first ? ITEM_FIRST : 0) | (last ? ITEM_LAST : 0);
    }
  }
  *n_seg = seg + 1 - slab0;
}

}  // namespace

struct pinn_ctx {
  pinn_config cfg{};
  Shape sh{};
  int n_sub = 0;
  std::vector<pinn_subdomain> subs;
  int device = 0, num_cu = 0;
  void* noalloc_scratch = nullptr;   // device address of the library-held query scratch
  int tile_points = 16, value_points = 0;
  int threads = 0;
  int lds_floats = 0, qlds_floats = 0;
  int step_occ = 1;
  int query_occ[4] = {1, 1, 1, 1};   // resident query workgroups per compute unit, by query kind
  int qlds_small_floats = 0;         // LDS of the small-tile query (value and gradient modes)
  int query_occ_small[2] = {1, 1};   // its resident workgroups per compute unit (value, gradient)
  int exch_occ = 1;
  // grouped launch: n_wg workgroups over n_ranges item ranges (taken in
  // turn through a counter when several workgroups share a compute unit)
  int n_wg = 0, n_ranges = 0, n_items = 0, n_seg = 0;
  bool dynamic = false;
  // per-subdomain launches
  std::vector<int> ps_wg, ps_nr, ps_wgb_off;
  int ps_items = 0, ps_seg = 0;
  int n_slabs = 0, n_chunks = 1;
  int64_t stash_per_wg = 0;
  // device regions inside the workspace
  SubDev* d_subs = nullptr;
  Item* d_items = nullptr;
  int32_t* d_wg_begin = nullptr;
  int32_t* d_counters = nullptr;   // [1 + n_sub]: grouped launch, then each plain launch
  int32_t* d_seg_begin = nullptr;
  Item* d_items_ps = nullptr;
  int32_t* d_wgb_ps = nullptr;
  int32_t* d_seg_ps = nullptr;
  float* d_slabs = nullptr;
  float* d_stash = nullptr;
  float* d_frag = nullptr;
  float* d_partial = nullptr;
  float* d_loss_ws = nullptr;
  float* d_gbuf = nullptr;
  float* d_normpart = nullptr;
  float* d_clip = nullptr;
  float* d_boxes = nullptr;
  ExchangeItem* d_xitems = nullptr;
  float** d_targets = nullptr;
  int x_cap = 0;
  std::vector<ExchangeItem> x_host;
  std::vector<float*> x_targets_host;
  // exchange: each launch is ordered after the previous one (x_done), on
  // whatever stream; host copies of a changed work list stay alive until the
  // copy that reads them has run (x_staged, reaped without waiting)
  hipEvent_t x_done = nullptr;
  bool x_done_recorded = false;
  struct Staged {
    std::vector<char> bytes;
    hipEvent_t copied;
  };
  std::vector<Staged*> x_staged;
  float gmax[4] = {0, 0, 0, 0};
  // graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraphNode_t n_reduce = nullptr;   // Adam node (t, lr, update change per step)
  hipGraphNode_t n_grad = nullptr;     // gradient node (output pointers change per step)
  ReduceArgs rargs{};
  StepArgs sargs{};
  PrepArgs pargs{};
  // memory-check mode: guard zones (offset, bytes) after each workspace region
  std::vector<std::pair<size_t, size_t>> guards;
  char* ws = nullptr;
  int guard_bytes = 0;
  // kernel timing (PINN_TIME_KERNEL)
  std::vector<hipEvent_t> ev_start, ev_stop;
  int ev_used = 0;
  double ev_folded_ms = 0.0;
  int64_t ev_folded_n = 0;
};

namespace {
constexpr int kEventPool = 1024;

// wait for the recorded event pairs, add their durations to the folded sum
pinn_status fold_events(pinn_ctx* c) {
  for (int i = 0; i < c->ev_used; ++i) {
    HIPCHECK(hipEventSynchronize(c->ev_stop[i]));
    float ms = 0.f;
    HIPCHECK(hipEventElapsedTime(&ms, c->ev_start[i], c->ev_stop[i]));
    c->ev_folded_ms += ms;
    c->ev_folded_n += 1;
  }
  c->ev_used = 0;
  return PINN_OK;
}

pinn_status next_event_pair(pinn_ctx* c, hipEvent_t* a, hipEvent_t* b) {
  if (c->ev_start.empty()) {
    c->ev_start.resize(kEventPool);
    c->ev_stop.resize(kEventPool);
    for (int i = 0; i < kEventPool; ++i) {
      HIPCHECK(hipEventCreate(&c->ev_start[i]));
      HIPCHECK(hipEventCreate(&c->ev_stop[i]));
    }
  }
  if (c->ev_used == kEventPool) {
    pinn_status st = fold_events(c);
    if (st != PINN_OK) return st;
  }
  *a = c->ev_start[c->ev_used];
  *b = c->ev_stop[c->ev_used];
  c->ev_used++;
  return PINN_OK;
}
}  // namespace

extern "C" {

const char* pinn_last_error(void) { return g_err.c_str(); }

int64_t pinn_num_params(int32_t dim, int32_t width, int32_t depth) {
  if (dim < 2 || dim > 3 || width < 1 || depth < 1) return -1;
  return nparams(dim, width, depth);
}

static pinn_status validate(const pinn_config* cfg, const pinn_subdomain* subs) {
  if (!cfg) return fail(PINN_E_INVAL, "cfg is NULL");
  if (cfg->dim != 2 && cfg->dim != 3) return fail(PINN_E_INVAL, "dim must be 2 or 3 (got %d)", cfg->dim);
  if (cfg->width < 1) return fail(PINN_E_INVAL, "width must be >= 1");
  if (cfg->width > kMaxWidth) return fail(PINN_E_UNSUPPORTED, "width %d > %d", cfg->width, kMaxWidth);
  if (cfg->depth < 1) return fail(PINN_E_INVAL, "depth must be >= 1");
  if (cfg->depth > kMaxDepth) return fail(PINN_E_UNSUPPORTED, "depth %d > %d", cfg->depth, kMaxDepth);
  if (cfg->n_sub < 1 || cfg->n_sub > kMaxSub) return fail(PINN_E_INVAL, "n_sub must be in [1, %d]", kMaxSub);
  if (cfg->activation != 0 && cfg->activation != 1)
    return fail(PINN_E_UNSUPPORTED, "activation must be 0 (tanh) or 1 (sin)");
  for (int k = 0; k < 3; ++k)
    if (!(std::isfinite(cfg->comp_w[k]) && cfg->comp_w[k] >= 0)) return fail(PINN_E_INVAL, "comp_w[%d] must be finite and >= 0", k);
  if (!(std::isfinite(cfg->clip_norm) && cfg->clip_norm >= 0)) return fail(PINN_E_INVAL, "clip_norm must be finite and >= 0");
  if (cfg->lr_interval < 0) return fail(PINN_E_INVAL, "lr_interval must be >= 0");
  if (cfg->lr_interval > 0 && !(std::isfinite(cfg->lr_factor) && cfg->lr_factor > 0))
    return fail(PINN_E_INVAL, "lr_factor must be finite and > 0");
  if (!(std::isfinite(cfg->nu) && cfg->nu >= 0)) return fail(PINN_E_INVAL, "nu must be finite and >= 0");
  for (int k = 0; k < 6; ++k)
    if (!std::isfinite(cfg->lam[k])) return fail(PINN_E_INVAL, "lam[%d] not finite", k);
  if (!(cfg->lr >= 0 && std::isfinite(cfg->lr))) return fail(PINN_E_INVAL, "lr must be finite and >= 0");
  if (!(cfg->beta1 >= 0 && cfg->beta1 < 1 && cfg->beta2 >= 0 && cfg->beta2 < 1))
    return fail(PINN_E_INVAL, "Adam betas must be in [0, 1)");
  if (!(cfg->eps > 0)) return fail(PINN_E_INVAL, "Adam eps must be > 0");
  if (cfg->tile_points != 0 && cfg->tile_points != 16 && cfg->tile_points != 32)
    return fail(PINN_E_INVAL, "tile_points must be 0, 16 or 32");
  if (cfg->blocks_per_cu < 0) return fail(PINN_E_INVAL, "blocks_per_cu must be >= 0");
  if (cfg->gemm_priority_off != 0 && cfg->gemm_priority_off != 1)
    return fail(PINN_E_INVAL, "gemm_priority_off must be 0 or 1");
  if (cfg->ranges_per_wg < 0 || cfg->ranges_per_wg > 64) return fail(PINN_E_INVAL, "ranges_per_wg must be 0..64");
  if (cfg->guard_bytes < 0 || cfg->guard_bytes > (1 << 20) || (cfg->guard_bytes & 255))
    return fail(PINN_E_INVAL, "guard_bytes must be a multiple of 256 in [0, 1 MiB]");
  if (cfg->max_query_points < 0 || cfg->max_query_points > (int64_t)INT32_MAX)
    return fail(PINN_E_INVAL, "max_query_points out of range");
  if (cfg->flags & ~PINN_GRAPH) return fail(PINN_E_INVAL, "unknown config flags 0x%x", cfg->flags);
  if (!subs) return fail(PINN_E_INVAL, "subs is NULL");
  const int D = cfg->dim + 1;
  for (int s = 0; s < cfg->n_sub; ++s) {
    const pinn_subdomain& d = subs[s];
    if (!d.theta || !d.adam_m || !d.adam_v) return fail(PINN_E_INVAL, "sub %d: theta/adam_m/adam_v NULL", s);
    const int64_t cnt[4] = {d.n_pde, d.n_obs, d.n_gh, d.n_anc};
    for (int k = 0; k < 4; ++k)
      if (cnt[k] < 0 || cnt[k] > (int64_t)INT32_MAX / 2)
        return fail(PINN_E_INVAL, "sub %d: point count %d out of range", s, k);
    if (d.n_obs + d.n_gh + d.n_anc > (int64_t)INT32_MAX / 2)
      return fail(PINN_E_INVAL, "sub %d: too many value points", s);
    if (d.n_pde && !d.pde_x) return fail(PINN_E_INVAL, "sub %d: pde_x NULL", s);
    if (d.n_obs && (!d.obs_x || !d.obs_u)) return fail(PINN_E_INVAL, "sub %d: obs arrays NULL", s);
    if (d.n_gh && (!d.gh_x || !d.gh_up || !d.gh_kind)) return fail(PINN_E_INVAL, "sub %d: ghost arrays NULL", s);
    if (d.n_anc && (!d.anc_x || !d.anc_p)) return fail(PINN_E_INVAL, "sub %d: anchor arrays NULL", s);
    for (int q = 0; q < D; ++q)
      if (!(d.lo[q] <= d.hi[q])) return fail(PINN_E_INVAL, "sub %d: box lo > hi on axis %d", s, q);
  }
  return PINN_OK;
}

pinn_status pinn_create(const pinn_config* cfg, const pinn_subdomain* subs, void* workspace,
                        size_t* workspace_bytes, void* stream, pinn_ctx** out) {
  g_err.clear();
  pinn_status st = validate(cfg, subs);
  if (st != PINN_OK) return st;
  if (!workspace_bytes) return fail(PINN_E_INVAL, "workspace_bytes is NULL");
  if (workspace && !out) return fail(PINN_E_INVAL, "out is NULL");
  if (workspace && ((uintptr_t)workspace & 255)) return fail(PINN_E_INVAL, "workspace must be 256-byte aligned");

  pinn_ctx tmp;
  pinn_ctx* c = &tmp;
  c->cfg = *cfg;
  c->n_sub = cfg->n_sub;
  c->sh = make_shape(cfg->dim, cfg->width, cfg->depth);
  c->sh.act = cfg->activation;
  c->subs.assign(subs, subs + cfg->n_sub);
  const Shape& sh = c->sh;

  HIPCHECK(hipGetDevice(&c->device));
  HIPCHECK(resolve_noalloc_scratch(c->device, &c->noalloc_scratch));
  HIPCHECK(hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, c->device));
  int max_lds = 0, optin = 0;
  HIPCHECK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
  if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, c->device) == hipSuccess)
    max_lds = std::max(max_lds, optin);
  HIPCHECK(ddp::set_lds_limits(max_lds));

  // two row blocks per wave: the column-split LDS plan when the plain one
  // does not fit
  if (sh.NW > sh.NWV && (int64_t)step_lds_floats(sh, 16) * 4 > max_lds) c->sh.split = 1;

  // tile shape: 32-point collocation tiles when they fit in LDS with at
  // least the occupancy of 16-point tiles, unless fixed by the caller
  c->threads = sh.NWV * 64;
  auto occ_of = [&](int tp, int* occ) -> pinn_status {
    const int lf = step_lds_floats(sh, tp);
    const void* k = step_kernel_ptr(sh, tp);
    // 32-point tiles hold twice the registers: at most 4 waves (Wp <= 64)
    if (!k || (int64_t)lf * 4 > max_lds || (tp == 32 && c->threads > 256)) { *occ = 0; return PINN_OK; }
    int nb = 0;
    HIPCHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, c->threads, (size_t)lf * 4));
    *occ = nb;
    return PINN_OK;
  };
  int occ16 = 0, occ32 = 0;
  if ((st = occ_of(16, &occ16)) != PINN_OK) return st;
  if ((st = occ_of(32, &occ32)) != PINN_OK) return st;
  int tp = cfg->tile_points;
  if (tp == 0) tp = 16;
  const int occ = (tp == 32) ? occ32 : occ16;
  if (occ < 1) {
    if (!step_kernel_ptr(sh, tp))
      return fail(PINN_E_UNSUPPORTED, "width %d: only 16-point tiles above %d neurons", cfg->width, 16 * kMaxWaves);
    return fail(PINN_E_UNSUPPORTED, "tile of %d points needs %d B of LDS per workgroup (device limit %d B)", tp,
                step_lds_floats(sh, tp) * 4, max_lds);
  }
  c->tile_points = tp;
  c->value_points = step_value_points(sh.dim, tp);
  c->lds_floats = step_lds_floats(sh, tp);
  c->step_occ = cfg->blocks_per_cu > 0 ? std::min(cfg->blocks_per_cu, occ) : occ;
  c->qlds_floats = query_lds_floats(sh);
  // resident workgroups per compute unit (registers and LDS): the query and
  // exchange grids are persistent, so a grid larger than what is resident
  // would leave its last workgroups to start after the others finish
  for (int q = 0; q < 4; ++q) {
    int nb = 0;
    HIPCHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, query_kernel_ptr(sh, q), c->threads,
                                                          (size_t)c->qlds_floats * 4));
    c->query_occ[q] = std::max(1, nb);
  }
  c->qlds_small_floats = query_lds_floats(sh, 1);
  for (int q = 0; q < 2; ++q) {
    int nb = 0;
    HIPCHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, query_kernel_ptr(sh, q, 1), c->threads,
                                                          (size_t)c->qlds_small_floats * 4));
    c->query_occ_small[q] = std::max(1, nb);
  }
  {
    int nb = 0;
    HIPCHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, exchange_kernel_ptr(sh), c->threads,
                                                          (size_t)c->qlds_floats * 4));
    c->exch_occ = std::max(1, nb);
  }

  // work items: grouped partition and per-subdomain partitions
  std::vector<Item> items;
  for (int s = 0; s < c->n_sub; ++s) tiles_of(c->subs[s], s, c->tile_points, c->value_points, items);
  c->n_items = (int)items.size();
  const int max_wg = c->num_cu * c->step_occ;
  c->n_wg = std::max(1, std::min(c->n_items, max_wg));
  // With several workgroups per compute unit the co-resident ones advance at
  // different rates; ranges handed out in turn (four per workgroup unless the
  // caller's tuning says otherwise) even it out.
  c->dynamic = c->step_occ > 1;
  const int rpw = cfg->ranges_per_wg > 0 ? cfg->ranges_per_wg : 4;
  auto ranges_for = [&](int n_items, int n_wg) {
    return c->dynamic ? std::max(1, std::min(n_items, rpw * n_wg)) : n_wg;
  };
  c->n_ranges = ranges_for(c->n_items, c->n_wg);
  std::vector<int32_t> wg_begin;
  partition(items, c->n_ranges, value_tile_cost(sh), 0, wg_begin, &c->n_seg);
  // segments are numbered in item order, which is sorted by subdomain, so
  // each subdomain owns a contiguous slab range
  std::vector<int32_t> seg_begin(c->n_sub + 1, 0);
  for (size_t i = 0; i < items.size(); ++i)
    if (items[i].flags & ITEM_FIRST) seg_begin[items[i].sub + 1]++;
  for (int s = 0; s < c->n_sub; ++s) seg_begin[s + 1] += seg_begin[s];
  std::vector<Item> items_ps;
  std::vector<int32_t> wgb_ps, seg_ps(c->n_sub + 1, 0);
  c->ps_wg.assign(c->n_sub, 0);
  c->ps_nr.assign(c->n_sub, 0);
  c->ps_wgb_off.assign(c->n_sub, 0);
  {
    int slab0 = 0;
    for (int s = 0; s < c->n_sub; ++s) {
      std::vector<Item> its;
      tiles_of(c->subs[s], s, c->tile_points, c->value_points, its);
      seg_ps[s] = slab0;
      if (its.empty()) continue;
      const int nw = std::max(1, std::min((int)its.size(), max_wg));
      const int nr = ranges_for((int)its.size(), nw);
      std::vector<int32_t> wb;
      int nseg = 0;
      partition(its, nr, value_tile_cost(sh), slab0, wb, &nseg);
      c->ps_wg[s] = nw;
      c->ps_nr[s] = nr;
      c->ps_wgb_off[s] = (int)wgb_ps.size();
      const int base = (int)items_ps.size();
      for (int32_t v : wb) wgb_ps.push_back(v + base);
      items_ps.insert(items_ps.end(), its.begin(), its.end());
      slab0 += nseg;
    }
    seg_ps[c->n_sub] = slab0;
    c->ps_seg = slab0;
    c->ps_items = (int)items_ps.size();
  }
  c->n_slabs = std::max(std::max(c->n_seg, c->ps_seg), 1);
  int max_seg_sub = 1;
  for (int s = 0; s < c->n_sub; ++s) {
    max_seg_sub = std::max(max_seg_sub, seg_begin[s + 1] - seg_begin[s]);
    max_seg_sub = std::max(max_seg_sub, seg_ps[s + 1] - seg_ps[s]);
  }
  c->n_chunks = (max_seg_sub + kSlabChunk - 1) / kSlabChunk;
  const int stash_wg = std::max(c->n_wg, 1);
  const int NCB = (2 * sh.dim + 2) * (c->tile_points / 16);
  c->stash_per_wg = (int64_t)sh.NW * sh.H * NCB * 256;

  // exchange capacity: every ghost point in a half tile, plus one partial tile per face
  int64_t xcap = 0;
  const int xhalf = 16 * (2 * sh.dim + 2) / 2;
  for (int s = 0; s < c->n_sub; ++s) xcap += (c->subs[s].n_gh + xhalf - 1) / xhalf;
  xcap += 8LL * c->n_sub + 64;
  c->x_cap = (int)std::min<int64_t>(xcap, 1 << 24);

  // workspace layout (in memory-check mode each region is followed by a guard zone)
  size_t off = 0;
  const size_t gb = (size_t)cfg->guard_bytes;
  std::vector<std::pair<size_t, size_t>> guards;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    if (gb) {
      guards.emplace_back(off, gb);
      off += gb;
    }
    return o;
  };
  const size_t o_subs = take(sizeof(SubDev) * c->n_sub);
  const size_t o_items = take(sizeof(Item) * std::max(c->n_items, 1));
  const size_t o_wgb = take(sizeof(int32_t) * (c->n_ranges + 1));
  const size_t o_counters = take(sizeof(int32_t) * (1 + c->n_sub));
  const size_t o_segb = take(sizeof(int32_t) * (c->n_sub + 1));
  const size_t o_items_ps = take(sizeof(Item) * std::max(c->ps_items, 1));
  const size_t o_wgb_ps = take(sizeof(int32_t) * std::max<size_t>(wgb_ps.size(), 1));
  const size_t o_seg_ps = take(sizeof(int32_t) * (c->n_sub + 1));
  const size_t o_slabs = take(sizeof(float) * (size_t)c->n_slabs * sh.slab_floats);
  const size_t o_stash = take(sizeof(float) * (size_t)stash_wg * c->stash_per_wg);
  const size_t o_partial = take(sizeof(float) * (size_t)c->n_sub * c->n_chunks * sh.slab_floats);
  const size_t o_frag = take(sizeof(float) * (size_t)c->n_sub * sh.frag_floats);
  const size_t o_loss = take(sizeof(float) * 8 * c->n_sub);
  const int n_gblk = (int)((sh.P + 255) / 256);
  const size_t o_gbuf = take(sizeof(float) * (size_t)c->n_sub * sh.P);
  const size_t o_normpart = take(sizeof(float) * (size_t)c->n_sub * n_gblk);
  const size_t o_clip = take(sizeof(float) * c->n_sub);
  const size_t o_boxes = take(sizeof(float) * 8 * c->n_sub);
  const size_t o_xitems = take(sizeof(ExchangeItem) * c->x_cap);
  const size_t o_targets = take(sizeof(float*) * c->n_sub);
  const size_t total = off;
  if (!workspace) {
    *workspace_bytes = total;
    return PINN_OK;
  }
  if (*workspace_bytes < total)
    return fail(PINN_E_NOMEM, "workspace has %zu bytes, needs %zu", *workspace_bytes, total);

  char* ws = (char*)workspace;
  c->d_subs = (SubDev*)(ws + o_subs);
  c->d_items = (Item*)(ws + o_items);
  c->d_wg_begin = (int32_t*)(ws + o_wgb);
  c->d_counters = (int32_t*)(ws + o_counters);
  c->d_seg_begin = (int32_t*)(ws + o_segb);
  c->d_items_ps = (Item*)(ws + o_items_ps);
  c->d_wgb_ps = (int32_t*)(ws + o_wgb_ps);
  c->d_seg_ps = (int32_t*)(ws + o_seg_ps);
  c->d_slabs = (float*)(ws + o_slabs);
  c->d_stash = (float*)(ws + o_stash);
  c->d_frag = (float*)(ws + o_frag);
  c->d_partial = (float*)(ws + o_partial);
  c->d_loss_ws = (float*)(ws + o_loss);
  c->d_gbuf = (float*)(ws + o_gbuf);
  c->d_normpart = (float*)(ws + o_normpart);
  c->d_clip = (float*)(ws + o_clip);
  c->d_boxes = (float*)(ws + o_boxes);
  c->d_xitems = (ExchangeItem*)(ws + o_xitems);
  c->d_targets = (float**)(ws + o_targets);

  // subdomain descriptors
  std::vector<SubDev> sd(c->n_sub);
  std::vector<float> boxes(8 * c->n_sub, 0.f);
  for (int q = 0; q < 4; ++q) c->gmax[q] = -INFINITY;
  for (int s = 0; s < c->n_sub; ++s) {
    const pinn_subdomain& u = c->subs[s];
    SubDev& d = sd[s];
    std::memset(&d, 0, sizeof d);
    d.theta = u.theta;
    d.m = u.adam_m;
    d.v = u.adam_v;
    d.pde_x = u.pde_x;
    d.obs_x = u.obs_x;
    d.obs_u = u.obs_u;
    d.gh_x = u.gh_x;
    d.gh_up = u.gh_up;
    d.gh_kind = u.gh_kind;
    d.anc_x = u.anc_x;
    d.anc_p = u.anc_p;
    d.frag = c->d_frag + (size_t)s * sh.frag_floats;
    d.n_pde = (int32_t)u.n_pde;
    d.n_obs = (int32_t)u.n_obs;
    d.n_gh = (int32_t)u.n_gh;
    d.n_anc = (int32_t)u.n_anc;
    for (int k = 0; k < 6; ++k) d.lam[k] = cfg->lam[k];
    if (u.is_master) d.lam[3] = 0.f;   // master: no spatial ghost pressure term
    d.inv_n[0] = u.n_pde ? 1.f / (float)u.n_pde : 0.f;
    d.inv_n[1] = u.n_obs ? 1.f / (float)u.n_obs : 0.f;
    d.inv_n[2] = u.n_gh ? 1.f / (float)u.n_gh : 0.f;
    d.inv_n[3] = u.n_anc ? 1.f / (float)u.n_anc : 0.f;
    for (int q = 0; q < 4; ++q) {
      d.lo[q] = u.lo[q];
      d.hi[q] = u.hi[q];
      boxes[s * 8 + q] = u.lo[q];
      boxes[s * 8 + 4 + q] = u.hi[q];
      if (q <= cfg->dim) c->gmax[q] = std::max(c->gmax[q], u.hi[q]);
    }
    d.is_master = u.is_master ? 1 : 0;
    const bool cw_set = cfg->comp_w[0] != 0.f || cfg->comp_w[1] != 0.f || cfg->comp_w[2] != 0.f;
    for (int q = 0; q < 3; ++q) d.cw[q] = cw_set ? cfg->comp_w[q] : 1.f;
    d.cw[3] = 0.f;
  }
  hipStream_t s = (hipStream_t)stream;
  HIPCHECK(hipMemcpyAsync(c->d_subs, sd.data(), sizeof(SubDev) * c->n_sub, hipMemcpyHostToDevice, s));
  if (c->n_items) HIPCHECK(hipMemcpyAsync(c->d_items, items.data(), sizeof(Item) * c->n_items, hipMemcpyHostToDevice, s));
  HIPCHECK(hipMemcpyAsync(c->d_wg_begin, wg_begin.data(), sizeof(int32_t) * (c->n_ranges + 1), hipMemcpyHostToDevice, s));
  HIPCHECK(hipMemcpyAsync(c->d_seg_begin, seg_begin.data(), sizeof(int32_t) * (c->n_sub + 1), hipMemcpyHostToDevice, s));
  if (c->ps_items) HIPCHECK(hipMemcpyAsync(c->d_items_ps, items_ps.data(), sizeof(Item) * c->ps_items, hipMemcpyHostToDevice, s));
  if (!wgb_ps.empty()) HIPCHECK(hipMemcpyAsync(c->d_wgb_ps, wgb_ps.data(), sizeof(int32_t) * wgb_ps.size(), hipMemcpyHostToDevice, s));
  HIPCHECK(hipMemcpyAsync(c->d_seg_ps, seg_ps.data(), sizeof(int32_t) * (c->n_sub + 1), hipMemcpyHostToDevice, s));
  HIPCHECK(hipMemcpyAsync(c->d_boxes, boxes.data(), sizeof(float) * 8 * c->n_sub, hipMemcpyHostToDevice, s));
  c->guards = guards;
  c->ws = ws;
  c->guard_bytes = (int)gb;
  for (const auto& gz : c->guards) HIPCHECK(hipMemsetAsync(ws + gz.first, 0xA5, gz.second, s));

  // kernel argument blocks
  c->pargs.sh = sh;
  c->pargs.subs = c->d_subs;
  c->pargs.n_sub = c->n_sub;
  c->pargs.counters = c->d_counters;
  c->pargs.n_counters = 1 + c->n_sub;
  c->sargs.sh = sh;
  c->sargs.subs = c->d_subs;
  c->sargs.items = c->d_items;
  c->sargs.wg_begin = c->d_wg_begin;
  c->sargs.counter = c->dynamic ? c->d_counters : nullptr;
  c->sargs.n_ranges = c->n_ranges;
  c->sargs.prio = cfg->gemm_priority_off ? 0 : 1;
  c->sargs.slabs = c->d_slabs;
  c->sargs.stash = c->d_stash;
  c->sargs.stash_per_wg = c->stash_per_wg;
  c->sargs.nu = (float)cfg->nu;
  c->sargs.lds_floats = c->lds_floats;
  c->rargs.sh = sh;
  c->rargs.subs = c->d_subs;
  c->rargs.seg_begin = c->d_seg_begin;
  c->rargs.slabs = c->d_slabs;
  c->rargs.partial = c->d_partial;
  c->rargs.n_chunks = c->n_chunks;
  c->rargs.loss_ws = c->d_loss_ws;
  c->rargs.gbuf = c->d_gbuf;
  c->rargs.normpart = c->d_normpart;
  c->rargs.clip_scale = c->d_clip;
  c->rargs.clip = cfg->clip_norm;
  c->rargs.n_sub = c->n_sub;
  c->rargs.lr = cfg->lr;
  c->rargs.beta1 = cfg->beta1;
  c->rargs.beta2 = cfg->beta2;
  c->rargs.eps = cfg->eps;

  HIPCHECK(launch_prep(c->pargs, s));

  if (cfg->flags & PINN_GRAPH) {
    hipGraph_t gr;
    HIPCHECK(hipGraphCreate(&gr, 0));
    hipGraphNode_t n1, n2, n3, n4;
    hipKernelNodeParams kp{};
    void* pa[] = {&c->pargs};
    grid_prep(c->pargs, &kp.gridDim, &kp.blockDim);
    kp.func = (void*)prep_kernel_ptr();
    kp.kernelParams = pa;
    kp.sharedMemBytes = 0;
    HIPCHECK(hipGraphAddKernelNode(&n1, gr, nullptr, 0, &kp));
    void* sa[] = {&c->sargs};
    hipKernelNodeParams ks{};
    ks.func = (void*)step_kernel_ptr(sh, c->tile_points);
    ks.gridDim = dim3(c->n_wg);
    ks.blockDim = dim3(c->threads);
    ks.sharedMemBytes = (unsigned)(c->lds_floats * 4);
    ks.kernelParams = sa;
    HIPCHECK(hipGraphAddKernelNode(&n2, gr, &n1, 1, &ks));
    c->rargs.t = 1;
    c->rargs.update = 0;
    void* ra[] = {&c->rargs};
    hipKernelNodeParams kq{};
    grid_slab_sum(c->rargs, &kq.gridDim, &kq.blockDim);
    kq.func = (void*)slab_sum_kernel_ptr();
    kq.kernelParams = ra;
    hipGraphNode_t n25;
    HIPCHECK(hipGraphAddKernelNode(&n25, gr, &n2, 1, &kq));
    hipKernelNodeParams kg{};
    grid_reduce(c->rargs, &kg.gridDim, &kg.blockDim);
    kg.func = (void*)grad_kernel_ptr();
    kg.kernelParams = ra;
    hipGraphNode_t ng;
    HIPCHECK(hipGraphAddKernelNode(&ng, gr, &n25, 1, &kg));
    c->n_grad = ng;
    hipGraphNode_t last = ng;
    int nblk = (int)kg.gridDim.x;
    void* ca[] = {&c->rargs, &nblk};
    if (cfg->clip_norm > 0.f) {
      hipKernelNodeParams kc{};
      kc.gridDim = dim3(c->n_sub);
      kc.blockDim = dim3(256);
      kc.func = (void*)clip_kernel_ptr();
      kc.kernelParams = ca;
      hipGraphNode_t nc;
      HIPCHECK(hipGraphAddKernelNode(&nc, gr, &ng, 1, &kc));
      last = nc;
    }
    hipKernelNodeParams kr{};
    grid_reduce(c->rargs, &kr.gridDim, &kr.blockDim);
    kr.func = (void*)adam_kernel_ptr();
    kr.kernelParams = ra;
    HIPCHECK(hipGraphAddKernelNode(&n3, gr, &last, 1, &kr));
    HIPCHECK(hipGraphAddKernelNode(&n4, gr, &n3, 1, &kp));
    c->graph = gr;
    c->n_reduce = n3;
    HIPCHECK(hipGraphInstantiate(&c->gexec, gr, nullptr, nullptr, 0));
  }
  HIPCHECK(hipStreamSynchronize(s));

  pinn_ctx* h = new pinn_ctx(std::move(tmp));
  *out = h;
  *workspace_bytes = total;
  return PINN_OK;
}

static pinn_status run_step_eager(pinn_ctx* c, bool per_sub, bool timed, hipStream_t s) {
  HIPCHECK(launch_prep(c->pargs, s));
  ReduceArgs ra = c->rargs;
  // timed launches: the events are tied to the dispatches themselves (start
  // time stamp of the first step-kernel launch, end time stamp of the last),
  // so the measured span holds kernel execution only
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (timed) {
    pinn_status st = next_event_pair(c, &e0, &e1);
    if (st != PINN_OK) return st;
  }
  if (!per_sub) {
    if (c->n_items) {
      if (timed) HIPCHECK(launch_step_timed(c->sargs, c->tile_points, c->n_wg, s, e0, e1));
      else HIPCHECK(launch_step(c->sargs, c->tile_points, c->n_wg, s));
    } else if (timed) {
      HIPCHECK(hipEventRecord(e0, s));
      HIPCHECK(hipEventRecord(e1, s));
    }
  } else {
    // one plain launch per subdomain over its own partition and slabs
    int first = -1, last = -1;
    for (int k = 0; k < c->n_sub; ++k)
      if (c->ps_wg[k]) {
        if (first < 0) first = k;
        last = k;
      }
    if (timed && first < 0) {
      HIPCHECK(hipEventRecord(e0, s));
      HIPCHECK(hipEventRecord(e1, s));
    }
    for (int k = 0; k < c->n_sub; ++k) {
      if (!c->ps_wg[k]) continue;
      StepArgs a = c->sargs;
      a.items = c->d_items_ps;
      a.wg_begin = c->d_wgb_ps + c->ps_wgb_off[k];
      a.counter = c->dynamic ? c->d_counters + 1 + k : nullptr;
      a.n_ranges = c->ps_nr[k];
      if (timed) HIPCHECK(launch_step_timed(a, c->tile_points, c->ps_wg[k], s, k == first ? e0 : nullptr,
                                            k == last ? e1 : nullptr));
      else HIPCHECK(launch_step(a, c->tile_points, c->ps_wg[k], s));
    }
    ra.seg_begin = c->d_seg_ps;
  }
  HIPCHECK(launch_reduce(ra, s));
  HIPCHECK(launch_prep(c->pargs, s));
  return PINN_OK;
}

pinn_status pinn_step(pinn_ctx* c, int64_t t, uint32_t flags, float* loss_out, float* grad_out, void* stream) {
  g_err.clear();
  if (!c) return fail(PINN_E_INVAL, "ctx is NULL");
  if (flags & ~(PINN_NO_UPDATE | PINN_CHECK_FINITE | PINN_PER_SUBDOMAIN | PINN_TIME_KERNEL))
    return fail(PINN_E_INVAL, "unknown step flags 0x%x", flags);
  const bool update = !(flags & PINN_NO_UPDATE);
  if (update && t < 1) return fail(PINN_E_INVAL, "Adam step t must be >= 1 (got %lld)", (long long)t);
  hipStream_t s = (hipStream_t)stream;
  const bool per_sub = flags & PINN_PER_SUBDOMAIN;
  c->rargs.t = update ? t : 1;
  c->rargs.update = update ? 1 : 0;
  c->rargs.loss_out = loss_out;
  c->rargs.grad_out = grad_out;
  // step decay of the learning rate (appendix B): lr * factor^floor((t-1)/interval)
  c->rargs.lr = c->cfg.lr;
  if (c->cfg.lr_interval > 0 && t >= 1)
    c->rargs.lr = (float)((double)c->cfg.lr * std::pow((double)c->cfg.lr_factor, (double)((t - 1) / c->cfg.lr_interval)));
  const bool timed = flags & PINN_TIME_KERNEL;
  if (!per_sub && !timed && c->gexec) {
    void* ra[] = {&c->rargs};
    hipKernelNodeParams kg{};
    grid_reduce(c->rargs, &kg.gridDim, &kg.blockDim);
    kg.func = (void*)grad_kernel_ptr();
    kg.kernelParams = ra;
    HIPCHECK(hipGraphExecKernelNodeSetParams(c->gexec, c->n_grad, &kg));
    hipKernelNodeParams kr{};
    grid_reduce(c->rargs, &kr.gridDim, &kr.blockDim);
    kr.func = (void*)adam_kernel_ptr();
    kr.kernelParams = ra;
    HIPCHECK(hipGraphExecKernelNodeSetParams(c->gexec, c->n_reduce, &kr));
    HIPCHECK(hipGraphLaunch(c->gexec, s));
  } else {
    pinn_status st = run_step_eager(c, per_sub, timed, s);
    if (st != PINN_OK) return st;
  }
  if (flags & PINN_CHECK_FINITE) {
    std::vector<float> L(8 * c->n_sub);
    HIPCHECK(hipMemcpyAsync(L.data(), c->d_loss_ws, sizeof(float) * L.size(), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    for (size_t k = 0; k < L.size(); ++k)
      if (!std::isfinite(L[k])) return fail(PINN_E_NONFINITE, "loss of subdomain %zu is not finite", k / 8);
  }
  return PINN_OK;
}

size_t pinn_query_scratch_bytes(const pinn_ctx* c, int64_t n) {
  if (!c || n < 0) return 0;
  return align256(4 * (size_t)n) * 2 + align256(4 * (size_t)(c->n_sub + 1)) * 3;
}

pinn_status pinn_query(pinn_ctx* c, const float* x, int64_t n, int32_t sub, uint32_t what, float* out,
                       void* scratch, size_t scratch_bytes, void* stream) {
  g_err.clear();
  if (!c) return fail(PINN_E_INVAL, "ctx is NULL");
  if (n < 0) return fail(PINN_E_INVAL, "n < 0");
  if (what > PINN_Q_RESIDUAL) return fail(PINN_E_INVAL, "unknown query kind %u", what);
  if (what == PINN_Q_UVPW && c->sh.dim != 2) return fail(PINN_E_INVAL, "PINN_Q_UVPW needs dim 2");
  if (sub < -1 || sub >= c->n_sub) return fail(PINN_E_INVAL, "sub %d out of range", sub);
  if (n == 0) return PINN_OK;
  if (!x || !out) return fail(PINN_E_INVAL, "x or out is NULL");
  if (n > (int64_t)INT32_MAX) return fail(PINN_E_INVAL, "n too large");
  hipStream_t s = (hipStream_t)stream;
  const Shape& sh = c->sh;
  QueryArgs qa{};
  qa.sh = sh;
  qa.subs = c->d_subs;
  qa.x = x;
  qa.out = out;
  qa.n = n;
  qa.sub = sub;
  qa.n_sub = c->n_sub;
  qa.what = (int32_t)what;
  qa.nu = (float)c->cfg.nu;
  qa.lds_floats = c->qlds_floats;
  const int CF = 2 * sh.dim + 2;
  // requests too small to fill the chip take 16-point tiles: a tile's chain of
  // layers is the latency, and smaller tiles shorten it
  const bool small = what <= PINN_Q_UVPW && n <= 16LL * c->num_cu * c->query_occ_small[what];
  qa.small = small ? 1 : 0;
  if (small) qa.lds_floats = c->qlds_small_floats;
  const int npts = small ? 16 : (what == PINN_Q_VALUE) ? 16 * CF : (what == PINN_Q_UVPW ? 16 * CF / (sh.dim + 1) : 16);
  const int max_wg = c->num_cu * (small ? c->query_occ_small[what] : c->query_occ[what]);
  if (sub >= 0) {
    const int64_t tiles = (n + npts - 1) / npts;
    HIPCHECK(launch_query(qa, (int)std::min<int64_t>(tiles, max_wg), s));
    return PINN_OK;
  }
  if (n > c->cfg.max_query_points)
    return fail(PINN_E_BUDGET, "routed query of %lld points exceeds max_query_points %lld", (long long)n,
                (long long)c->cfg.max_query_points);
  const size_t need = pinn_query_scratch_bytes(c, n);
  if (!scratch || scratch_bytes < need) return fail(PINN_E_NOMEM, "query scratch needs %zu bytes", need);
  if ((uintptr_t)scratch & 255) return fail(PINN_E_INVAL, "scratch must be 256-byte aligned");
  char* p = (char*)scratch;
  RouteArgs ra{};
  ra.x = x;
  ra.n = n;
  ra.boxes = c->d_boxes;
  for (int q = 0; q < 4; ++q) ra.gmax[q] = c->gmax[q];
  ra.n_sub = c->n_sub;
  ra.D = sh.D;
  const int out_cols = (what == PINN_Q_UVPW) ? 4 : (what == PINN_Q_CHANNELS ? CF * sh.D : sh.D);
  ra.out_cols = out_cols;
  ra.sub_id = (int32_t*)p; p += align256(4 * (size_t)n);
  ra.perm = (int32_t*)p;   p += align256(4 * (size_t)n);
  ra.counts = (int32_t*)p; p += align256(4 * (size_t)(c->n_sub + 1));
  ra.cursor = (int32_t*)p; p += align256(4 * (size_t)(c->n_sub + 1));
  ra.offsets = (int32_t*)p;
  ra.out = out;
  HIPCHECK(launch_route(ra, s));
  qa.perm = ra.perm;
  qa.counts = ra.counts;
  qa.offsets = ra.offsets;
  const int64_t tiles = (n + npts - 1) / npts + c->n_sub;
  HIPCHECK(launch_query(qa, (int)std::min<int64_t>(tiles, max_wg), s));
  return PINN_OK;
}

pinn_status pinn_query_noalloc(pinn_ctx* c, const float* x, int64_t n, int32_t sub, uint32_t what, float* out,
                               void* stream) {
  g_err.clear();
  if (!c) return fail(PINN_E_INVAL, "ctx is NULL");
  if (sub == -1 && n > kNoallocQueryPoints)
    return fail(PINN_E_BUDGET, "routed query of %lld points exceeds the %lld points of the library-held scratch",
                (long long)n, (long long)kNoallocQueryPoints);
  if (!c->noalloc_scratch) return fail(PINN_E_DEVICE, "library-held query scratch not resolved");
  // the same launches as pinn_query, on the library-held scratch of this
  // context's device (the scratch covers n <= kNoallocQueryPoints points and
  // up to kMaxSub subdomains)
  return pinn_query(c, x, n, sub, what, out, c->noalloc_scratch, kNoallocScratchBytes, stream);
}

pinn_status pinn_exchange(pinn_ctx* c, const pinn_face* faces, int32_t n_faces, const float* x_anc,
                          float* const* targets, void* stream) {
  g_err.clear();
  if (!c) return fail(PINN_E_INVAL, "ctx is NULL");
  if (n_faces < 0 || (n_faces && (!faces || !targets))) return fail(PINN_E_INVAL, "bad faces/targets");
  if (!x_anc) return fail(PINN_E_INVAL, "x_anc is NULL");
  const Shape& sh = c->sh;
  const int NCOL = 16 * (2 * sh.dim + 2);
  std::vector<ExchangeItem> its;
  for (int f = 0; f < n_faces; ++f) {
    const pinn_face& fc = faces[f];
    if (fc.a < 0 || fc.a >= c->n_sub || fc.b < 0 || fc.b >= c->n_sub)
      return fail(PINN_E_INVAL, "face %d: subdomain out of range", f);
    if (fc.first < 0 || fc.count < 0 || fc.first + fc.count > c->subs[fc.a].n_gh)
      return fail(PINN_E_INVAL, "face %d: ghost range outside subdomain %d", f, fc.a);
    if (!targets[fc.a]) return fail(PINN_E_INVAL, "face %d: targets[%d] is NULL", f, fc.a);
    const int paired = c->subs[fc.b].is_master ? 1 : 0;
    const int tp = paired ? NCOL / 2 : NCOL;
    for (int64_t st = 0; st < fc.count; st += tp)
      its.push_back(ExchangeItem{fc.a, fc.b, (int32_t)(fc.first + st),
                                 (int32_t)std::min<int64_t>(tp, fc.count - st), paired, {0, 0, 0}});
  }
  if ((int)its.size() > c->x_cap) return fail(PINN_E_NOMEM, "exchange needs %zu tiles > capacity %d", its.size(), c->x_cap);
  if (its.empty()) return PINN_OK;
  hipStream_t s = (hipStream_t)stream;
  if (!c->x_done) HIPCHECK(hipEventCreateWithFlags(&c->x_done, hipEventDisableTiming));
  // stream order only, never a host wait: this exchange (its copies of the
  // work list and its launch) runs after the previous exchange, whichever
  // stream that was on, so the device work list is not rewritten under it
  if (c->x_done_recorded) HIPCHECK(hipStreamWaitEvent(s, c->x_done, 0));
  // host copies whose upload has run are released (queried, not waited for)
  for (size_t k = 0; k < c->x_staged.size();) {
    if (hipEventQuery(c->x_staged[k]->copied) == hipSuccess) {
      (void)hipEventDestroy(c->x_staged[k]->copied);
      delete c->x_staged[k];
      c->x_staged[k] = c->x_staged.back();
      c->x_staged.pop_back();
    } else {
      ++k;
    }
  }
  std::vector<float*> tg(targets, targets + c->n_sub);
  const bool same = its.size() == c->x_host.size() &&
                    std::memcmp(its.data(), c->x_host.data(), its.size() * sizeof(ExchangeItem)) == 0 &&
                    tg == c->x_targets_host;
  if (!same) {
    c->x_host = its;
    c->x_targets_host = tg;
    // the upload reads a host copy that lives until the copy has run
    const size_t ib = sizeof(ExchangeItem) * its.size(), tb = sizeof(float*) * c->n_sub;
    auto* st = new pinn_ctx::Staged{std::vector<char>(ib + tb), nullptr};
    std::memcpy(st->bytes.data(), its.data(), ib);
    std::memcpy(st->bytes.data() + ib, tg.data(), tb);
    hipError_t e = hipEventCreateWithFlags(&st->copied, hipEventDisableTiming);
    if (e != hipSuccess) {
      delete st;
      return fail(PINN_E_DEVICE, "hipEventCreate: %s", hipGetErrorString(e));
    }
    c->x_staged.push_back(st);
    HIPCHECK(hipMemcpyAsync(c->d_xitems, st->bytes.data(), ib, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(c->d_targets, st->bytes.data() + ib, tb, hipMemcpyHostToDevice, s));
    HIPCHECK(hipEventRecord(st->copied, s));
  }
  ExchangeArgs ea{};
  ea.sh = sh;
  ea.subs = c->d_subs;
  ea.items = c->d_xitems;
  ea.n_items = (int32_t)its.size();
  ea.lds_floats = c->qlds_floats;
  ea.targets = c->d_targets;
  for (int q = 0; q < sh.dim; ++q) ea.x_anc[q] = x_anc[q];
  HIPCHECK(launch_exchange(ea, (int)std::min<int64_t>((int64_t)its.size(), (int64_t)c->num_cu * c->exch_occ), s));
  HIPCHECK(hipEventRecord(c->x_done, s));
  c->x_done_recorded = true;
  return PINN_OK;
}

pinn_status pinn_kernel_time(pinn_ctx* c, double* total_ms, int64_t* launches) {
  g_err.clear();
  if (!c || !total_ms || !launches) return fail(PINN_E_INVAL, "NULL argument");
  pinn_status st = fold_events(c);
  if (st != PINN_OK) return st;
  *total_ms = c->ev_folded_ms;
  *launches = c->ev_folded_n;
  c->ev_folded_ms = 0.0;
  c->ev_folded_n = 0;
  return PINN_OK;
}

pinn_status pinn_check_guards(pinn_ctx* c, int64_t* bad_bytes, void* stream) {
  g_err.clear();
  if (!c || !bad_bytes) return fail(PINN_E_INVAL, "NULL argument");
  *bad_bytes = 0;
  if (c->guards.empty()) return PINN_OK;
  HIPCHECK(hipStreamSynchronize((hipStream_t)stream));
  std::vector<unsigned char> h((size_t)c->guard_bytes);
  int64_t bad = 0;
  for (const auto& gz : c->guards) {
    HIPCHECK(hipMemcpy(h.data(), c->ws + gz.first, gz.second, hipMemcpyDeviceToHost));
    for (size_t k = 0; k < gz.second; ++k) bad += h[k] != 0xA5;
  }
  *bad_bytes = bad;
  return PINN_OK;
}

size_t pinn_evaluate_scratch_bytes(const pinn_ctx* c, int64_t n, int32_t n_snap, int64_t max_snap) {
  if (!c || n < 0 || n_snap < 1 || max_snap < 0) return 0;
  const int D = c->sh.D;
  const int64_t nblk = std::max<int64_t>(1, (max_snap + kEvalChunk - 1) / kEvalChunk);
  return pinn_query_scratch_bytes(c, n) + 3 * align256(sizeof(float) * (size_t)n * D) +
         align256(sizeof(int64_t) * (n_snap + 1)) + align256(sizeof(int32_t) * (c->n_sub + 1)) +
         align256(sizeof(float) * 2 * n_snap * nblk) +
         align256(sizeof(float) * 2 * (D + 1) * n_snap * nblk);
}

pinn_status pinn_evaluate(pinn_ctx* c, const float* x, const float* ref, int64_t n, const int64_t* snap_off,
                          int32_t n_snap, const float* x_anc, float* err_out, void* scratch,
                          size_t scratch_bytes, void* stream) {
  g_err.clear();
  if (!c) return fail(PINN_E_INVAL, "ctx is NULL");
  if (n < 1 || !x || !ref || !snap_off || n_snap < 1 || !x_anc || !err_out)
    return fail(PINN_E_INVAL, "bad evaluation arguments");
  if (snap_off[0] != 0 || snap_off[n_snap] != n) return fail(PINN_E_INVAL, "snap_off must run from 0 to n");
  int64_t max_snap = 0;
  for (int k = 0; k < n_snap; ++k) {
    if (snap_off[k + 1] < snap_off[k]) return fail(PINN_E_INVAL, "snap_off must be nondecreasing");
    max_snap = std::max(max_snap, snap_off[k + 1] - snap_off[k]);
  }
  if (n > c->cfg.max_query_points) return fail(PINN_E_BUDGET, "evaluation of %lld points exceeds max_query_points", (long long)n);
  const size_t need = pinn_evaluate_scratch_bytes(c, n, n_snap, max_snap);
  if (!scratch || scratch_bytes < need) return fail(PINN_E_NOMEM, "evaluation scratch needs %zu bytes", need);
  if ((uintptr_t)scratch & 255) return fail(PINN_E_INVAL, "scratch must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  const Shape& sh = c->sh;
  const int D = sh.D;
  char* p = (char*)scratch;
  char* qscr = p;
  p += pinn_query_scratch_bytes(c, n);
  float* pred = (float*)p; p += align256(sizeof(float) * (size_t)n * D);
  float* xa = (float*)p;   p += align256(sizeof(float) * (size_t)n * D);
  float* pa = (float*)p;   p += align256(sizeof(float) * (size_t)n * D);
  int64_t* d_off = (int64_t*)p; p += align256(sizeof(int64_t) * (n_snap + 1));
  int32_t* mcounts = (int32_t*)p; p += align256(sizeof(int32_t) * (c->n_sub + 1));
  const int nblk = (int)std::max<int64_t>(1, (max_snap + kEvalChunk - 1) / kEvalChunk);
  float* mpart = (float*)p; p += align256(sizeof(float) * 2 * n_snap * nblk);
  float* epart = (float*)p;
  // routing shared by both value queries
  RouteArgs ra{};
  ra.x = x;
  ra.n = n;
  ra.boxes = c->d_boxes;
  for (int q = 0; q < 4; ++q) ra.gmax[q] = c->gmax[q];
  ra.n_sub = c->n_sub;
  ra.D = D;
  ra.out_cols = D;
  char* r = qscr;
  ra.sub_id = (int32_t*)r;  r += align256(4 * (size_t)n);
  ra.perm = (int32_t*)r;    r += align256(4 * (size_t)n);
  ra.counts = (int32_t*)r;  r += align256(4 * (size_t)(c->n_sub + 1));
  ra.cursor = (int32_t*)r;  r += align256(4 * (size_t)(c->n_sub + 1));
  ra.offsets = (int32_t*)r;
  ra.out = pred;
  HIPCHECK(launch_route(ra, s));
  QueryArgs qa{};
  qa.sh = sh;
  qa.subs = c->d_subs;
  qa.x = x;
  qa.out = pred;
  qa.perm = ra.perm;
  qa.counts = ra.counts;
  qa.offsets = ra.offsets;
  qa.n = n;
  qa.sub = -1;
  qa.n_sub = c->n_sub;
  qa.what = Q_VALUE;
  qa.nu = (float)c->cfg.nu;
  qa.lds_floats = c->qlds_floats;
  const int npts = 16 * (2 * sh.dim + 2);
  const int nwg = (int)std::min<int64_t>((n + npts - 1) / npts + c->n_sub, (int64_t)c->num_cu * c->query_occ[Q_VALUE]);
  HIPCHECK(launch_query(qa, nwg, s));
  // p(x_anc, t) by the same network, only where that network is a master
  HIPCHECK(launch_anchor_points(x, n, D, x_anc, xa, s));
  HIPCHECK(launch_master_counts(c->d_subs, ra.counts, c->n_sub, mcounts, s));
  qa.x = xa;
  qa.out = pa;
  qa.counts = mcounts;
  HIPCHECK(launch_query(qa, nwg, s));
  HIPCHECK(hipMemcpyAsync(d_off, snap_off, sizeof(int64_t) * (n_snap + 1), hipMemcpyHostToDevice, s));
  EvalArgs ea{};
  ea.subs = c->d_subs;
  ea.pred = pred;
  ea.pa = pa;
  ea.ref = ref;
  ea.sub_id = ra.sub_id;
  ea.snap_off = d_off;
  ea.mpart = mpart;
  ea.epart = epart;
  ea.err_out = err_out;
  ea.D = D;
  ea.n_snap = n_snap;
  ea.nblk = nblk;
  HIPCHECK(launch_evaluate(ea, s));
  HIPCHECK(hipStreamSynchronize(s));
  return PINN_OK;
}

pinn_status pinn_refresh(pinn_ctx* c, void* stream) {
  g_err.clear();
  if (!c) return fail(PINN_E_INVAL, "ctx is NULL");
  HIPCHECK(launch_prep(c->pargs, (hipStream_t)stream));
  return PINN_OK;
}

pinn_status pinn_get_launch_info(const pinn_ctx* c, pinn_launch_info* info) {
  if (!c || !info) return fail(PINN_E_INVAL, "NULL argument");
  info->tile_points = c->tile_points;
  info->value_points = c->value_points;
  info->n_wg = c->n_wg;
  info->n_items = c->n_items;
  info->n_segments = c->n_seg;
  info->threads = c->threads;
  info->lds_bytes = (int64_t)c->lds_floats * 4;
  info->stash_bytes = (int64_t)c->n_wg * c->stash_per_wg * 4;
  info->slab_floats = c->sh.slab_floats;
  return PINN_OK;
}

pinn_status pinn_destroy(pinn_ctx* c) {
  g_err.clear();
  if (!c) return PINN_OK;
  hipError_t e = hipDeviceSynchronize();
  for (pinn_ctx::Staged* st : c->x_staged) {
    (void)hipEventDestroy(st->copied);
    delete st;
  }
  if (c->x_done) (void)hipEventDestroy(c->x_done);
  for (hipEvent_t ev : c->ev_start) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : c->ev_stop) (void)hipEventDestroy(ev);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  delete c;
  if (e != hipSuccess) return fail(PINN_E_DEVICE, "device error at destroy: %s", hipGetErrorString(e));
  return PINN_OK;
}

}  // extern "C"
