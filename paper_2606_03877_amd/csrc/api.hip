// C ABI of the msplat library: argument checks, workspace layout and the
// launch sequence of the forward and backward passes.
#include <cstdio>
#include <cstring>
#include <mutex>

#include "common.h"

using namespace msplat;

// Optional per-stage timing with HIP events recorded on the caller's stream
// around each launch; pairs are harvested when read (or when a ring fills).
enum Stage {
  ST_ZERO, ST_PREPROCESS, ST_PACK, ST_BIN_COUNT, ST_SCAN, ST_BIN_FILL, ST_MLP_FWD, ST_COMPOSITE,
  ST_MLP_FIXUP, ST_COMP_ADJ, ST_MLP_BWD, ST_HIT_GEO, ST_GEO_FINAL, ST_SLOT_FWD, ST_SLOT_BWD_HITS,
  ST_SLOT_BWD_PRIMS, ST_HIT_REC, ST_COUNT
};
static const char* kStageNames[ST_COUNT] = {
    "zero", "preprocess", "pack_weights", "bin_count", "scan", "bin_fill", "mlp_forward",
    "composite", "mlp_fixup", "composite_adjoint", "mlp_backward", "hit_geometry", "geo_finalize",
    "slot_forward", "slot_backward_hits", "slot_backward_prims", "hit_records"};
constexpr int kRing = 64;
struct StageTimer {
  hipEvent_t a[kRing], b[kRing];
  int head = 0, pending = 0;
  double total_ms = 0.0;
  int64_t count = 0;
  bool created = false;
};

// work-item sizes recorded by msplat_autotune, per network and workload
struct TuneEntry {
  NetShape n;
  int64_t rays;
  int32_t samples_fixed, samples_min, samples_max, order;
  float samples_per_unit;
  int32_t hits_per_item;
  int32_t group;   // work items per workgroup of the network kernels; 0 = not tuned
};
constexpr int kTuneSlots = 32;

// The workspace of msplat_render_forward_noalloc: a device array of the
// library's own (each device holds its copy until the process ends).  Host
// code never uses this name as an address: msplat_create looks up the
// array's address on its device and keeps it in the context.
static __device__ __align__(256) uint8_t scratch[MSPLAT_NOALLOC_SCRATCH_BYTES];

struct msplat_ctx {
  int device;
  void* scratch_ptr = nullptr;   // this device's scratch array
  bool profiling = false;
  TuneEntry tuned[kTuneSlots];
  int num_tuned = 0;
  StageTimer timers[ST_COUNT];
  DevCounters* host_ctr;   // pinned host mirror of the device counters
  // record of the last successful forward (used to size the backward launch)
  const void* last_ws;
  int64_t last_items;
  int64_t last_hits;
  int64_t last_rays;
  uint64_t last_bytes;
  NetShape last_shape;
  int32_t last_hpi;
  int32_t last_group = 0;   // work items per workgroup of the last forward
};

namespace {

constexpr uint64_t kAlign = 256;
inline uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool shape_of(const msplat_model* m, NetShape* n) {
  if (!m) return false;
  n->P = m->num_prims;
  n->L = m->pe_freqs;
  n->W = m->hidden_width;
  n->D = m->hidden_layers;
  n->NOUT = m->out_dim;
  n->prec = m->precision;
  n->kind = m->primitive;
  if (n->P < 1 || n->L < 1 || n->W < 1 || n->D < 1 || n->NOUT < 4 || n->NOUT > kMaxOut) return false;
  if (n->prec != MSPLAT_FP32 && n->prec != MSPLAT_BF16 && n->prec != MSPLAT_BF16X3) return false;
  if (n->kind != MSPLAT_CHORD && n->kind != MSPLAT_CONTACT) return false;
  int64_t in = n->kind == MSPLAT_CONTACT ? 12 * n->L : 3 + 6 * n->L, np = 0, prev = in;
  for (int j = 0; j < n->D; ++j) {
    np += prev * n->W + n->W;
    prev = n->W;
  }
  np += prev * n->NOUT + n->NOUT;
  n->n_params = (int)np;
  return true;
}

// Lay out the workspace at `base` (may be null to measure).  Returns the bytes
// used for hit capacity `hcap`.
uint64_t layout(const NetShape& n, int64_t R, int64_t hcap, uint8_t* base, Workspace* w) {
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    uint64_t o = off;
    off = align_up(off + bytes);
    return base ? base + o : nullptr;
  };
  Workspace ws{};
  int P = n.P;
  ws.counters = (DevCounters*)take(sizeof(DevCounters));
  ws.geo = (float*)take((uint64_t)P * kGeoStride * 4);
  ws.wpack_bytes = mlp_wpack_bytes(n);
  ws.wpack = (uint8_t*)take((uint64_t)P * ws.wpack_bytes);
  ws.prim_nhit = (int32_t*)take((uint64_t)P * 4);
  ws.prim_off = (int32_t*)take((uint64_t)(P + 1) * 4);
  ws.prim_cursor = (int32_t*)take((uint64_t)P * 4);
  ws.wi_off = (int32_t*)take((uint64_t)(P + 1) * 4);
  ws.gw_off = (int32_t*)take((uint64_t)(P + 1) * 4);
  ws.geo_grad = (float*)take((uint64_t)P * 12 * 4);
  ws.ray_off = (int32_t*)take((uint64_t)(R + 1) * 4);
  int64_t nb = (R + 1023) / 1024;
  ws.scan_tmp = (int32_t*)take((uint64_t)(nb + 1) * 4);
  ws.ray_tf = (float*)take((uint64_t)R * 4);
  int nc = n.NOUT - 1;
  uint64_t H = (uint64_t)hcap;
  ws.hit_prim = (int32_t*)take(H * 4);
  ws.hit_ray = (int32_t*)take(H * 4);
  ws.hit_k = (int32_t*)take(H * 4);
  ws.hit_nused = (int32_t*)take(H * 4);
  ws.hit_tc_hi = (float*)take(H * 4);
  ws.hit_tc_lo = (float*)take(H * 4);
  ws.hit_eta = (float*)take(H * 4);
  ws.hit_sa = (float*)take(H * 4);
  ws.hit_sa_lo = (float*)take(H * 4);
  ws.hit_dlt = (float*)take(H * 4);
  ws.hit_dlt_lo = (float*)take(H * 4);
  ws.hit_pc = (float*)take(H * 12);
  ws.hit_pc_lo = (float*)take(H * 12);
  ws.hit_e = (float*)take(H * 12);
  ws.hit_e_lo = (float*)take(H * 12);
  ws.hit_tau = (float*)take(H * 4);
  ws.hit_cloc = (float*)take(H * 4 * nc);
  ws.hit_sb_hi = (float*)take(H * 4);
  ws.hit_sb_lo = (float*)take(H * 4);
  ws.hit_gsa = (float*)take(H * 4);
  ws.hit_tb = (float*)take(H * 4);
  ws.hit_gtot = (float*)take(H * 4);
  ws.hit_gv = (float*)take(H * 4 * 9);
  ws.phit = (int32_t*)take(H * 4);
  ws.hit_q = (float*)take(H * 4);
  ws.hit_gpc = (float*)take(H * 12);
  ws.slot_on = 0;
  ws.num_rays = R;
  ws.hit_cap = hcap;
  ws.nc = nc;
  if (w) *w = ws;
  return off;
}

// bytes per hit and fixed bytes (for capacity from a given size)
void size_model(const NetShape& n, int64_t R, uint64_t* fixed, uint64_t* per_hit) {
  uint64_t a = layout(n, R, 0, nullptr, nullptr);
  uint64_t b = layout(n, R, 1 << 20, nullptr, nullptr);
  *fixed = a;
  *per_hit = (b - a + (1 << 20) - 1) >> 20;
}

int64_t capacity_of(const NetShape& n, int64_t R, uint64_t bytes) {
  uint64_t fixed, ph;
  size_model(n, R, &fixed, &ph);
  if (bytes <= fixed + 32 * kAlign) return 0;
  int64_t h = (int64_t)((bytes - fixed - 32 * kAlign) / ph);
  while (h > 0 && layout(n, R, h, nullptr, nullptr) > bytes) h -= 1 + h / 1000;
  return h;
}

#define HIPCHK(expr)                       \
  do {                                     \
    hipError_t e_ = (expr);                \
    if (e_ != hipSuccess) return MSPLAT_E_HIP; \
  } while (0)

hipError_t harvest_one(StageTimer& t) {
  int idx = (t.head - t.pending + kRing) % kRing;
  hipError_t e = hipEventSynchronize(t.b[idx]);
  if (e != hipSuccess) return e;
  float ms = 0.f;
  e = hipEventElapsedTime(&ms, t.a[idx], t.b[idx]);
  if (e != hipSuccess) return e;
  t.total_ms += ms;
  t.count += 1;
  t.pending -= 1;
  return hipSuccess;
}

hipError_t create_events(StageTimer& t) {
  if (t.created) return hipSuccess;
  for (int i = 0; i < kRing; ++i) {
    if (hipEventCreate(&t.a[i]) != hipSuccess || hipEventCreate(&t.b[i]) != hipSuccess)
      return hipErrorOutOfMemory;
  }
  t.created = true;
  return hipSuccess;
}

hipError_t stage_begin(msplat_ctx* c, int id, hipStream_t s) {
  if (!c->profiling) return hipSuccess;
  StageTimer& t = c->timers[id];
  hipError_t ce = create_events(t);
  if (ce != hipSuccess) return ce;
  if (t.pending == kRing) {
    hipError_t e = harvest_one(t);
    if (e != hipSuccess) return e;
  }
  return hipEventRecord(t.a[t.head], s);
}

hipError_t stage_end(msplat_ctx* c, int id, hipStream_t s) {
  if (!c->profiling) return hipSuccess;
  StageTimer& t = c->timers[id];
  hipError_t e = hipEventRecord(t.b[t.head], s);
  t.head = (t.head + 1) % kRing;
  t.pending += 1;
  return e;
}

// launch `call` as stage `id` (timed when profiling is on)
#define STAGE(ctx, id, s, call)           \
  do {                                    \
    HIPCHK(stage_begin(ctx, id, s));      \
    HIPCHK(call);                         \
    HIPCHK(stage_end(ctx, id, s));        \
  } while (0)

bool opts_ok(const msplat_opts* o) {
  if (!o) return false;
  if (o->samples_fixed < 0 || o->samples_fixed > kMaxSamplesPerHit) return false;
  if (o->samples_fixed == 0) {
    if (o->samples_min < 1 || o->samples_max > kMaxSamplesPerHit || o->samples_min > o->samples_max)
      return false;
    if (!(o->samples_per_unit > 0.f)) return false;
  }
  if (!(o->t_stop >= 0.f && o->t_stop < 1.f)) return false;
  if (o->order != 0 && o->order != 1) return false;
  if (o->tile_rays && o->order != 1) return false;
  if (o->hits_per_item != 0 && o->hits_per_item != 16 && o->hits_per_item != 32 && o->hits_per_item != 64)
    return false;
  const int32_t g = o->items_per_group;
  if (g != 0 && g != 1 && g != 2 && g != 4 && g != 8) return false;
  return true;
}

bool tune_match(const TuneEntry& t, const NetShape& n, int64_t R, const msplat_opts& o) {
  return t.n.P == n.P && t.n.L == n.L && t.n.W == n.W && t.n.D == n.D && t.n.NOUT == n.NOUT &&
         t.n.prec == n.prec && t.n.kind == n.kind && t.rays == R && t.samples_fixed == o.samples_fixed &&
         t.samples_min == o.samples_min && t.samples_max == o.samples_max && t.order == o.order &&
         t.samples_per_unit == o.samples_per_unit;
}

// work-item size of a call: the option, else the recorded choice, else 64
int32_t hits_per_item_of(const msplat_ctx* c, const NetShape& n, int64_t R, const msplat_opts& o) {
  if (o.hits_per_item) return o.hits_per_item;
  for (int i = 0; i < c->num_tuned; ++i)
    if (tune_match(c->tuned[i], n, R, o)) return c->tuned[i].hits_per_item;
  return kHitsPerItem;
}

// work items per workgroup of the network kernels: the option, else the
// recorded choice, else the most (up to 8) that leave at least 2048
// workgroups (eight per CU)
int32_t group_of(const msplat_ctx* c, const NetShape& n, int64_t R, const msplat_opts& o, int64_t items) {
  if (o.items_per_group) return o.items_per_group;
  for (int i = 0; i < c->num_tuned; ++i)
    if (tune_match(c->tuned[i], n, R, o) && c->tuned[i].group) return c->tuned[i].group;
  int32_t g = 1;
  while (g < 8 && items >= (int64_t)2048 * 2 * g) g *= 2;
  return g;
}

// the options a call runs with: the contact-point primitive has one
// interaction per hit (K = 1, no sample offsets)
msplat_opts effective_opts(const NetShape& n, const msplat_opts& o) {
  msplat_opts e = o;
  if (n.kind == MSPLAT_CONTACT) {
    e.samples_fixed = 1;
    e.jitter = 0;
  }
  return e;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

extern "C" {

const char* msplat_status_string(int s) {
  switch (s) {
    case MSPLAT_OK: return "ok";
    case MSPLAT_E_INVALID: return "invalid argument";
    case MSPLAT_E_CAPACITY: return "workspace too small";
    case MSPLAT_E_UNSUPPORTED: return "unsupported network shape or precision";
    case MSPLAT_E_HIP: return "HIP runtime error";
    case MSPLAT_E_STATE: return "no matching forward pass";
    default: return "unknown status";
  }
}

int msplat_create(int device, msplat_ctx** out) {
  if (!out) return MSPLAT_E_INVALID;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess) return MSPLAT_E_HIP;
  if (device < 0 || device >= ndev) return MSPLAT_E_INVALID;
  DeviceGuard dg(device);
  msplat_ctx* c = new msplat_ctx();
  c->device = device;
  // the scratch array's address on this device (the device is current)
  if (hipGetSymbolAddress(&c->scratch_ptr, HIP_SYMBOL(scratch)) != hipSuccess || !c->scratch_ptr) {
    delete c;
    return MSPLAT_E_HIP;
  }
  c->last_ws = nullptr;
  c->last_items = -1;
  c->last_hits = -1;
  if (hipHostMalloc((void**)&c->host_ctr, sizeof(DevCounters), hipHostMallocDefault) != hipSuccess) {
    delete c;
    return MSPLAT_E_HIP;
  }
  *out = c;
  return MSPLAT_OK;
}

void msplat_destroy(msplat_ctx* c) {
  if (!c) return;
  {
    DeviceGuard dg(c->device);
    for (auto& t : c->timers)
      if (t.created)
        for (int i = 0; i < kRing; ++i) {
          (void)hipEventDestroy(t.a[i]);
          (void)hipEventDestroy(t.b[i]);
        }
    (void)hipHostFree(c->host_ctr);
  }
  delete c;
}

int msplat_profile_enable(msplat_ctx* c, int enable) {
  if (!c) return MSPLAT_E_INVALID;
  DeviceGuard dg(c->device);
  for (auto& t : c->timers) {
    while (t.pending > 0)
      if (harvest_one(t) != hipSuccess) return MSPLAT_E_HIP;
    t.total_ms = 0.0;
    t.count = 0;
    // every stage's events exist before the first timed launch
    if (enable && create_events(t) != hipSuccess) return MSPLAT_E_HIP;
  }
  c->profiling = enable != 0;
  return MSPLAT_OK;
}

int msplat_profile_read(msplat_ctx* c, int max_stages, const char** names, double* total_ms,
                        int64_t* launches, int* num_stages) {
  if (!c || !num_stages || max_stages < 0) return MSPLAT_E_INVALID;
  DeviceGuard dg(c->device);
  *num_stages = ST_COUNT;
  for (int i = 0; i < ST_COUNT; ++i) {
    StageTimer& t = c->timers[i];
    while (t.pending > 0)
      if (harvest_one(t) != hipSuccess) return MSPLAT_E_HIP;
    if (i < max_stages) {
      if (names) names[i] = kStageNames[i];
      if (total_ms) total_ms[i] = t.total_ms;
      if (launches) launches[i] = t.count;
    }
  }
  return MSPLAT_OK;
}

int64_t msplat_num_params(const msplat_model* m) {
  NetShape n;
  if (!shape_of(m, &n)) return 0;
  return n.n_params;
}

int msplat_workspace_size(const msplat_model* m, int64_t num_rays, int64_t max_hits, uint64_t* bytes) {
  NetShape n;
  if (!bytes || !shape_of(m, &n) || num_rays < 0 || max_hits < 0) return MSPLAT_E_INVALID;
  if (num_rays >= ((int64_t)1 << 31) || max_hits > kMaxHits) return MSPLAT_E_INVALID;
  if (!mlp_supported(n)) return MSPLAT_E_UNSUPPORTED;
  *bytes = layout(n, num_rays, max_hits, nullptr, nullptr) + 32 * kAlign;
  return MSPLAT_OK;
}

int msplat_render_forward(msplat_ctx* ctx, const msplat_model* m, const msplat_opts* o,
                          const float* center, const float* scale, const float* quat, const float* mlp,
                          const float* ray_o, const float* ray_d, int64_t R, float* rgb, float* trans,
                          float* feat, void* wsp, uint64_t ws_bytes, uint64_t* need_bytes, void* stream) {
  NetShape n;
  if (!ctx || !shape_of(m, &n) || !opts_ok(o)) return MSPLAT_E_INVALID;
  const msplat_opts eo = effective_opts(n, *o);
  o = &eo;
  if (!center || !scale || !quat || !mlp || !wsp || R < 0 || R >= (int64_t)1 << 31) return MSPLAT_E_INVALID;
  if (R > 0 && (!ray_o || !ray_d || !rgb || !trans)) return MSPLAT_E_INVALID;
  int cf = n.NOUT - 4;
  if (cf > 0 && R > 0 && !feat) return MSPLAT_E_INVALID;
  if (((uintptr_t)wsp) % kAlign) return MSPLAT_E_INVALID;
  if (!mlp_supported(n)) return MSPLAT_E_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  DeviceGuard dg(ctx->device);
  int64_t hcap = capacity_of(n, R, ws_bytes);
  uint64_t need0 = layout(n, R, 0, nullptr, nullptr) + 32 * kAlign;
  if (ws_bytes < need0) {
    if (need_bytes) *need_bytes = need0;
    return MSPLAT_E_CAPACITY;
  }
  Workspace ws;
  layout(n, R, hcap, (uint8_t*)wsp, &ws);
  ws.hits_per_item = hits_per_item_of(ctx, n, R, *o);
  ctx->last_ws = nullptr;
  STAGE(ctx, ST_ZERO, s, launch_zero(ws.counters, sizeof(DevCounters), s));
  STAGE(ctx, ST_ZERO, s, launch_zero(ws.prim_nhit, (size_t)n.P * 4, s));
  STAGE(ctx, ST_ZERO, s, launch_zero(ws.ray_off, 4, s));
  // min |g| starts at +inf
  STAGE(ctx, ST_ZERO, s, launch_fill(&ws.counters->min_abs_g_bits, 4, 0x7f800000u, s));
  STAGE(ctx, ST_PREPROCESS, s, launch_preprocess(ws, center, scale, quat, n.P, n.kind, s));
  STAGE(ctx, ST_PACK, s, launch_pack_weights(n, ws, mlp, s));
  STAGE(ctx, ST_BIN_COUNT, s, launch_bin_count(ws, ray_o, ray_d, center, scale, quat, R, n.P, *o, n.kind, s));
  STAGE(ctx, ST_SCAN, s, launch_scans(ws, R, n, s));
  HIPCHK(hipMemcpyAsync(ctx->host_ctr, ws.counters, sizeof(DevCounters), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  // more hits than 32-bit offsets address: the 32-bit scans have wrapped, so
  // nothing after them is launched
  if (ctx->host_ctr->hit_total > kMaxHits) return MSPLAT_E_INVALID;
  int64_t nh = ctx->host_ctr->num_hits;
  int64_t items = ctx->host_ctr->num_work_items;
  if (nh > hcap) {
    if (need_bytes) *need_bytes = layout(n, R, nh, nullptr, nullptr) + 32 * kAlign;
    return MSPLAT_E_CAPACITY;
  }
  if (need_bytes) *need_bytes = layout(n, R, nh, nullptr, nullptr) + 32 * kAlign;
  STAGE(ctx, ST_BIN_FILL, s, launch_bin_fill(ws, ray_o, ray_d, center, scale, quat, R, n.P, *o, n.kind, s));
  STAGE(ctx, ST_HIT_REC, s, launch_hit_records(ws, ray_o, ray_d, nh, n.kind, s));
  const int32_t group = group_of(ctx, n, R, *o, items);
  STAGE(ctx, ST_MLP_FWD, s, launch_mlp_forward(n, ws, *o, nh, group, 0, rgb, trans, feat, s));
  STAGE(ctx, ST_COMPOSITE, s, launch_composite(ws, R, *o, rgb, trans, feat, cf, s));
  if (o->t_stop > 0.f)
    STAGE(ctx, ST_MLP_FIXUP, s, launch_mlp_forward(n, ws, *o, nh, group, 1, rgb, trans, feat, s));
  ctx->last_ws = wsp;
  ctx->last_items = items;
  ctx->last_hits = nh;
  ctx->last_rays = R;
  ctx->last_bytes = ws_bytes;
  ctx->last_shape = n;
  ctx->last_hpi = ws.hits_per_item;
  ctx->last_group = group;
  return MSPLAT_OK;
}

int msplat_render_forward_noalloc(msplat_ctx* ctx, const msplat_model* m, const msplat_opts* o,
                                  const float* center, const float* scale, const float* quat, const float* mlp,
                                  const float* ray_o, const float* ray_d, int64_t R, float* rgb, float* trans,
                                  float* feat, uint64_t* need_bytes, void* stream) {
  if (!ctx || !ctx->scratch_ptr) return MSPLAT_E_INVALID;
  // every launch of the forward clears what it reads before writing it (the
  // counters, per-primitive counts and the first ray offset), so the array's
  // contents from an earlier call do not matter
  return msplat_render_forward(ctx, m, o, center, scale, quat, mlp, ray_o, ray_d, R, rgb, trans, feat,
                               ctx->scratch_ptr, MSPLAT_NOALLOC_SCRATCH_BYTES, need_bytes, stream);
}

// slot-feature arguments of a backward (null when it carries none)
struct SlotArgs {
  const float* slots;
  int C;
  const float* grad_slot;
  float* g_slots;
};

// C, pointers and alignment of slot-feature arrays (float4 accesses)
static bool slot_args_ok(const float* slots, int C, const void* a, const void* b) {
  if (!slots || C <= 0 || C % 4 != 0 || C > (1 << 16)) return false;
  for (const void* q : {(const void*)slots, a, b})
    if (q && ((uintptr_t)q % 16) != 0) return false;
  return true;
}

// the forward state a call on `wsp` relies on: (work items, hits), or an error
// (the workspace layout follows from the model, the ray count and the byte
// size: a call whose arguments differ from the forward's would read it at
// other offsets, so that is refused)
static bool same_net(const NetShape& a, const NetShape& b) {
  return a.P == b.P && a.L == b.L && a.W == b.W && a.D == b.D && a.NOUT == b.NOUT && a.prec == b.prec &&
         a.n_params == b.n_params && a.kind == b.kind;
}

static int forward_state(msplat_ctx* ctx, const NetShape& n, Workspace& ws, const void* wsp, int64_t R,
                         uint64_t ws_bytes, int64_t hcap, hipStream_t s, int64_t* items, int64_t* nh) {
  if (ctx->last_ws == wsp && ctx->last_rays == R && ctx->last_bytes == ws_bytes && same_net(ctx->last_shape, n)) {
    *items = ctx->last_items;
    *nh = ctx->last_hits;
    ws.hits_per_item = ctx->last_hpi;
  } else {
    // workspace of an earlier forward: read its counters
    HIPCHK(hipMemcpyAsync(ctx->host_ctr, ws.counters, sizeof(DevCounters), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const DevCounters& c = *ctx->host_ctr;
    // (the packed operands, whose size depends on the precision, precede the
    // hit arrays: another network or precision would read them elsewhere)
    if (c.magic != kCountersMagic || c.num_rays != R || c.hit_cap != hcap || c.num_prims != n.P ||
        c.num_params != n.n_params || c.net[0] != n.L || c.net[1] != n.W || c.net[2] != n.D ||
        c.net[3] != n.NOUT || c.net[4] != n.prec || c.net[5] != n.kind)
      return MSPLAT_E_STATE;
    if (c.hits_per_item != 16 && c.hits_per_item != 32 && c.hits_per_item != 64) return MSPLAT_E_STATE;
    *items = c.num_work_items;
    *nh = c.num_hits;
    ws.hits_per_item = c.hits_per_item;
  }
  if (*nh > hcap) return MSPLAT_E_STATE;
  return MSPLAT_OK;
}

static int backward_impl(msplat_ctx* ctx, const msplat_model* m, const msplat_opts* o, const float* center,
                         const float* scale, const float* quat, const float* mlp, const float* ray_o,
                         const float* ray_d, int64_t R, const float* grad_rgb, const float* grad_trans,
                         const float* grad_feat, void* wsp, uint64_t ws_bytes, float* g_center, float* g_scale,
                         float* g_quat, float* g_mlp, const SlotArgs* sa, void* stream) {
  NetShape n;
  if (!ctx || !shape_of(m, &n) || !opts_ok(o)) return MSPLAT_E_INVALID;
  const msplat_opts eo = effective_opts(n, *o);
  o = &eo;
  if (!center || !scale || !quat || !mlp || !wsp || R < 0) return MSPLAT_E_INVALID;
  if (!g_center || !g_scale || !g_quat || !g_mlp) return MSPLAT_E_INVALID;
  if (R > 0 && (!ray_o || !ray_d || !grad_rgb)) return MSPLAT_E_INVALID;
  if (sa && (!slot_args_ok(sa->slots, sa->C, sa->grad_slot, sa->g_slots) || !sa->g_slots ||
             (R > 0 && !sa->grad_slot)))
    return MSPLAT_E_INVALID;
  if (!mlp_supported(n) || (sa && n.kind != MSPLAT_CHORD)) return MSPLAT_E_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  DeviceGuard dg(ctx->device);
  int64_t hcap = capacity_of(n, R, ws_bytes);
  Workspace ws;
  layout(n, R, hcap, (uint8_t*)wsp, &ws);
  int64_t items, nh;
  int st = forward_state(ctx, n, ws, wsp, R, ws_bytes, hcap, s, &items, &nh);
  if (st != MSPLAT_OK) return st;
  int cf = n.NOUT - 4;
  STAGE(ctx, ST_ZERO, s, launch_zero(g_mlp, (size_t)n.P * n.n_params * 4, s));
  STAGE(ctx, ST_ZERO, s, launch_zero(ws.geo_grad, (size_t)n.P * 12 * 4, s));
  if (sa) {
    STAGE(ctx, ST_ZERO, s, launch_zero(sa->g_slots, (size_t)n.P * 4 * sa->C * 4, s));
    STAGE(ctx, ST_SLOT_BWD_HITS, s, launch_slot_backward_hits(ws, R, sa->slots, sa->C, sa->grad_slot, s));
    ws.slot_on = 1;
  }
  STAGE(ctx, ST_COMP_ADJ, s,
        launch_composite_adjoint(ws, R, *o, grad_rgb, grad_trans, cf > 0 ? grad_feat : nullptr, cf,
                                 ws.ray_tf, s));
  const int32_t group = group_of(ctx, n, R, *o, items);
  STAGE(ctx, ST_MLP_BWD, s,
        launch_mlp_backward(n, ws, *o, nh, group, ray_d, grad_rgb, cf > 0 ? grad_feat : nullptr, g_mlp, s));
  if (sa)
    STAGE(ctx, ST_SLOT_BWD_PRIMS, s,
          launch_slot_backward_prims(ws, n.P, (int)items, sa->slots, sa->C, sa->grad_slot, ray_d, sa->g_slots,
                                     s));
  STAGE(ctx, ST_HIT_GEO, s, launch_hit_geometry(ws, ray_d, nh, n.kind, s));
  STAGE(ctx, ST_GEO_FINAL, s, launch_geo_finalize(ws, n.P, g_center, g_scale, g_quat, n.kind, s));
  return MSPLAT_OK;
}

int msplat_render_backward(msplat_ctx* ctx, const msplat_model* m, const msplat_opts* o,
                           const float* center, const float* scale, const float* quat, const float* mlp,
                           const float* ray_o, const float* ray_d, int64_t R, const float* grad_rgb,
                           const float* grad_trans, const float* grad_feat, void* wsp,
                           uint64_t ws_bytes, float* g_center, float* g_scale, float* g_quat,
                           float* g_mlp, void* stream) {
  return backward_impl(ctx, m, o, center, scale, quat, mlp, ray_o, ray_d, R, grad_rgb, grad_trans, grad_feat,
                       wsp, ws_bytes, g_center, g_scale, g_quat, g_mlp, nullptr, stream);
}

int msplat_slot_forward(msplat_ctx* ctx, const msplat_model* m, const float* slots, int32_t slot_dim,
                        int64_t R, float* out, const void* wsp, uint64_t ws_bytes, void* stream) {
  NetShape n;
  if (!ctx || !shape_of(m, &n) || !wsp || R < 0) return MSPLAT_E_INVALID;
  if (!slot_args_ok(slots, slot_dim, out, nullptr) || (R > 0 && !out)) return MSPLAT_E_INVALID;
  if (n.kind != MSPLAT_CHORD) return MSPLAT_E_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  DeviceGuard dg(ctx->device);
  int64_t hcap = capacity_of(n, R, ws_bytes);
  Workspace ws;
  layout(n, R, hcap, (uint8_t*)const_cast<void*>(wsp), &ws);
  int64_t items, nh;
  int st = forward_state(ctx, n, ws, wsp, R, ws_bytes, hcap, s, &items, &nh);
  if (st != MSPLAT_OK) return st;
  STAGE(ctx, ST_SLOT_FWD, s, launch_slot_forward(ws, R, slots, slot_dim, out, s));
  return MSPLAT_OK;
}

int msplat_render_backward_slots(msplat_ctx* ctx, const msplat_model* m, const msplat_opts* o,
                                 const float* center, const float* scale, const float* quat, const float* mlp,
                                 const float* ray_o, const float* ray_d, int64_t R, const float* grad_rgb,
                                 const float* grad_trans, const float* grad_feat, const float* slots,
                                 int32_t slot_dim, const float* grad_slot, void* wsp, uint64_t ws_bytes,
                                 float* g_center, float* g_scale, float* g_quat, float* g_mlp, float* g_slots,
                                 void* stream) {
  SlotArgs sa{slots, slot_dim, grad_slot, g_slots};
  return backward_impl(ctx, m, o, center, scale, quat, mlp, ray_o, ray_d, R, grad_rgb, grad_trans, grad_feat,
                       wsp, ws_bytes, g_center, g_scale, g_quat, g_mlp, &sa, stream);
}

int msplat_autotune(msplat_ctx* ctx, const msplat_model* m, const msplat_opts* o, const float* center,
                    const float* scale, const float* quat, const float* mlp, const float* ray_o, const float* ray_d,
                    int64_t R, float* rgb, float* trans, float* feat, const float* grad_rgb, void* wsp,
                    uint64_t ws_bytes, float* g_center, float* g_scale, float* g_quat, float* g_mlp,
                    int32_t* chosen, int32_t* chosen_group, void* stream) {
  NetShape n;
  if (!ctx || !chosen || !shape_of(m, &n) || !opts_ok(o)) return MSPLAT_E_INVALID;
  if (grad_rgb && (!g_center || !g_scale || !g_quat || !g_mlp)) return MSPLAT_E_INVALID;
  const msplat_opts key = effective_opts(n, *o);
  hipStream_t s = (hipStream_t)stream;
  DeviceGuard dg(ctx->device);
  hipEvent_t ev[2];
  if (hipEventCreate(&ev[0]) != hipSuccess) return MSPLAT_E_HIP;
  if (hipEventCreate(&ev[1]) != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return MSPLAT_E_HIP;
  }
  auto fwd = [&](const msplat_opts& oc) {
    return msplat_render_forward(ctx, m, &oc, center, scale, quat, mlp, ray_o, ray_d, R, rgb, trans, feat, wsp,
                                 ws_bytes, nullptr, stream);
  };
  auto bwd = [&](const msplat_opts& oc) {
    return msplat_render_backward(ctx, m, &oc, center, scale, quat, mlp, ray_o, ray_d, R, grad_rgb, nullptr,
                                  nullptr, wsp, ws_bytes, g_center, g_scale, g_quat, g_mlp, stream);
  };
  // runs `step` twice (the first run warms up) and times the second
  auto timed = [&](auto step, float* ms) {
    int st = step();
    if (st == MSPLAT_OK && hipEventRecord(ev[0], s) != hipSuccess) st = MSPLAT_E_HIP;
    if (st == MSPLAT_OK) st = step();
    if (st == MSPLAT_OK && hipEventRecord(ev[1], s) != hipSuccess) st = MSPLAT_E_HIP;
    if (st == MSPLAT_OK && (hipEventSynchronize(ev[1]) != hipSuccess ||
                            hipEventElapsedTime(ms, ev[0], ev[1]) != hipSuccess))
      st = MSPLAT_E_HIP;
    return st;
  };
  const int32_t cand[3] = {64, 32, 16};
  int32_t best = 0, best_group = 0;
  float best_ms = 0.f;
  int st = MSPLAT_OK;
  for (int c = 0; c < 3 && st == MSPLAT_OK; ++c) {
    msplat_opts oc = *o;
    oc.hits_per_item = cand[c];
    float ms = 0.f;
    st = timed([&] {
      int r = fwd(oc);
      return (r == MSPLAT_OK && grad_rgb) ? bwd(oc) : r;
    }, &ms);
    if (st == MSPLAT_OK && (best == 0 || ms < best_ms)) {
      best = cand[c];
      best_ms = ms;
    }
  }
  if (st == MSPLAT_OK && o->items_per_group == 0) {
    msplat_opts oc = *o;
    oc.hits_per_item = best;
    const int32_t gcand[4] = {1, 2, 4, 8};
    float gbest_ms = 0.f;
    for (int c = 0; c < 4 && st == MSPLAT_OK; ++c) {
      oc.items_per_group = gcand[c];
      float ms = 0.f;
      st = timed([&] {
        int r = fwd(oc);
        return (r == MSPLAT_OK && grad_rgb) ? bwd(oc) : r;
      }, &ms);
      if (st == MSPLAT_OK && (best_group == 0 || ms < gbest_ms)) {
        best_group = gcand[c];
        gbest_ms = ms;
      }
    }
  } else {
    best_group = o->items_per_group;
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (st != MSPLAT_OK) return st;
  TuneEntry e{n, R, key.samples_fixed, key.samples_min, key.samples_max, key.order, key.samples_per_unit, best,
              best_group};
  int slot = -1;
  for (int i = 0; i < ctx->num_tuned; ++i)
    if (tune_match(ctx->tuned[i], n, R, key)) slot = i;
  if (slot < 0) slot = ctx->num_tuned < kTuneSlots ? ctx->num_tuned++ : kTuneSlots - 1;
  ctx->tuned[slot] = e;
  *chosen = best;
  if (chosen_group) *chosen_group = best_group;
  return MSPLAT_OK;
}

int msplat_get_stats(msplat_ctx* ctx, const void* wsp, uint64_t ws_bytes, msplat_stats* out, void* stream) {
  if (!ctx || !wsp || !out) return MSPLAT_E_INVALID;
  if (ctx->last_ws != wsp) return MSPLAT_E_STATE;
  DeviceGuard dg(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipMemcpyAsync(ctx->host_ctr, wsp, sizeof(DevCounters), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const DevCounters& c = *ctx->host_ctr;
  std::memset(out, 0, sizeof(*out));
  out->num_rays = ctx->last_rays;
  out->num_hits = c.num_hits;
  out->num_samples = c.num_samples;
  out->num_work_items = c.num_work_items;
  out->num_terminated = c.num_terminated;
  out->num_fallbacks = c.num_fallbacks;
  float mg;
  std::memcpy(&mg, &c.min_abs_g_bits, 4);
  out->min_abs_g = mg;
  out->hits_per_item = c.hits_per_item;
  out->items_per_group = ctx->last_group;
  (void)ws_bytes;
  return MSPLAT_OK;
}

int msplat_debug_hits(msplat_ctx* ctx, const void* wsp, uint64_t ws_bytes, int64_t num_rays,
                      int64_t* ray_off, int32_t* prim, double* t_c, int32_t* n_used, int64_t capacity,
                      void* stream) {
  if (!ctx || !wsp || !ray_off || !prim || !t_c || !n_used || capacity < 0) return MSPLAT_E_INVALID;
  if (ctx->last_ws != wsp || ctx->last_rays != num_rays || ctx->last_bytes != ws_bytes)
    return MSPLAT_E_STATE;
  int64_t nh = ctx->last_hits;
  if (nh > capacity) return MSPLAT_E_CAPACITY;
  DeviceGuard dg(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  Workspace ws;
  layout(ctx->last_shape, num_rays, capacity_of(ctx->last_shape, num_rays, ws_bytes), (uint8_t*)wsp, &ws);
  int32_t* off32 = new int32_t[num_rays + 1];
  float* hi = new float[nh > 0 ? nh : 1];
  float* lo = new float[nh > 0 ? nh : 1];
  int rc = MSPLAT_OK;
  if (hipMemcpyAsync(off32, ws.ray_off, (num_rays + 1) * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
      (nh > 0 && (hipMemcpyAsync(prim, ws.hit_prim, nh * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
                  hipMemcpyAsync(n_used, ws.hit_nused, nh * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
                  hipMemcpyAsync(hi, ws.hit_tc_hi, nh * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
                  hipMemcpyAsync(lo, ws.hit_tc_lo, nh * 4, hipMemcpyDeviceToHost, s) != hipSuccess)) ||
      hipStreamSynchronize(s) != hipSuccess) {
    rc = MSPLAT_E_HIP;
  } else {
    for (int64_t i = 0; i <= num_rays; ++i) ray_off[i] = off32[i];
    for (int64_t i = 0; i < nh; ++i) t_c[i] = (double)hi[i] + (double)lo[i];
  }
  delete[] off32;
  delete[] hi;
  delete[] lo;
  return rc;
}

int msplat_render_forward_f64(msplat_ctx* ctx, const msplat_model* m, const msplat_opts* o,
                              const double* center, const double* scale, const double* quat,
                              const double* mlp, const double* ray_o, const double* ray_d,
                              int64_t R, double* rgb, double* trans, double* feat,
                              uint32_t* decisions, void* wsp, uint64_t ws_bytes, uint64_t* need_bytes,
                              void* stream) {
  NetShape n;
  if (!ctx || !shape_of(m, &n) || !opts_ok(o)) return MSPLAT_E_INVALID;
  if (!center || !scale || !quat || !mlp || !wsp || R < 0) return MSPLAT_E_INVALID;
  if (R > 0 && (!ray_o || !ray_d || !rgb || !trans)) return MSPLAT_E_INVALID;
  if (n.NOUT > 4 && R > 0 && !feat) return MSPLAT_E_INVALID;
  if (!mlp_supported(n) || o->order != 0 || n.kind != MSPLAT_CHORD) return MSPLAT_E_UNSUPPORTED;
  if (need_bytes) *need_bytes = 256;
  if (ws_bytes < 256) return MSPLAT_E_CAPACITY;
  hipStream_t s = (hipStream_t)stream;
  DeviceGuard dg(ctx->device);
  HIPCHK(launch_forward_f64(n, *o, center, scale, quat, mlp, ray_o, ray_d, R, rgb, trans, feat, decisions,
                            wsp, ws_bytes, 0, s));
  HIPCHK(hipMemcpyAsync(ctx->host_ctr, wsp, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  // more hits on one ray than the float64 checker keeps: refuse rather than truncate
  if (*reinterpret_cast<int32_t*>(ctx->host_ctr) != 0) return MSPLAT_E_CAPACITY;
  return MSPLAT_OK;
}

}  // extern "C"
