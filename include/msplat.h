/*
 * msplat.h -- C ABI of the MLP-Splatting render path on AMD MI355X (gfx950).
 *
 * The library renders camera rays against a set of neural primitives
 * (Sec. 3 of "MLP Splatting: Object-Centric Neural Fields"): every ray is
 * intersected with each primitive's ellipsoidal support, the hits are sorted by
 * contact depth, each primitive's own MLP is evaluated at stratified samples of
 * its hit interval, and the samples are composited front to back with early
 * termination.  The backward pass returns the gradients of a scalar loss with
 * respect to every primitive parameter.
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers owned by the caller, dense, row-major,
 *     float32 unless stated.  The library never allocates device memory and
 *     never frees caller memory.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on
 *     it; a call returns once its work is enqueued, except that
 *     msplat_render_forward synchronises `stream` once (to size its launches)
 *     and msplat_get_stats / msplat_debug_hits synchronise before returning.
 *   - Every entry point returns an msplat_status; arguments are validated on
 *     the host before anything is enqueued.  NaN or non-positive scales in the
 *     data are not checked on the device; NaN propagates to the outputs.
 *   - Calls that share a workspace must be serialised by the caller.
 */
#ifndef MSPLAT_H
#define MSPLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum msplat_status {
  MSPLAT_OK = 0,
  MSPLAT_E_INVALID = 1,     /* null pointer, bad size or option (host check) */
  MSPLAT_E_CAPACITY = 2,    /* workspace too small; *need_bytes tells how much */
  MSPLAT_E_UNSUPPORTED = 3, /* network shape or precision that is not compiled */
  MSPLAT_E_HIP = 4,         /* a HIP runtime call failed */
  MSPLAT_E_STATE = 5        /* backward or debug call without a matching forward */
} msplat_status;

typedef enum msplat_precision {
  MSPLAT_FP32 = 0, /* MLP products and sums in float32 (matrix cores, f32 operands) */
  MSPLAT_BF16 = 1, /* MLP operands in bfloat16 on the matrix cores, float32 accumulation */
  MSPLAT_BF16X3 = 2 /* weights and activations as hi + lo bfloat16 pairs, products
                       hi*hi + hi*lo + lo*hi on the matrix cores, float32 accumulation
                       (about 16 significant bits; three times the matrix work) */
} msplat_precision;

/*
 * The primitive a model renders.
 *
 * MSPLAT_CHORD: K samples of the chord the ray cuts from the ellipsoid of
 *   semi-axes `scale` (see msplat_model); density zero outside it.
 * MSPLAT_CONTACT: the paper's own primitive (Sec. 3.2-3.3, Sec. 4.1): one
 *   interaction per ray and primitive, at the contact depth
 *   t* = max(0, t_c), t_c = d^T Lambda (mu - o) / d^T Lambda d (Eq. 2), with
 *   Lambda = R diag(scale)^-2 R^T.  The network reads x = [d; delta], the
 *   ray direction and the residual delta = mu - (o + t* d), each of the six
 *   components encoded as sin and cos of 2^l pi x_c for l < pe_freqs (no
 *   identity term: 12 * pe_freqs inputs, 72 for pe_freqs = 6).  `scale`
 *   holds the standard deviations of a Gaussian support: a ray interacts
 *   with the primitive when it passes within 3 of them (t_c + eta > 0 on the
 *   ellipsoid of semi-axes 3 * scale), in depth order of t_c.  The opacity
 *   is alpha = 1 - exp(-sigma G delta_i), with the Gaussian falloff
 *   G = exp(-|diag(scale)^-1 R^T delta|^2 / 2) at the contact point and the
 *   thickness delta_i = sqrt(2 pi) / |diag(scale)^-1 R^T d| (the length over
 *   which a unit Gaussian of this covariance integrates along the ray), so
 *   that sigma G delta_i is the density's line integral along the ray when
 *   t* = t_c.  The sample options (samples_*, jitter) do not apply; slot
 *   features and the float64 checker are not available for it
 *   (MSPLAT_E_UNSUPPORTED).
 */
typedef enum msplat_primitive {
  MSPLAT_CHORD = 0,
  MSPLAT_CONTACT = 1
} msplat_primitive;

/*
 * Per-primitive network (Sec. 3.2).  The input of a chord sample is its local
 * position p (the scale-normalised ellipsoid frame) encoded as
 * [p, sin(2^l pi p), cos(2^l pi p) for l < pe_freqs]: 3 + 6*pe_freqs values.
 * Hidden layers use ReLU; outputs are RGB (sigmoid), density (softplus) and
 * out_dim-4 feature channels (identity), composited like RGB.
 * Compiled shapes (pe_freqs, hidden_width, hidden_layers, out_dim):
 *   chord primitives (4, 32, 2, 4), (6, 64, 3, 4), (6, 64, 3, 20),
 *   (6, 128, 4, 20); the contact-point primitive (6, 32, 2, 4), the paper's
 *   72-32-32-4 network, in MSPLAT_FP32 and MSPLAT_BF16X3 (plain bfloat16
 *   misses the 2e-3 colour bar on its 72 inputs).  Others:
 *   MSPLAT_E_UNSUPPORTED.  For networks wider than 64 the forward keeps in LDS
 *   what fits of the weights (all of them in BF16, the hi halves of the split
 *   form), the backward reads them from global memory and runs in two passes
 *   over ranges of layers.
 */
typedef struct msplat_model {
  int32_t num_prims;     /* P >= 1 */
  int32_t pe_freqs;      /* L */
  int32_t hidden_width;
  int32_t hidden_layers;
  int32_t out_dim;       /* 4 (RGB + density) or 4 + feature channels */
  int32_t precision;     /* msplat_precision */
  int32_t primitive;     /* msplat_primitive */
} msplat_model;

/* Sampling and compositing options (Sec. 3.3). */
typedef struct msplat_opts {
  int32_t samples_fixed;    /* K samples per hit; 0 = ceil(samples_per_unit * chord)
                               clamped to [samples_min, samples_max] */
  int32_t samples_min;
  int32_t samples_max;      /* <= 128 */
  float samples_per_unit;
  float t_stop;             /* stop after the first sample with transmittance
                               below t_stop; 0 disables early termination */
  int32_t jitter;           /* 0: bin midpoints; 1: hashed stratified offsets */
  uint32_t jitter_seed;
  float background[3];      /* added as T_final * background */
  int32_t order;            /* depth order of a ray's hits (Sec. 3.3, after Eq. 2):
                               0: contact depth along the ray itself (exact);
                               1: tile order -- every ray of a packet of 64
                               consecutive rays takes the order of the contact
                               depths along one virtual ray of the packet (origin:
                               mean of the packet's origins; direction: normalised
                               sum of its directions, (0,0,1) if that sum is 0),
                               ties broken by primitive index.  Meant for rays given
                               as 8x8 pixel tiles; hit sets and sample positions are
                               those of order 0, only the compositing order changes */
  int32_t hits_per_item;    /* hits of one primitive per work item of the network
                               kernels: 16, 32 or 64; 0 = the choice msplat_autotune
                               recorded for this network and workload (64 if none) */
  int32_t items_per_group;  /* one workgroup of the network kernels (forward and
                               backward) takes the hits of this many consecutive
                               work items of one primitive (at most 64 hits per wave
                               of the kernel), deals them to its waves in one
                               balanced deal, stages the primitive's weights once and
                               (backward) keeps its weight-gradient sums in registers
                               across them: 1, 2, 4 or 8; 0 = the choice
                               msplat_autotune recorded, else the most that leave at
                               least 2048 workgroups */
  const float* tile_rays;   /* order 1 only (else MSPLAT_E_INVALID): NULL, or device
                               memory [ceil(num_rays / 64)][6] holding, per packet of
                               64 consecutive rays, the virtual ray its hits are
                               ordered along -- origin xyz, direction xyz (non-zero;
                               its length does not matter) -- such as the ray
                               through the centre of the packet's 8x8 pixel tile, as
                               the paper orders a tile (Sec. 3.3, after Eq. 2).  NULL
                               takes the mean origin and normalised direction sum
                               described above.  Read by the forward only; owned by
                               the caller */
} msplat_opts;

/* Counters filled by the forward pass (read with msplat_get_stats). */
typedef struct msplat_stats {
  int64_t num_rays;
  int64_t num_hits;           /* ray/primitive intersections */
  int64_t num_samples;        /* network evaluations scheduled */
  int64_t num_work_items;     /* primitive-grouped work items of hits_per_item hits
                                 (a workgroup takes items_per_group of them) */
  int64_t num_terminated;     /* rays that stopped early */
  int64_t num_fallbacks;      /* hit tests decided in double-float arithmetic */
  float min_abs_g;            /* smallest |1 - |p_c|^2| seen among tested pairs */
  int32_t hits_per_item;      /* work-item size the network kernels ran with */
  int32_t items_per_group;    /* work items per workgroup the forward ran with */
} msplat_stats;

typedef struct msplat_ctx msplat_ctx;

/* Create a context bound to HIP device `device` (it becomes current on the
 * calling thread while the library works).  *out receives the handle. */
int msplat_create(int device, msplat_ctx** out);
/* Destroy a context (NULL is a no-op). */
void msplat_destroy(msplat_ctx* ctx);
/* Static English text for a status code. */
const char* msplat_status_string(int status);

/* Number of float32 weights per primitive for the model (layout per layer:
 * W[out][in] row-major, then b[out]); 0 if the shape is invalid. */
int64_t msplat_num_params(const msplat_model* model);

/*
 * Workspace bytes needed for `num_rays` rays producing at most `max_hits`
 * ray/primitive hits.  The workspace holds the hit lists, per-hit partial
 * colours and everything the backward pass reads; it must stay untouched
 * between a forward call and the backward call that uses it.  Hit lists are
 * addressed with 32-bit offsets: num_rays and max_hits above 2^31 - 1 are
 * MSPLAT_E_INVALID.
 */
int msplat_workspace_size(const msplat_model* model, int64_t num_rays, int64_t max_hits,
                          uint64_t* bytes);

/*
 * Forward render (Sec. 3.2-3.3).
 *   center [P,3], scale [P,3] (semi-axes, > 0), quat [P,4] (w,x,y,z, any
 *   non-zero norm), mlp [P, num_params]; ray_o [R,3], ray_d [R,3] (unit).
 *   Rays are best given in coherent groups of 64 (e.g. 8x8 pixel tiles);
 *   any order is correct.
 * Outputs: rgb [R,3], trans [R] (final transmittance), feat [R, out_dim-4]
 *   (may be NULL when out_dim == 4).
 * The workspace `ws` (ws_bytes, 256-byte aligned) is written.  If it is too
 * small for the hits found, returns MSPLAT_E_CAPACITY with *need_bytes set and
 * outputs untouched; the caller grows the workspace and calls again.
 * need_bytes may be NULL.  A call whose rays find more than 2^31 - 1 hits in
 * total returns MSPLAT_E_INVALID (split the rays over several calls).
 */
int msplat_render_forward(msplat_ctx* ctx, const msplat_model* model, const msplat_opts* opts,
                          const float* center, const float* scale, const float* quat,
                          const float* mlp, const float* ray_o, const float* ray_d,
                          int64_t num_rays, float* rgb, float* trans, float* feat,
                          void* ws, uint64_t ws_bytes, uint64_t* need_bytes, void* stream);

/*
 * msplat_render_forward for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same render, with the workspace taken from a device array
 * the library holds, MSPLAT_NOALLOC_SCRATCH_BYTES (256 MiB) on every device
 * it runs on, until the process ends.  The call allocates nothing; the caller
 * still passes inputs and outputs.  It returns MSPLAT_E_CAPACITY (and the
 * bytes the render needs in *need_bytes, which may be NULL) when the render
 * needs more than the array holds.  Every call on a device shares that
 * device's array, and calls of it that overlap on one device race (as calls
 * that share a workspace do): serialise them.  The workspace is internal, so
 * a backward, msplat_get_stats and msplat_debug_hits need a forward into a
 * caller workspace (msplat_render_forward).
 */
#define MSPLAT_NOALLOC_SCRATCH_BYTES (256ull << 20)
int msplat_render_forward_noalloc(msplat_ctx* ctx, const msplat_model* model, const msplat_opts* opts,
                                  const float* center, const float* scale, const float* quat,
                                  const float* mlp, const float* ray_o, const float* ray_d,
                                  int64_t num_rays, float* rgb, float* trans, float* feat,
                                  uint64_t* need_bytes, void* stream);

/*
 * Backward of the forward call that last wrote `ws` with the same arguments
 * (same network shape and precision, ray count and workspace size; a call
 * that differs in any of them returns MSPLAT_E_STATE before launching work).
 * grad_rgb [R,3] = dL/drgb, grad_trans [R] = dL/dtrans (NULL = zero),
 * grad_feat [R,out_dim-4] (NULL = zero).
 * Outputs (overwritten, not accumulated): g_center [P,3], g_scale [P,3],
 * g_quat [P,4], g_mlp [P,num_params].  Hit sets, depth order, sample counts,
 * sample offsets and the termination cut are held fixed.  The recomputed
 * network activations are not stored.  Weight gradients are accumulated with
 * atomics, so their low bits may differ between runs.
 */
int msplat_render_backward(msplat_ctx* ctx, const msplat_model* model, const msplat_opts* opts,
                           const float* center, const float* scale, const float* quat,
                           const float* mlp, const float* ray_o, const float* ray_d,
                           int64_t num_rays, const float* grad_rgb, const float* grad_trans,
                           const float* grad_feat, void* ws, uint64_t ws_bytes, float* g_center,
                           float* g_scale,
                           float* g_quat, float* g_mlp, void* stream);

/*
 * Slot features (Sec. 3.4, the feature-embedding equation), rendered from the
 * hits of the forward call that last wrote `ws` (same model, same num_rays).
 *   slots [P, 4, slot_dim]: four slot embeddings e_k per primitive.
 *   out [num_rays, slot_dim] (overwritten): F = sum over the ray's hits of
 *   W * sum_k g_k e_k, where W is the hit's compositing weight (the sum of its
 *   samples' weights, T_before (1 - exp(-tau)), zero past the termination
 *   cut) and g = softmax_k(a_k . u) over the regular tetrahedral frame
 *   a_k = (1,1,1), (1,-1,-1), (-1,1,-1), (-1,-1,1) / sqrt 3 of the hit's local
 *   offset u = R^T (mu - p_c) / s at its (unclamped) contact point p_c.
 * slot_dim must be a positive multiple of 4 (at most 65536), slots and out
 * 16-byte aligned: MSPLAT_E_INVALID otherwise.  MSPLAT_E_STATE without a
 * matching forward.
 */
int msplat_slot_forward(msplat_ctx* ctx, const msplat_model* model, const float* slots, int32_t slot_dim,
                        int64_t num_rays, float* out, const void* ws, uint64_t ws_bytes, void* stream);

/*
 * msplat_render_backward for a loss that also depends on the slot features of
 * msplat_slot_forward: grad_slot [num_rays, slot_dim] = dL/dF (16-byte
 * aligned).  Returns the same gradients as msplat_render_backward, now
 * including the features' dependence on the densities (through W) and on
 * the geometry (through u), and g_slots [P, 4, slot_dim] = dL/de (overwritten;
 * accumulated with atomics, so its low bits may differ between runs).
 */
int msplat_render_backward_slots(msplat_ctx* ctx, const msplat_model* model, const msplat_opts* opts,
                                 const float* center, const float* scale, const float* quat,
                                 const float* mlp, const float* ray_o, const float* ray_d,
                                 int64_t num_rays, const float* grad_rgb, const float* grad_trans,
                                 const float* grad_feat, const float* slots, int32_t slot_dim,
                                 const float* grad_slot, void* ws, uint64_t ws_bytes, float* g_center,
                                 float* g_scale, float* g_quat, float* g_mlp, float* g_slots, void* stream);

/*
 * Per-stage timing (instrumentation; not part of the rendering method).
 * When enabled, every kernel launch of the context is bracketed by a pair of
 * HIP events recorded on the launch's own stream.  Enabling (or disabling)
 * resets the totals.  msplat_profile_read waits for the recorded events and
 * returns, per stage, a static name, the summed GPU time in milliseconds and
 * the number of timed launches; *num_stages receives the stage count, and
 * at most max_stages entries of each non-NULL array are written.
 */
int msplat_profile_enable(msplat_ctx* ctx, int enable);
int msplat_profile_read(msplat_ctx* ctx, int max_stages, const char** names, double* total_ms,
                        int64_t* launches, int* num_stages);

/*
 * Work-item autotuner (an implementation choice, not part of the method).
 * The network kernels take the hits of one primitive in work items of
 * hits_per_item hits, items_per_group of them per workgroup; the best sizes
 * depend on the network and on the workload's hit and sample counts.  This call runs the
 * forward (and, when grad_rgb is not NULL, the backward) of the given
 * arguments once per candidate size (64, 32, 16), times each on `stream`
 * with HIP events, records the fastest for this context, network and
 * workload (ray count, primitive count and sample options) and writes it to
 * *chosen.  Unless opts->items_per_group is set, it then runs the same calls
 * at that size with 1, 2, 4 and 8 work items per workgroup, records the
 * fastest beside it and writes it to *chosen_group (if not NULL).  Later
 * calls with opts->hits_per_item == 0 (and opts->items_per_group == 0) and
 * the same network and workload use them.  Arguments as for
 * msplat_render_forward and msplat_render_backward; every output buffer is
 * overwritten (with the last candidate's results) and ws is left as the
 * last forward wrote it.  Synchronises `stream`.
 */
int msplat_autotune(msplat_ctx* ctx, const msplat_model* model, const msplat_opts* opts,
                    const float* center, const float* scale, const float* quat, const float* mlp,
                    const float* ray_o, const float* ray_d, int64_t num_rays, float* rgb, float* trans,
                    float* feat, const float* grad_rgb, void* ws, uint64_t ws_bytes, float* g_center,
                    float* g_scale, float* g_quat, float* g_mlp, int32_t* chosen, int32_t* chosen_group,
                    void* stream);

/* Counters of the last forward that used `ws` (synchronises `stream`). */
int msplat_get_stats(msplat_ctx* ctx, const void* ws, uint64_t ws_bytes, msplat_stats* out,
                     void* stream);

/*
 * Depth-sorted hit lists of the last forward that used `ws`, copied to HOST
 * memory (synchronises `stream`): ray_off [R+1] (int64, prefix offsets),
 * prim [num_hits] (int32, primitive of each hit in per-ray depth order),
 * t_c [num_hits] (float64, contact depth, double-float accurate),
 * n_used [num_hits] (int32, samples composited per hit).  Capacities are
 * given in elements; MSPLAT_E_CAPACITY if num_hits exceeds them.
 */
int msplat_debug_hits(msplat_ctx* ctx, const void* ws, uint64_t ws_bytes, int64_t num_rays,
                      int64_t* ray_off, int32_t* prim, double* t_c, int32_t* n_used,
                      int64_t capacity, void* stream);

/*
 * Float64 forward of the same render (finite-difference gradient checker
 * only; not a product path).  Same arguments as msplat_render_forward with
 * float64 inputs and outputs; the workspace needs 256 bytes (*need_bytes).
 * The network is evaluated in float64 on the vector units; at most 48 hits
 * per ray are kept (MSPLAT_E_CAPACITY beyond that).  Exact order only
 * (opts->order == 1: MSPLAT_E_UNSUPPORTED).
 * decisions [R] (uint32, may be NULL) receives a hash of each ray's discrete
 * decisions: the depth-ordered primitives, the samples evaluated, every open
 * ReLU gate and the termination cut.  Two calls whose hashes agree for a ray
 * took the same decisions for it (up to hash collisions), so a central
 * difference over that ray's loss differentiates one smooth branch.
 */
int msplat_render_forward_f64(msplat_ctx* ctx, const msplat_model* model, const msplat_opts* opts,
                              const double* center, const double* scale, const double* quat,
                              const double* mlp, const double* ray_o, const double* ray_d,
                              int64_t num_rays, double* rgb, double* trans, double* feat,
                              uint32_t* decisions, void* ws, uint64_t ws_bytes, uint64_t* need_bytes,
                              void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MSPLAT_H */
