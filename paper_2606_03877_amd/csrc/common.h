// Internal definitions shared by the msplat HIP sources: workspace layout,
// small device helpers (double-float arithmetic, the PCG hash, wave scans).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/msplat.h"

namespace msplat {

constexpr int kWave = 64;
constexpr int kGeoStride = 40;       // floats per preprocessed primitive record
constexpr int kHitsPerItem = 64;     // most hits per primitive-grouped work item (one per lane)
constexpr int kMaxSamplesPerHit = 128;
constexpr int kClippedBit = 0x10000;   // flag in hit_k: interval clamped at t = 0
constexpr int kKMask = 0xFFFF;

// ---- preprocessed primitive record (float offsets inside kGeoStride) ----
enum GeoField {
  G_MU = 0,       // centre (3)
  G_M_HI = 3,     // M = diag(s)^-1 R^T, row-major, high part (9)
  G_M_LO = 12,    // low part of M as a double-float (9)
  G_QN = 21,      // normalised quaternion (4)
  G_S = 25,       // scale (3)
  G_INVQ = 28,    // 1/|q|
  G_RAD = 29,     // bounding-sphere radius (max semi-axis, slightly inflated)
  G_R = 30,       // rotation matrix R, row-major (9)
};

// ---- device counters at the start of the workspace ----
struct DevCounters {
  int64_t num_hits;
  int64_t num_samples;
  int32_t num_work_items;
  int32_t num_terminated;
  int32_t num_fallbacks;
  uint32_t min_abs_g_bits;   // float bits of min |g| (non-negative floats order as ints)
  int32_t overflow;          // set if the hit list outgrew the capacity
  uint32_t magic;            // kCountersMagic once a forward pass has filled the workspace
  // what the workspace was laid out for (checked by the calls that read it)
  int64_t num_rays;
  int64_t hit_cap;
  int32_t num_prims;
  int32_t num_params;
  int64_t hit_total;         // hits counted in 64 bits (offsets and scans are 32-bit)
  int32_t net[6];            // network the workspace was laid out for: L, W, D, NOUT, precision, kind
  int32_t hits_per_item;     // hits per work item of the network kernels
  int32_t pad;
};
static_assert(sizeof(DevCounters) == 104, "counter block size");
constexpr uint32_t kCountersMagic = 0x4d53504cu;

// Workspace layout: every section 256-byte aligned, sized from (model, R, H).
struct Workspace {
  DevCounters* counters;
  float* geo;            // [P, kGeoStride]
  uint8_t* wpack;        // packed network operands, wpack_bytes per primitive
  int32_t* prim_nhit;    // [P]
  int32_t* prim_off;     // [P+1]
  int32_t* prim_cursor;  // [P]
  int32_t* wi_off;       // [P+1] work-item offsets
  int32_t* gw_off;       // [P+1] backward: offsets of each primitive's workgroups
  float* geo_grad;       // [P, 12] accumulated dL/dM (9) and M^T-free dL/dv (3)
  int32_t* ray_off;      // [R+1] (counts, then exclusive offsets)
  int32_t* scan_tmp;     // scan block sums
  float* ray_tf;         // [R] final transmittance (kept for the backward)
  // per hit
  int32_t* hit_prim;
  int32_t* hit_ray;
  int32_t* hit_k;        // samples of the hit (bits 0-15), kClippedBit if the chord starts at t = 0
  int32_t* hit_nused;    // samples composited (after early termination)
  float* hit_tc_hi;
  float* hit_tc_lo;
  float* hit_eta;
  // sample geometry of a hit as double-float pairs (hi in the first array,
  // lo in the second): sample k sits at p_c + s_k e with s_k = s_a + (k+u) Delta
  float* hit_sa;         // t_a - t_c
  float* hit_sa_lo;
  float* hit_dlt;        // bin width Delta = (t_b - t_a) / K
  float* hit_dlt_lo;
  float* hit_pc;         // [3][H] contact point in the local frame (SoA)
  float* hit_pc_lo;      // [3][H]
  float* hit_e;          // [3][H] M d (SoA)
  float* hit_e_lo;       // [3][H]
  float* hit_tau;        // optical depth of the whole hit (or of its used part)
  float* hit_cloc;       // [NC][H] hit-local colour (and feature) sums
  float* hit_sb_hi;      // optical depth before the hit (double-float)
  float* hit_sb_lo;
  float* hit_gsa;        // backward: g . (colour composited after the hit)
  float* hit_tb;         // backward: transmittance before the hit
  float* hit_gtot;       // backward: g . (the hit's own composited colour)
  float* hit_gv;         // [9][H] backward: the hit's sums of the sample-position
                         // adjoints (dL/dp, s dL/dp, dL/ds_k, omega_k dL/ds_k, dL/dDelta
                         // terms), indexed by the hit's entry in phit
  int32_t* phit;         // [H] hits grouped by primitive
  float* hit_q;          // [H] slot features, backward: dL/dF . (the hit's feature)
  float* hit_gpc;        // [3][H] slot features, backward: dL/d(local contact point)
  int32_t slot_on;       // 1 while a backward carries slot-feature gradients
  int32_t hits_per_item; // hits per work item (16, 32 or 64)
  int64_t num_rays;
  int64_t hit_cap;
  int64_t wpack_bytes;
  int32_t nc;            // 3 + feature channels
};

// ---------------------------------------------------------------------------
// double-float ("df") arithmetic on (hi, lo) float pairs: TwoSum (Knuth),
// FastTwoSum (Dekker 1971), TwoProd via fused multiply-add.  These
// error-free transformations need every product and sum rounded as written:
// contraction of a product into a following sum (which hipcc allows by
// default) silently degrades them to single-float accuracy, so each body
// switches it off.
#define MSPLAT_EXACT_FP _Pragma("clang fp contract(off)")
// ---------------------------------------------------------------------------
struct df { float hi, lo; };

__device__ __forceinline__ df two_sum(float a, float b) {
  MSPLAT_EXACT_FP
  float s = a + b;
  float bb = s - a;
  float err = (a - (s - bb)) + (b - bb);
  return {s, err};
}
__device__ __forceinline__ df fast_two_sum(float a, float b) {
  MSPLAT_EXACT_FP
  float s = a + b;
  return {s, b - (s - a)};
}
__device__ __forceinline__ df two_prod(float a, float b) {
  MSPLAT_EXACT_FP
  float p = a * b;
  return {p, __builtin_fmaf(a, b, -p)};
}
__device__ __forceinline__ df df_from(float a) { return {a, 0.f}; }
__device__ __forceinline__ df df_add(df x, df y) {
  MSPLAT_EXACT_FP
  df s = two_sum(x.hi, y.hi);
  df t = two_sum(x.lo, y.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ df df_neg(df x) { return {-x.hi, -x.lo}; }
__device__ __forceinline__ df df_sub(df x, df y) { return df_add(x, df_neg(y)); }
__device__ __forceinline__ df df_mul(df x, df y) {
  MSPLAT_EXACT_FP
  df p = two_prod(x.hi, y.hi);
  p.lo = __builtin_fmaf(x.hi, y.lo, __builtin_fmaf(x.lo, y.hi, p.lo));
  return fast_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ df df_mulf(df x, float y) {
  MSPLAT_EXACT_FP
  df p = two_prod(x.hi, y);
  p.lo = __builtin_fmaf(x.lo, y, p.lo);
  return fast_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ df df_div(df x, df y) {
  MSPLAT_EXACT_FP
  float q1 = x.hi / y.hi;
  df r = df_sub(x, df_mulf(y, q1));
  float q2 = r.hi / y.hi;
  r = df_sub(r, df_mulf(y, q2));
  float q3 = r.hi / y.hi;
  df q = fast_two_sum(q1, q2);
  return df_add(q, df_from(q3));
}
__device__ __forceinline__ df df_sqrt(df x) {
  MSPLAT_EXACT_FP
  if (x.hi <= 0.f) return {0.f, 0.f};
  float s = sqrtf(x.hi);
  df r = df_sub(x, two_prod(s, s));
  float c = r.hi / (2.f * s);
  return fast_two_sum(s, c);
}
__device__ __forceinline__ int df_sign(df x) {
  return x.hi > 0.f ? 1 : (x.hi < 0.f ? -1 : (x.lo > 0.f ? 1 : (x.lo < 0.f ? -1 : 0)));
}

// ---------------------------------------------------------------------------
// PCG output permutation used as a stateless 32-bit hash (Jarzynski and
// Olano, "Hash Functions for GPU Rendering", JCGT 2020), and the stratified
// sample offset u in [0,1) derived from (seed, ray, rank, k).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t pcg_hash(uint32_t v) {
  uint32_t state = v * 747796405u + 2891336453u;
  uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
  return (word >> 22u) ^ word;
}
__device__ __forceinline__ float sample_offset(uint32_t seed_hash, uint32_t ray, uint32_t rank,
                                               uint32_t k) {
  uint32_t h = pcg_hash(pcg_hash(pcg_hash(seed_hash + ray) + rank) + k);
  return (float)(h >> 8) * 5.9604644775390625e-8f;   // 2^-24
}

// ---------------------------------------------------------------------------
// wave helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}
// inclusive prefix sum over the 64 lanes
__device__ __forceinline__ int wave_incl_scan(int v) {
  int l = lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int t = __shfl_up(v, off, 64);
    if (l >= off) v += t;
  }
  return v;
}

// ---------------------------------------------------------------------------
// host-side launch wrappers implemented in the .hip files
// ---------------------------------------------------------------------------
struct NetShape {
  int P, L, W, D, NOUT, prec, n_params;
  int kind;   // msplat_primitive
};
// support of the contact-point primitive: the ellipsoid of KAPPA standard
// deviations (the extent 3DGS-style Gaussian splatting culls at)
constexpr float kContactKappa = 3.f;
// hits of one call: offsets and scans are 32-bit
constexpr int64_t kMaxHits = 0x7fffffffLL;
// outputs of a network: RGB, density and up to 16 feature channels
constexpr int kMaxOut = 20;

// geometry.hip
hipError_t launch_preprocess(const Workspace& ws, const float* center, const float* scale,
                             const float* quat, int P, int kind, hipStream_t s);
hipError_t launch_bin_count(const Workspace& ws, const float* ray_o, const float* ray_d,
                            const float* center, const float* scale, const float* quat, int64_t R,
                            int P, const msplat_opts& o, int kind, hipStream_t s);
hipError_t launch_scans(const Workspace& ws, int64_t R, const NetShape& n, hipStream_t s);
hipError_t launch_bin_fill(const Workspace& ws, const float* ray_o, const float* ray_d,
                           const float* center, const float* scale, const float* quat,
                           int64_t R, int P, const msplat_opts& o, int kind, hipStream_t s);
hipError_t launch_hit_records(const Workspace& ws, const float* ray_o, const float* ray_d, int64_t num_hits,
                              int kind, hipStream_t s);
// offsets of each primitive's runs of ghits hits (the workgroups of the
// network kernels) into ws.gw_off
hipError_t launch_group_scan(const Workspace& ws, int P, int ghits, hipStream_t s);
hipError_t launch_composite(const Workspace& ws, int64_t R, const msplat_opts& o, float* rgb,
                            float* trans, float* feat, int cf, hipStream_t s);
hipError_t launch_composite_adjoint(const Workspace& ws, int64_t R, const msplat_opts& o,
                                    const float* grad_rgb, const float* grad_trans,
                                    const float* grad_feat, int cf, const float* trans,
                                    hipStream_t s);
hipError_t launch_hit_geometry(const Workspace& ws, const float* ray_d, int64_t num_hits, int kind,
                               hipStream_t s);
hipError_t launch_geo_finalize(const Workspace& ws, int P, float* g_center, float* g_scale,
                               float* g_quat, int kind, hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
// every 32-bit word of [p, p + bytes) set to value (a kernel: no memset node in a captured graph)
hipError_t launch_fill(void* p, size_t bytes, uint32_t value, hipStream_t s);
// slot features (slots.hip)
hipError_t launch_slot_forward(const Workspace& ws, int64_t R, const float* slots, int C, float* out,
                               hipStream_t s);
hipError_t launch_slot_backward_hits(const Workspace& ws, int64_t R, const float* slots, int C,
                                     const float* grad_slot, hipStream_t s);
hipError_t launch_slot_backward_prims(const Workspace& ws, int P, int items, const float* slots, int C,
                                      const float* grad_slot, const float* ray_d, float* g_slots,
                                      hipStream_t s);

// mlp.hip
bool mlp_supported(const NetShape& n);
int64_t mlp_wpack_bytes(const NetShape& n);
hipError_t launch_pack_weights(const NetShape& n, const Workspace& ws, const float* mlp,
                               hipStream_t s);
// (group >= 1: a workgroup takes the hits of that many work items of one
// primitive, at most 64 per wave of the kernel)
hipError_t launch_mlp_forward(const NetShape& n, const Workspace& ws, const msplat_opts& o,
                              int64_t num_hits, int group, int mode, float* rgb, float* trans, float* feat,
                              hipStream_t s);
// mlp_bwd.hip
// (group >= 1: a workgroup takes the hits of that many work items of one
// primitive, at most 64 per wave of the kernel)
hipError_t launch_mlp_backward(const NetShape& n, const Workspace& ws, const msplat_opts& o,
                               int64_t num_hits, int group, const float* ray_d, const float* grad_rgb,
                               const float* grad_feat, float* g_mlp, hipStream_t s);

// f64.hip
hipError_t launch_forward_f64(const NetShape& n, const msplat_opts& o, const double* center,
                              const double* scale, const double* quat, const double* mlp,
                              const double* ray_o, const double* ray_d, int64_t R,
                              double* rgb, double* trans, double* feat, uint32_t* decisions,
                              void* ws, uint64_t ws_bytes, int max_hits_per_ray, hipStream_t s);

}  // namespace msplat
