// Slot features (Sec. 3.4, the feature-embedding equation): every primitive
// carries four slot embeddings e_k in R^C; a hit's feature is
// f = sum_k g_k e_k with gates g = softmax_k(a_k . u) over a regular
// tetrahedral frame {a_k} of the hit's scale-normalised local offset
// u = R^T (mu - p*) / s, and the features are composited with the same
// volumetric weights as colour, F = sum_i T_i alpha_i f_i.
//
// A hit's samples all share its feature, so its compositing weight is the
// sum of its samples' weights, W = T_before (1 - exp(-tau_used)), from the
// records the forward pass leaves in the workspace.  The offset is taken at
// the unclamped contact point, u = -p_c; |p_c| < 1 for a hit, so the paper's
// clip to the unit cube never acts.
//
// Forward: one wave per ray, four channels per lane, up to four 256-channel
// chunks per walk over the ray's hits.  Backward: one wave per
// ray forms, per hit, q = dL/dF . f (which enters the compositing adjoint as a
// colour channel constant over the hit) and dL/dp_c through the gates; one
// wave per primitive-grouped work item accumulates dL/de_k and the contact
// points' geometry terms.
#include "common.h"

namespace msplat {
namespace {

// the tetrahedral frame, rows a_k = (+-1, +-1, +-1) / sqrt 3 with an even
// number of minus signs
__device__ __forceinline__ void slot_gates(const float u[3], float g[4]) {
  constexpr float r3 = 0.57735026918962576f;
  const float s0 = (u[0] + u[1] + u[2]) * r3;
  const float s1 = (u[0] - u[1] - u[2]) * r3;
  const float s2 = (-u[0] + u[1] - u[2]) * r3;
  const float s3 = (-u[0] - u[1] + u[2]) * r3;
  const float m = fmaxf(fmaxf(s0, s1), fmaxf(s2, s3));
  const float e0 = __expf(s0 - m), e1 = __expf(s1 - m), e2 = __expf(s2 - m), e3 = __expf(s3 - m);
  const float inv = 1.f / (e0 + e1 + e2 + e3);
  g[0] = e0 * inv;
  g[1] = e1 * inv;
  g[2] = e2 * inv;
  g[3] = e3 * inv;
}

// compositing weight of hit j: zero for hits past the termination cut
__device__ __forceinline__ float hit_weight(const Workspace& ws, int64_t j) {
  if (ws.hit_nused[j] <= 0) return 0.f;
  const float tb = __expf(-(ws.hit_sb_hi[j] + ws.hit_sb_lo[j]));
  return tb * -expm1f(-ws.hit_tau[j]);
}

__device__ __forceinline__ void local_offset(const Workspace& ws, int64_t j, float u[3]) {
  const int64_t H = ws.hit_cap;
#pragma unroll
  for (int a = 0; a < 3; ++a) u[a] = -ws.hit_pc[a * H + j];
}

constexpr int kSlotChunk = 4 * kWave;   // channels a wave covers per pass (4 per lane)
typedef float f4v __attribute__((ext_vector_type(4)));

// NCH chunks of 256 channels per walk over the ray's hits (one walk for
// C <= 256 NCH): the hit records are read once per walk and the chunks' loads
// are independent
template <int NCH>
__global__ __launch_bounds__(256) void slot_forward_kernel(Workspace ws, int64_t R, const float* __restrict__ slots,
                                                           int C, float* __restrict__ out) {
  const int64_t ray = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (ray >= R) return;   // (whole wave)
  const int lane = lane_id();
  const int64_t a = ws.ray_off[ray], b = ws.ray_off[ray + 1];
  for (int cb = 0; cb < C; cb += NCH * kSlotChunk) {
    float4 acc[NCH];
#pragma unroll
    for (int q = 0; q < NCH; ++q) acc[q] = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int64_t j = a; j < b; ++j) {
      const float W = hit_weight(ws, j);
      if (W == 0.f) continue;   // (wave-uniform: every lane reads the same hit)
      float u[3], g[4];
      local_offset(ws, j, u);
      slot_gates(u, g);
      const int p = ws.hit_prim[j];
      const float* sp = slots + (int64_t)p * 4 * C;
#pragma unroll
      for (int q = 0; q < NCH; ++q) {
        const int c = cb + q * kSlotChunk + 4 * lane;
        if (c >= C) continue;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float4 e = *reinterpret_cast<const float4*>(sp + k * C + c);
          const float wk = W * g[k];
          acc[q].x = __builtin_fmaf(wk, e.x, acc[q].x);
          acc[q].y = __builtin_fmaf(wk, e.y, acc[q].y);
          acc[q].z = __builtin_fmaf(wk, e.z, acc[q].z);
          acc[q].w = __builtin_fmaf(wk, e.w, acc[q].w);
        }
      }
    }
    // F is written once and not read again here: streaming stores
#pragma unroll
    for (int q = 0; q < NCH; ++q) {
      const int c = cb + q * kSlotChunk + 4 * lane;
      if (c < C) {
        const f4v v = {acc[q].x, acc[q].y, acc[q].z, acc[q].w};
        __builtin_nontemporal_store(v, reinterpret_cast<f4v*>(out + ray * C + c));
      }
    }
  }
}

// per hit: q = dL/dF . f and dL/dp_c = -dL/du with
// dL/du = sum_k W g_k (h_k - q) a_k, h_k = dL/dF . e_k
// (NCH > 0: the ray's dL/dF row, C <= 256 NCH, is held in registers for all
// its hits; NCH = 0: it is streamed per hit)
template <int NCH>
__global__ __launch_bounds__(256) void slot_backward_hits_kernel(Workspace ws, int64_t R,
                                                                 const float* __restrict__ slots, int C,
                                                                 const float* __restrict__ grad_slot) {
  const int64_t ray = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (ray >= R) return;   // (whole wave)
  const int lane = lane_id();
  const int64_t H = ws.hit_cap;
  const int64_t a = ws.ray_off[ray], b = ws.ray_off[ray + 1];
  float4 gfr[NCH > 0 ? NCH : 1];
  if constexpr (NCH > 0) {
    if (b > a) {
#pragma unroll
      for (int q = 0; q < NCH; ++q) {
        const int c = q * kSlotChunk + 4 * lane;
        gfr[q] = c < C ? *reinterpret_cast<const float4*>(grad_slot + ray * C + c) : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
  }
  for (int64_t j = a; j < b; ++j) {
    const float W = hit_weight(ws, j);
    if (W == 0.f) {   // (wave-uniform)
      if (lane == 0) {
        ws.hit_q[j] = 0.f;
        for (int d = 0; d < 3; ++d) ws.hit_gpc[d * H + j] = 0.f;
      }
      continue;
    }
    const int p = ws.hit_prim[j];
    float h[4] = {0.f, 0.f, 0.f, 0.f};
    if constexpr (NCH > 0) {
#pragma unroll
      for (int q = 0; q < NCH; ++q) {
        const int c = q * kSlotChunk + 4 * lane;
        if (c >= C) continue;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float4 e = *reinterpret_cast<const float4*>(slots + ((int64_t)p * 4 + k) * C + c);
          h[k] += gfr[q].x * e.x + gfr[q].y * e.y + gfr[q].z * e.z + gfr[q].w * e.w;
        }
      }
    } else {
#pragma unroll 4
      for (int c = 4 * lane; c < C; c += kSlotChunk) {
        const float4 gf = *reinterpret_cast<const float4*>(grad_slot + ray * C + c);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float4 e = *reinterpret_cast<const float4*>(slots + ((int64_t)p * 4 + k) * C + c);
          h[k] += gf.x * e.x + gf.y * e.y + gf.z * e.z + gf.w * e.w;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) h[k] = wave_sum(h[k]);
    if (lane == 0) {
      float u[3], g[4];
      local_offset(ws, j, u);
      slot_gates(u, g);
      const float q = g[0] * h[0] + g[1] * h[1] + g[2] * h[2] + g[3] * h[3];
      float ds[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) ds[k] = W * g[k] * (h[k] - q);
      constexpr float r3 = 0.57735026918962576f;
      const float du0 = (ds[0] + ds[1] - ds[2] - ds[3]) * r3;
      const float du1 = (ds[0] - ds[1] + ds[2] - ds[3]) * r3;
      const float du2 = (ds[0] - ds[1] - ds[2] + ds[3]) * r3;
      ws.hit_q[j] = q;
      ws.hit_gpc[0 * H + j] = -du0;
      ws.hit_gpc[1 * H + j] = -du1;
      ws.hit_gpc[2 * H + j] = -du2;
    }
  }
}

// Geometry terms of dL/dp_c at the contact point, in the accumulator form of
// the per-hit geometry kernel ([dL/dM as c1 (x) delta_c + c2 (x) d, c1]).
// p_c = (I - e e^T / |e|^2) M (o - mu) with e = M d: the point moves with the
// frame and, through t_c, along e; with g = dL/dp_c,
// c1 = (g.e) e / |e|^2 - g and c2 = -(g.e) p_c / |e|^2.
__device__ __forceinline__ void contact_geometry_terms(const Workspace& ws, const float* __restrict__ ray_d,
                                                       int hit, int p, float (&acc)[12]) {
  const int64_t H = ws.hit_cap;
  const float* gp = ws.geo + (int64_t)p * kGeoStride;
  float g[3], pc[3], ee[3];
  for (int a = 0; a < 3; ++a) {
    g[a] = ws.hit_gpc[a * H + hit];
    pc[a] = ws.hit_pc[a * H + hit];
    ee[a] = ws.hit_e[a * H + hit];
  }
  const int ray = ws.hit_ray[hit];
  const float dd[3] = {ray_d[3 * ray], ray_d[3 * ray + 1], ray_d[3 * ray + 2]};
  const float a2 = ee[0] * ee[0] + ee[1] * ee[1] + ee[2] * ee[2];
  const float x = (g[0] * ee[0] + g[1] * ee[1] + g[2] * ee[2]) / a2;
  // delta_c = mu - o - t_c d = -R diag(s) p_c
  float dc[3];
  for (int r = 0; r < 3; ++r) {
    dc[r] = 0.f;
    for (int c = 0; c < 3; ++c) dc[r] -= gp[G_R + 3 * r + c] * gp[G_S + c] * pc[c];
  }
  for (int r = 0; r < 3; ++r) {
    const float c1 = x * ee[r] - g[r];
    const float c2 = -x * pc[r];
    for (int c = 0; c < 3; ++c) acc[3 * r + c] = c1 * dc[c] + c2 * dd[c];
    acc[9 + r] = c1;
  }
}

// consecutive work items per wave of the embedding gradient: up to 16, fewer
// while that would leave fewer than kSlotWaves waves to fill the chip
constexpr int kSlotItemsMax = 16;
constexpr int kSlotWaves = 4096;

// add a wave's accumulated dL/de of one primitive to g_slots
template <int NCH>
__device__ __forceinline__ void flush_slots(float* __restrict__ g_slots, int p, int C, int cb, int lane,
                                            const float4 (&acc)[NCH][4]) {
#pragma unroll
  for (int q = 0; q < NCH; ++q) {
    const int c = cb + q * kSlotChunk + 4 * lane;
    if (c >= C) continue;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      float* dst = g_slots + ((int64_t)p * 4 + k) * C + c;
      atomicAdd(dst + 0, acc[q][k].x);
      atomicAdd(dst + 1, acc[q][k].y);
      atomicAdd(dst + 2, acc[q][k].z);
      atomicAdd(dst + 3, acc[q][k].w);
    }
  }
}

// One wave per run of `per_run` consecutive primitive-grouped work items
// (each up to kHitsPerItem hits of one primitive, listed in phit):
// dL/de_k += W g_k dL/dF over the hits, kept in registers until the run
// moves to another primitive (one set of atomics per primitive and run, not
// per item), and the contact points' geometry terms join the primitive's
// accumulators.
template <int NCH>
__global__ __launch_bounds__(256) void slot_backward_prims_kernel(Workspace ws, int P, int items,
                                                                  const float* __restrict__ slots, int C,
                                                                  const float* __restrict__ grad_slot,
                                                                  const float* __restrict__ ray_d,
                                                                  float* __restrict__ g_slots, int per_run) {
  const int run = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int it0 = run * per_run;
  if (it0 >= items) return;   // (whole wave)
  const int it1 = min(items, it0 + per_run);
  const int lane = lane_id();
  // the first item's primitive: the last p with wi_off[p] <= it0
  int lo = 0, hi = P;   // wi_off[lo] <= it0 < wi_off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (ws.wi_off[mid] <= it0) lo = mid;
    else hi = mid;
  }
  for (int cb = 0; cb < C; cb += NCH * kSlotChunk) {
    float4 acc[NCH][4];
#pragma unroll
    for (int q = 0; q < NCH; ++q)
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[q][k] = make_float4(0.f, 0.f, 0.f, 0.f);
    int p = lo;
    for (int item = it0; item < it1; ++item) {
      if (ws.wi_off[p + 1] <= item) {
        // the run moves to the next primitive with work items
        flush_slots<NCH>(g_slots, p, C, cb, lane, acc);
#pragma unroll
        for (int q = 0; q < NCH; ++q)
#pragma unroll
          for (int k = 0; k < 4; ++k) acc[q][k] = make_float4(0.f, 0.f, 0.f, 0.f);
        while (ws.wi_off[p + 1] <= item) ++p;
      }
      const int first = ws.prim_off[p] + (item - ws.wi_off[p]) * ws.hits_per_item;
      const int nh = min(ws.hits_per_item, ws.prim_off[p + 1] - first);
      // this lane's hit: weight, gates, ray (and, once, its contact point's
      // geometry terms)
      float W = 0.f, g[4] = {0.f, 0.f, 0.f, 0.f};
      int ray = 0;
      float geo[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) geo[k] = 0.f;
      if (lane < nh) {
        const int hit = ws.phit[first + lane];
        W = hit_weight(ws, hit);
        float u[3];
        local_offset(ws, hit, u);
        slot_gates(u, g);
        ray = ws.hit_ray[hit];
        if (cb == 0 && W != 0.f) contact_geometry_terms(ws, ray_d, hit, p, geo);
      }
      if (cb == 0) {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          const float v = wave_sum(geo[k]);
          if (lane == 0 && v != 0.f) atomicAdd(ws.geo_grad + (int64_t)p * 12 + k, v);
        }
      }
      // four hits at a time: their dL/dF rows are requested before any is
      // used (a hit past the cut has W = 0 and adds nothing)
      constexpr int G = 4;
      for (int i0 = 0; i0 < nh; i0 += G) {
        float gi[G][4];
        float4 gf[G][NCH];
#pragma unroll
        for (int t = 0; t < G; ++t) {
          const int i = min(i0 + t, kWave - 1);
          const bool ok = i0 + t < nh;   // (wave-uniform)
          const float Wi = ok ? __shfl(W, i, kWave) : 0.f;
          const int ri = __shfl(ray, i, kWave);
#pragma unroll
          for (int k = 0; k < 4; ++k) gi[t][k] = __shfl(g[k], i, kWave) * Wi;
          const float* gr = grad_slot + (int64_t)ri * C;
#pragma unroll
          for (int q = 0; q < NCH; ++q) {
            const int c = cb + q * kSlotChunk + 4 * lane;
            gf[t][q] = (ok && Wi != 0.f && c < C) ? *reinterpret_cast<const float4*>(gr + c)
                                                  : make_float4(0.f, 0.f, 0.f, 0.f);
          }
        }
#pragma unroll
        for (int t = 0; t < G; ++t)
#pragma unroll
          for (int q = 0; q < NCH; ++q)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              acc[q][k].x = __builtin_fmaf(gi[t][k], gf[t][q].x, acc[q][k].x);
              acc[q][k].y = __builtin_fmaf(gi[t][k], gf[t][q].y, acc[q][k].y);
              acc[q][k].z = __builtin_fmaf(gi[t][k], gf[t][q].z, acc[q][k].z);
              acc[q][k].w = __builtin_fmaf(gi[t][k], gf[t][q].w, acc[q][k].w);
            }
      }
    }
    flush_slots<NCH>(g_slots, p, C, cb, lane, acc);
  }
}

}  // namespace

hipError_t launch_slot_forward(const Workspace& ws, int64_t R, const float* slots, int C, float* out,
                               hipStream_t s) {
  if (R <= 0 || C <= 0) return hipSuccess;
  const dim3 grid((unsigned)((R + 3) / 4));
  if (C <= kSlotChunk) hipLaunchKernelGGL(slot_forward_kernel<1>, grid, dim3(256), 0, s, ws, R, slots, C, out);
  else if (C <= 2 * kSlotChunk) hipLaunchKernelGGL(slot_forward_kernel<2>, grid, dim3(256), 0, s, ws, R, slots, C, out);
  else hipLaunchKernelGGL(slot_forward_kernel<4>, grid, dim3(256), 0, s, ws, R, slots, C, out);
  return hipGetLastError();
}

hipError_t launch_slot_backward_hits(const Workspace& ws, int64_t R, const float* slots, int C,
                                     const float* grad_slot, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  const dim3 grid((unsigned)((R + 3) / 4));
  if (C <= kSlotChunk)
    hipLaunchKernelGGL(slot_backward_hits_kernel<1>, grid, dim3(256), 0, s, ws, R, slots, C, grad_slot);
  else if (C <= 2 * kSlotChunk)
    hipLaunchKernelGGL(slot_backward_hits_kernel<2>, grid, dim3(256), 0, s, ws, R, slots, C, grad_slot);
  else if (C <= 4 * kSlotChunk)
    hipLaunchKernelGGL(slot_backward_hits_kernel<4>, grid, dim3(256), 0, s, ws, R, slots, C, grad_slot);
  else
    hipLaunchKernelGGL(slot_backward_hits_kernel<0>, grid, dim3(256), 0, s, ws, R, slots, C, grad_slot);
  return hipGetLastError();
}

hipError_t launch_slot_backward_prims(const Workspace& ws, int P, int items, const float* slots, int C,
                                      const float* grad_slot, const float* ray_d, float* g_slots,
                                      hipStream_t s) {
  if (items <= 0) return hipSuccess;
  const int per_run = max(1, min(kSlotItemsMax, items / kSlotWaves));
  const int runs = (items + per_run - 1) / per_run;
  const dim3 grid((unsigned)((runs + 3) / 4));
  if (C <= kSlotChunk)
    hipLaunchKernelGGL(slot_backward_prims_kernel<1>, grid, dim3(256), 0, s, ws, P, items, slots, C, grad_slot,
                       ray_d, g_slots, per_run);
  else if (C <= 2 * kSlotChunk)
    hipLaunchKernelGGL(slot_backward_prims_kernel<2>, grid, dim3(256), 0, s, ws, P, items, slots, C, grad_slot,
                       ray_d, g_slots, per_run);
  else
    hipLaunchKernelGGL(slot_backward_prims_kernel<4>, grid, dim3(256), 0, s, ws, P, items, slots, C, grad_slot,
                       ray_d, g_slots, per_run);
  return hipGetLastError();
}

}  // namespace msplat
