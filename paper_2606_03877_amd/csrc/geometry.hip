// Ray/support geometry, binning, depth sort, per-ray compositing and their
// adjoints for the MLP-Splatting render path on gfx950.
//
// Hit test (Sec. 3.2, Eq. 1-2): with M = diag(s)^-1 R(q)^T, v = mu - o and
// e = M d, the contact depth t_c = (e . M v) / (e . e) is the unclamped
// minimiser of the Lambda-distance of Eq. 1; p_c = -M (v - t_c d) is the local
// contact point, g = 1 - |p_c|^2 and eta = sqrt(g / |e|^2) the half chord.  A
// pair is a hit iff g > 0 and t_c + eta > 0; the chord starts at
// max(t_c - eta, 0) (the clamp of Eq. 2).
//
// Every discrete decision (hit, front, clipped start, sample count, depth
// order) is taken in float32 when its margin is large and recomputed in
// double-float arithmetic otherwise, so the hit lists equal those of exact
// arithmetic except for margins below ~1e-12.
#include "common.h"

namespace msplat {

namespace {

constexpr float kEpsG = 1e-4f;       // |g| below this: decide in double-float
constexpr float kEpsT = 1e-5f;       // relative margin of the front / clip tests
constexpr float kEpsK = 1e-3f;       // distance of K*L to an integer
constexpr float kEpsKey = 1e-6f;     // relative depth gap below which keys are recomputed

__device__ __forceinline__ float3 ld3(const float* p, int64_t i) {
  return make_float3(p[3 * i], p[3 * i + 1], p[3 * i + 2]);
}

// ----------------------------------------------------------- preprocessing --

// kappa: the support's semi-axes in units of the scale (1 for chord
// primitives, whose scale is the semi-axes; kContactKappa for the
// contact-point primitive, whose scale is the Gaussian's standard deviations)
__global__ void preprocess_kernel(const float* __restrict__ center, const float* __restrict__ scale,
                                  const float* __restrict__ quat, float* __restrict__ geo, int P, float kappa) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  float* g = geo + (int64_t)i * kGeoStride;
  float q[4] = {quat[4 * i], quat[4 * i + 1], quat[4 * i + 2], quat[4 * i + 3]};
  float s[3] = {scale[3 * i], scale[3 * i + 1], scale[3 * i + 2]};
  // normalised quaternion and rotation, double-float
  df n2 = two_prod(q[0], q[0]);
  for (int k = 1; k < 4; ++k) n2 = df_add(n2, two_prod(q[k], q[k]));
  df nrm = df_sqrt(n2);
  df qn[4];
  for (int k = 0; k < 4; ++k) qn[k] = df_div(df_from(q[k]), nrm);
  const df& w = qn[0];
  const df& x = qn[1];
  const df& y = qn[2];
  const df& z = qn[3];
  df one = df_from(1.f), two = df_from(2.f);
  df r[9];
  r[0] = df_sub(one, df_mul(two, df_add(df_mul(y, y), df_mul(z, z))));
  r[1] = df_mul(two, df_sub(df_mul(x, y), df_mul(w, z)));
  r[2] = df_mul(two, df_add(df_mul(x, z), df_mul(w, y)));
  r[3] = df_mul(two, df_add(df_mul(x, y), df_mul(w, z)));
  r[4] = df_sub(one, df_mul(two, df_add(df_mul(x, x), df_mul(z, z))));
  r[5] = df_mul(two, df_sub(df_mul(y, z), df_mul(w, x)));
  r[6] = df_mul(two, df_sub(df_mul(x, z), df_mul(w, y)));
  r[7] = df_mul(two, df_add(df_mul(y, z), df_mul(w, x)));
  r[8] = df_sub(one, df_mul(two, df_add(df_mul(x, x), df_mul(y, y))));
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      df m = df_div(r[3 * b + a], two_prod(kappa, s[a]));   // M[a][b] = R[b][a] / (kappa s[a])
      g[G_M_HI + 3 * a + b] = m.hi;
      g[G_M_LO + 3 * a + b] = m.lo;
    }
  for (int k = 0; k < 9; ++k) g[G_R + k] = r[k].hi;
  for (int k = 0; k < 3; ++k) g[G_MU + k] = center[3 * i + k];
  for (int k = 0; k < 4; ++k) g[G_QN + k] = qn[k].hi;
  for (int k = 0; k < 3; ++k) g[G_S + k] = kappa * s[k];
  g[G_INVQ] = 1.f / nrm.hi;
  float rad = kappa * fmaxf(fmaxf(s[0], s[1]), s[2]);
  g[G_RAD] = rad * (1.f + 1e-4f) + 1e-6f;
}

// ------------------------------------------------------------ hit testing --

struct HitF {
  bool hit, uncertain;
  bool clipped;
  float tc_hi, tc_lo, eta, g, a;
};

// float32 test with one refinement step of the contact depth.
__device__ __forceinline__ HitF hit_test_f32(const float* __restrict__ g, float3 o, float3 d,
                                             const msplat_opts& opt, int* k_out) {
  HitF h;
  const float* M = g + G_M_HI;
  float v[3], vlo[3];
  {
    df t0 = two_sum(g[G_MU + 0], -o.x);
    df t1 = two_sum(g[G_MU + 1], -o.y);
    df t2 = two_sum(g[G_MU + 2], -o.z);
    v[0] = t0.hi; v[1] = t1.hi; v[2] = t2.hi;
    vlo[0] = t0.lo; vlo[1] = t1.lo; vlo[2] = t2.lo;
  }
  float dd[3] = {d.x, d.y, d.z};
  float m[3], e[3];
  for (int r = 0; r < 3; ++r) {
    m[r] = M[3 * r] * v[0] + M[3 * r + 1] * v[1] + M[3 * r + 2] * v[2];
    e[r] = M[3 * r] * dd[0] + M[3 * r + 1] * dd[1] + M[3 * r + 2] * dd[2];
  }
  float a = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
  float t0 = (e[0] * m[0] + e[1] * m[1] + e[2] * m[2]) / a;
  float dl0[3];
  for (int k = 0; k < 3; ++k) dl0[k] = __builtin_fmaf(-t0, dd[k], v[k]) + vlo[k];
  float md[3];
  for (int r = 0; r < 3; ++r) md[r] = M[3 * r] * dl0[0] + M[3 * r + 1] * dl0[1] + M[3 * r + 2] * dl0[2];
  float dt = (e[0] * md[0] + e[1] * md[1] + e[2] * md[2]) / a;
  float pc[3];
  for (int r = 0; r < 3; ++r) pc[r] = dt * e[r] - md[r];   // -M (dl0 - dt d)
  float gg = __builtin_fmaf(-pc[0], pc[0], __builtin_fmaf(-pc[1], pc[1], __builtin_fmaf(-pc[2], pc[2], 1.f)));
  df tc = fast_two_sum(t0, dt);
  h.tc_hi = tc.hi;
  h.tc_lo = tc.lo;
  h.g = gg;
  h.a = a;
  float eta = sqrtf(fmaxf(gg, 0.f) / a);
  h.eta = eta;
  float front = tc.hi + eta;
  float back = tc.hi - eta;
  float tscale = kEpsT * (1.f + fabsf(tc.hi));
  h.hit = gg > 0.f && front > 0.f;
  h.clipped = back <= 0.f;
  h.uncertain = fabsf(gg) < kEpsG || (gg > 0.f && (fabsf(front) < tscale || fabsf(back) < tscale));
  if (h.hit && !h.uncertain && k_out) {
    if (opt.samples_fixed > 0) {
      *k_out = opt.samples_fixed;
    } else {
      float L = h.clipped ? (tc.hi + eta) : 2.f * eta;
      float xk = opt.samples_per_unit * L;
      float c = ceilf(xk);
      if (fabsf(xk - rintf(xk)) < kEpsK) h.uncertain = true;
      int k = (int)c;
      k = k < opt.samples_min ? opt.samples_min : (k > opt.samples_max ? opt.samples_max : k);
      *k_out = k;
    }
  }
  return h;
}

struct HitDF {
  bool hit, clipped;
  df tc, eta;
  float g;
  int K;
};

// the same test evaluated entirely in double-float from the raw inputs
__device__ HitDF hit_test_df(const float* __restrict__ center, const float* __restrict__ scale,
                             const float* __restrict__ quat, int p, float3 o, float3 d,
                             const msplat_opts& opt, float kappa) {
  float q[4] = {quat[4 * p], quat[4 * p + 1], quat[4 * p + 2], quat[4 * p + 3]};
  df n2 = two_prod(q[0], q[0]);
  for (int k = 1; k < 4; ++k) n2 = df_add(n2, two_prod(q[k], q[k]));
  df nrm = df_sqrt(n2);
  df w = df_div(df_from(q[0]), nrm), x = df_div(df_from(q[1]), nrm);
  df y = df_div(df_from(q[2]), nrm), z = df_div(df_from(q[3]), nrm);
  df one = df_from(1.f), two = df_from(2.f);
  df r[9];
  r[0] = df_sub(one, df_mul(two, df_add(df_mul(y, y), df_mul(z, z))));
  r[1] = df_mul(two, df_sub(df_mul(x, y), df_mul(w, z)));
  r[2] = df_mul(two, df_add(df_mul(x, z), df_mul(w, y)));
  r[3] = df_mul(two, df_add(df_mul(x, y), df_mul(w, z)));
  r[4] = df_sub(one, df_mul(two, df_add(df_mul(x, x), df_mul(z, z))));
  r[5] = df_mul(two, df_sub(df_mul(y, z), df_mul(w, x)));
  r[6] = df_mul(two, df_sub(df_mul(x, z), df_mul(w, y)));
  r[7] = df_mul(two, df_add(df_mul(y, z), df_mul(w, x)));
  r[8] = df_sub(one, df_mul(two, df_add(df_mul(x, x), df_mul(y, y))));
  df v[3] = {two_sum(center[3 * p], -o.x), two_sum(center[3 * p + 1], -o.y),
             two_sum(center[3 * p + 2], -o.z)};
  float dd[3] = {d.x, d.y, d.z};
  df m[3], e[3];
  for (int a = 0; a < 3; ++a) {
    df inv_s = df_div(one, two_prod(kappa, scale[3 * p + a]));
    df sm = df_from(0.f), se = df_from(0.f);
    for (int b = 0; b < 3; ++b) {
      df mab = r[3 * b + a];
      sm = df_add(sm, df_mul(mab, v[b]));
      se = df_add(se, df_mulf(mab, dd[b]));
    }
    m[a] = df_mul(sm, inv_s);
    e[a] = df_mul(se, inv_s);
  }
  df aa = df_add(df_add(df_mul(e[0], e[0]), df_mul(e[1], e[1])), df_mul(e[2], e[2]));
  df em = df_add(df_add(df_mul(e[0], m[0]), df_mul(e[1], m[1])), df_mul(e[2], m[2]));
  df tc = df_div(em, aa);
  df gsum = df_from(0.f);
  for (int k = 0; k < 3; ++k) {
    df pck = df_sub(df_mul(tc, e[k]), m[k]);
    gsum = df_add(gsum, df_mul(pck, pck));
  }
  df g = df_sub(one, gsum);
  HitDF h;
  h.tc = tc;
  h.g = g.hi;
  h.hit = false;
  h.clipped = false;
  h.eta = df_from(0.f);
  h.K = 0;
  if (df_sign(g) <= 0) return h;
  df eta = df_sqrt(df_div(g, aa));
  h.eta = eta;
  if (df_sign(df_add(tc, eta)) <= 0) return h;
  h.hit = true;
  h.clipped = df_sign(df_sub(tc, eta)) <= 0;
  if (opt.samples_fixed > 0) {
    h.K = opt.samples_fixed;
  } else {
    df L = h.clipped ? df_add(tc, eta) : df_mul(two, eta);
    df xk = df_mulf(L, opt.samples_per_unit);
    float c = ceilf(xk.hi);
    if (c == xk.hi && xk.lo > 0.f) c += 1.f;
    int k = (int)c;
    h.K = k < opt.samples_min ? opt.samples_min : (k > opt.samples_max ? opt.samples_max : k);
  }
  return h;
}

// --------------------------------------------------------- packet culling --

struct Cone {
  float ox, oy, oz, dx, dy, dz, cos_t, sin_t, rho;
  bool all;
  float3 vo, vd;   // the packet's virtual ray: mean origin, normalised direction sum
};

__device__ __forceinline__ Cone packet_cone(bool valid, float3 o, float3 d) {
  Cone c;
  float nv = (float)__popcll(__ballot(valid));
  float sx = wave_sum(valid ? o.x : 0.f), sy = wave_sum(valid ? o.y : 0.f),
        sz = wave_sum(valid ? o.z : 0.f);
  c.ox = sx / nv; c.oy = sy / nv; c.oz = sz / nv;
  float ex = o.x - c.ox, ey = o.y - c.oy, ez = o.z - c.oz;
  float r2 = wave_max(valid ? ex * ex + ey * ey + ez * ez : 0.f);
  c.rho = sqrtf(r2);
  float ax = wave_sum(valid ? d.x : 0.f), ay = wave_sum(valid ? d.y : 0.f),
        az = wave_sum(valid ? d.z : 0.f);
  float an = sqrtf(ax * ax + ay * ay + az * az);
  c.vo = make_float3(c.ox, c.oy, c.oz);
  c.vd = an > 0.f ? make_float3(ax / an, ay / an, az / an) : make_float3(0.f, 0.f, 1.f);
  c.all = true;
  c.cos_t = -1.f;
  c.sin_t = 0.f;
  c.dx = c.dy = c.dz = 0.f;
  if (an > 1e-6f * nv) {
    c.dx = ax / an; c.dy = ay / an; c.dz = az / an;
    float dn = sqrtf(d.x * d.x + d.y * d.y + d.z * d.z);
    float cdot = (d.x * c.dx + d.y * c.dy + d.z * c.dz) / dn;
    float cmin = wave_min(valid ? cdot : 1.f);
    float ct = cmin - 1e-4f;                  // widen the cone a little
    if (ct > 0.1f) {
      c.all = false;
      c.cos_t = ct;
      c.sin_t = sqrtf(fmaxf(0.f, 1.f - ct * ct));
    }
  }
  return c;
}

// conservative test: can any ray of the packet pass within `rad` of `cen`?
__device__ __forceinline__ bool cone_may_hit(const Cone& c, float cx, float cy, float cz, float rad) {
  if (c.all) return true;
  float vx = cx - c.ox, vy = cy - c.oy, vz = cz - c.oz;
  float a = vx * c.dx + vy * c.dy + vz * c.dz;
  float v2 = vx * vx + vy * vy + vz * vz;
  float b = sqrtf(fmaxf(v2 - a * a, 0.f));
  float dist = (a * c.cos_t + b * c.sin_t >= 0.f) ? (b * c.cos_t - a * c.sin_t) : sqrtf(v2);
  float r = (rad + c.rho) * (1.f + 1e-4f) + 1e-5f * (1.f + sqrtf(v2));
  return dist <= r;
}

// ---------------------------------------------------------- count kernel --

constexpr int kBinHistMax = 8192;   // primitives counted in LDS per workgroup (32 KiB)

__global__ __launch_bounds__(256) void bin_count_kernel(
    const float* __restrict__ ray_o, const float* __restrict__ ray_d,
    const float* __restrict__ center, const float* __restrict__ scale,
    const float* __restrict__ quat, const float* __restrict__ geo, int64_t R, int P,
    msplat_opts opt, float kappa, int32_t* __restrict__ ray_cnt, int32_t* __restrict__ prim_nhit,
    DevCounters* __restrict__ ctr) {
  // per-primitive hit counts of the workgroup's packets, added to the global
  // counts once at the end (same-address atomics from every packet serialise)
  extern __shared__ int hist[];
  if (P <= kBinHistMax) {
    for (int i = threadIdx.x; i < P; i += blockDim.x) hist[i] = 0;
  }
  __syncthreads();
  int64_t packet = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  int lane = lane_id();
  int64_t ray = packet * kWave + lane;
  // a wave past the last ray skips the work but still meets the workgroup
  // barriers below (wave-uniform)
  const bool live = packet * kWave < R;
  bool valid = ray < R;
  float3 o = valid ? ld3(ray_o, ray) : make_float3(0.f, 0.f, 0.f);
  float3 d = valid ? ld3(ray_d, ray) : make_float3(0.f, 0.f, 1.f);
  Cone cone = packet_cone(valid, o, d);
  int nhit = 0;
  int64_t nsamp = 0;
  int nfall = 0;
  float min_g = 3.0e38f;
  for (int base = 0; live && base < P; base += kWave) {
    int pl = base + lane;
    bool cand = false;
    if (pl < P) {
      const float* gp = geo + (int64_t)pl * kGeoStride;
      cand = cone_may_hit(cone, gp[G_MU], gp[G_MU + 1], gp[G_MU + 2], gp[G_RAD]);
    }
    uint64_t mask = __ballot(cand);
    while (mask) {
      int bit = __builtin_ctzll(mask);
      mask &= mask - 1;
      int p = __builtin_amdgcn_readfirstlane(base + bit);
      const float* gp = geo + (int64_t)p * kGeoStride;
      bool hit = false;
      int K = 0;
      if (valid) {
        HitF h = hit_test_f32(gp, o, d, opt, &K);
        if (h.tc_hi + h.eta > 0.f) min_g = fminf(min_g, fabsf(h.g));
        hit = h.hit;
        if (h.uncertain) {
          HitDF hd = hit_test_df(center, scale, quat, p, o, d, opt, kappa);
          hit = hd.hit;
          K = hd.K;
          ++nfall;
        }
      }
      if (hit) {
        ++nhit;
        nsamp += K;
      }
      int cnt = __popcll(__ballot(hit));
      if (lane == 0 && cnt) {
        if (P <= kBinHistMax) atomicAdd(&hist[p], cnt);
        else atomicAdd(&prim_nhit[p], cnt);
      }
    }
  }
  if (valid) ray_cnt[ray + 1] = nhit;
  int64_t ws = wave_sum(nsamp);
  int64_t wh = wave_sum((int64_t)nhit);
  int wf = wave_sum(nfall);
  float wm = wave_min(min_g);
  // the workgroup's waves combine their counters in LDS first: one set of
  // atomics per workgroup (same-address atomics from every wave serialise)
  __shared__ unsigned long long bs_samp, bs_hits;
  __shared__ int bs_fall;
  __shared__ uint32_t bs_ming;
  if (threadIdx.x == 0) {
    bs_samp = 0ull;
    bs_hits = 0ull;
    bs_fall = 0;
    bs_ming = 0x7f7fffffu;
  }
  __syncthreads();
  if (lane == 0) {
    atomicAdd(&bs_samp, (unsigned long long)ws);
    atomicAdd(&bs_hits, (unsigned long long)wh);
    atomicAdd(&bs_fall, wf);
    atomicMin(&bs_ming, __float_as_uint(wm));
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicAdd((unsigned long long*)&ctr->num_samples, bs_samp);
    atomicAdd((unsigned long long*)&ctr->hit_total, bs_hits);
    if (bs_fall) atomicAdd(&ctr->num_fallbacks, bs_fall);
    atomicMin(&ctr->min_abs_g_bits, bs_ming);
  }
  if (P <= kBinHistMax) {
    for (int i = threadIdx.x; i < P; i += blockDim.x)
      if (hist[i]) atomicAdd(&prim_nhit[i], hist[i]);
  }
}

// ----------------------------------------------------------------- scans --

constexpr int kScanBlock = 1024;

// inclusive scan of data[0..n) in blocks of 1024, block totals to sums
__global__ __launch_bounds__(256) void scan_blocks_kernel(int32_t* __restrict__ data, int64_t n,
                                                          int32_t* __restrict__ sums) {
  __shared__ int32_t wsum[4];
  int64_t base = (int64_t)blockIdx.x * kScanBlock;
  int t = threadIdx.x;
  int32_t v[4];
  int32_t acc = 0;
  for (int k = 0; k < 4; ++k) {
    int64_t i = base + 4 * t + k;
    v[k] = i < n ? data[i] : 0;
    acc += v[k];
    v[k] = acc;
  }
  int incl = wave_incl_scan(acc);
  int w = t / kWave;
  if (lane_id() == kWave - 1) wsum[w] = incl;
  __syncthreads();
  int wo = 0;
  for (int k = 0; k < w; ++k) wo += wsum[k];
  int excl = incl - acc + wo;
  for (int k = 0; k < 4; ++k) {
    int64_t i = base + 4 * t + k;
    if (i < n) data[i] = v[k] + excl;
  }
  if (t == 255) sums[blockIdx.x] = excl + acc;
}

// exclusive scan of the (few) block sums by one workgroup, in chunks
__global__ __launch_bounds__(256) void scan_sums_kernel(int32_t* __restrict__ sums, int64_t nb,
                                                        int32_t* __restrict__ total) {
  __shared__ int32_t wsum[4];
  __shared__ int32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nb; base += 256) {
    int64_t i = base + threadIdx.x;
    int32_t v = i < nb ? sums[i] : 0;
    int incl = wave_incl_scan(v);
    int w = threadIdx.x / kWave;
    if (lane_id() == kWave - 1) wsum[w] = incl;
    __syncthreads();
    int wo = carry;
    for (int k = 0; k < w; ++k) wo += wsum[k];
    if (i < nb) sums[i] = incl - v + wo;
    __syncthreads();
    if (threadIdx.x == 255) carry = wo + incl;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(256) void scan_add_kernel(int32_t* __restrict__ data, int64_t n,
                                                       const int32_t* __restrict__ sums) {
  int64_t base = (int64_t)blockIdx.x * kScanBlock;
  int32_t add = sums[blockIdx.x];
  for (int k = threadIdx.x; k < kScanBlock; k += 256) {
    int64_t i = base + k;
    if (i < n) data[i] += add;
  }
}

// per-primitive offsets, cursors and work items (one workgroup)
__global__ __launch_bounds__(256) void prim_scan_kernel(const int32_t* __restrict__ prim_nhit,
                                                        int32_t* __restrict__ prim_off,
                                                        int32_t* __restrict__ prim_cursor,
                                                        int32_t* __restrict__ wi_off, int P,
                                                        const int32_t* __restrict__ ray_off,
                                                        int64_t R, DevCounters* __restrict__ ctr,
                                                        int64_t hit_cap, NetShape net, int hpi) {
  __shared__ int32_t wsum[2][4];
  __shared__ int32_t carry[2];
  if (threadIdx.x == 0) carry[0] = carry[1] = 0;
  __syncthreads();
  for (int base = 0; base < P; base += 256) {
    int i = base + threadIdx.x;
    int32_t n = i < P ? prim_nhit[i] : 0;
    int32_t wi = (n + hpi - 1) / hpi;
    int in = wave_incl_scan(n);
    int iw = wave_incl_scan(wi);
    int w = threadIdx.x / kWave;
    if (lane_id() == kWave - 1) {
      wsum[0][w] = in;
      wsum[1][w] = iw;
    }
    __syncthreads();
    int on = carry[0], ow = carry[1];
    for (int k = 0; k < w; ++k) {
      on += wsum[0][k];
      ow += wsum[1][k];
    }
    if (i < P) {
      prim_off[i] = in - n + on;
      prim_cursor[i] = in - n + on;
      wi_off[i] = iw - wi + ow;
    }
    __syncthreads();
    if (threadIdx.x == 255) {
      carry[0] = on + in;
      carry[1] = ow + iw;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    prim_off[P] = carry[0];
    wi_off[P] = carry[1];
    ctr->num_hits = ray_off[R];
    ctr->num_work_items = carry[1];
    ctr->num_rays = R;
    ctr->hit_cap = hit_cap;
    ctr->num_prims = P;
    ctr->num_params = net.n_params;
    ctr->net[0] = net.L;
    ctr->net[1] = net.W;
    ctr->net[2] = net.D;
    ctr->net[3] = net.NOUT;
    ctr->net[4] = net.prec;
    ctr->net[5] = net.kind;
    ctr->hits_per_item = hpi;
    ctr->magic = kCountersMagic;
  }
}

// offsets of each primitive's workgroups in the network kernels: primitive
// i's hits [prim_off[i], prim_off[i+1]) in runs of ghits (one workgroup)
__global__ __launch_bounds__(256) void group_scan_kernel(const int32_t* __restrict__ prim_off, int P, int ghits,
                                                         int32_t* __restrict__ gw_off) {
  __shared__ int32_t wsum[4];
  __shared__ int32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < P; base += 256) {
    const int i = base + threadIdx.x;
    const int32_t n = i < P ? (prim_off[i + 1] - prim_off[i] + ghits - 1) / ghits : 0;
    const int incl = wave_incl_scan(n);
    const int w = threadIdx.x / kWave;
    if (lane_id() == kWave - 1) wsum[w] = incl;
    __syncthreads();
    int o = carry;
    for (int k = 0; k < w; ++k) o += wsum[k];
    if (i < P) gw_off[i] = incl - n + o;
    __syncthreads();
    if (threadIdx.x == 255) carry = o + incl;
    __syncthreads();
  }
  if (threadIdx.x == 0) gw_off[P] = carry;
}

// ----------------------------------------------------------- tile order --

// contact depth of a primitive along the packet's virtual ray (vo, vd): the
// unclamped minimiser of Eq. 1, t = (M vd).(M (mu - vo)) / |M vd|^2, in
// float32.  The sort key of tile order (Sec. 3.3, after Eq. 2), shared by the
// packet's rays.
__device__ __forceinline__ float virtual_depth(const float* __restrict__ g, float3 vo, float3 vd) {
  const float* M = g + G_M_HI;
  const float v[3] = {g[G_MU] - vo.x, g[G_MU + 1] - vo.y, g[G_MU + 2] - vo.z};
  const float dd[3] = {vd.x, vd.y, vd.z};
  float em = 0.f, ee = 0.f;
  for (int r = 0; r < 3; ++r) {
    const float m = M[3 * r] * v[0] + M[3 * r + 1] * v[1] + M[3 * r + 2] * v[2];
    const float e = M[3 * r] * dd[0] + M[3 * r + 1] * dd[1] + M[3 * r + 2] * dd[2];
    em += e * m;
    ee += e * e;
  }
  return em / ee;
}

// (key, primitive) as one unsigned integer whose order is the lexicographic
// order of (key, primitive) for non-NaN keys (-0 is taken as +0)
__device__ __forceinline__ uint64_t kp_pack(float key, int p) {
  uint32_t u = __float_as_uint(key + 0.f);
  u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return ((uint64_t)u << 32) | (uint32_t)p;
}

constexpr int kTileNE = 8;                  // candidates held per lane
constexpr int kTileMax = kTileNE * kWave;   // candidates a packet sorts in registers

// a packet's candidates as packed (key, primitive), element e in lane e % 64
// of register e / 64; unused elements hold the largest value
struct TileList {
  uint64_t v[kTileNE];
};

// bit position of the i-th (from 0) set bit of m; i < popcount(m)
__device__ __forceinline__ int nth_bit(uint64_t m, int i) {
  int pos = 0;
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) {
    const int c = __popcll(m & ((1ull << w) - 1ull));
    if (i >= c) {
      i -= c;
      m >>= w;
      pos += w;
    }
  }
  return pos;
}

// gather the packet's candidates with their keys, in primitive order (the
// culling test of the hit passes); false if there are more than kTileMax
__device__ bool tile_collect(const Cone& cone, const float* __restrict__ geo, int P, int lane, TileList& t,
                             int& nc) {
#pragma unroll
  for (int r = 0; r < kTileNE; ++r) t.v[r] = ~0ull;
  nc = 0;
  for (int base = 0; base < P; base += kWave) {
    const int pl = base + lane;
    bool cand = false;
    uint64_t kv = 0;
    if (pl < P) {
      const float* gp = geo + (int64_t)pl * kGeoStride;
      cand = cone_may_hit(cone, gp[G_MU], gp[G_MU + 1], gp[G_MU + 2], gp[G_RAD]);
      if (cand) kv = kp_pack(virtual_depth(gp, cone.vo, cone.vd), pl);
    }
    const uint64_t mask = __ballot(cand);
    const int cnt = __popcll(mask);
    if (cnt == 0) continue;
    if (nc + cnt > kTileMax) return false;
    // element nc + i of the list takes the chunk's i-th candidate lane
#pragma unroll
    for (int r = 0; r < kTileNE; ++r) {
      if ((r + 1) * kWave <= nc || r * kWave >= nc + cnt) continue;   // (wave-uniform)
      const int i = r * kWave + lane - nc;
      const bool mine = i >= 0 && i < cnt;
      const uint64_t x = __shfl(kv, nth_bit(mask, mine ? i : 0), kWave);
      if (mine) t.v[r] = x;
    }
    nc += cnt;
  }
  return true;
}

// one stage (run length KK, partner distance J) of an ascending bitonic sort
// of the first 64 NR elements of a register list (element e in lane e % 64
// of register e / 64), then the stages after it.  Every index is a
// compile-time constant, so the list stays in registers.
template <int NR, int KK, int J, int CAP>
__device__ __forceinline__ void bitonic_stage(uint64_t (&v)[CAP], int lane) {
  if constexpr (J >= kWave) {
    // partner in the same lane, register r ^ (J / 64)
    constexpr int D = J / kWave;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (r & D) continue;
      const int q = r | D;
      const bool asc = ((r * kWave + lane) & KK) == 0;
      const uint64_t a = v[r], b = v[q];
      const bool sw = asc ? (b < a) : (a < b);
      v[r] = sw ? b : a;
      v[q] = sw ? a : b;
    }
  } else {
    // partner in lane ^ J: the lower lane keeps the smaller element of an
    // ascending run, the larger of a descending one
    const bool lower = (lane & J) == 0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const uint64_t x = __shfl_xor(v[r], J, kWave);
      const bool asc = ((r * kWave + lane) & KK) == 0;
      const bool take = (lower == asc) ? (x < v[r]) : (v[r] < x);
      if (take) v[r] = x;
    }
  }
  if constexpr (J > 1) bitonic_stage<NR, KK, J / 2>(v, lane);
  else if constexpr (KK < NR * kWave) bitonic_stage<NR, 2 * KK, KK>(v, lane);
}

template <int NR, int CAP>
__device__ __forceinline__ void reg_sort(uint64_t (&v)[CAP], int lane) {
  static_assert(NR <= CAP, "sorted registers exist");
  bitonic_stage<NR, 2, 1>(v, lane);
}

// primitive of list element i (wave-uniform i)
__device__ __forceinline__ int tile_prim(const TileList& t, int i) {
  const int r = i / kWave;
  uint32_t v = (uint32_t)t.v[0];
#pragma unroll
  for (int q = 1; q < kTileNE; ++q)
    if (r == q) v = (uint32_t)t.v[q];
  return (int)__builtin_amdgcn_readlane(v, i % kWave);
}

// ----------------------------------------------------------- fill kernel --

// strict weak order on (t_c, prim) with double-float recomputation of close keys
__device__ __forceinline__ bool key_less(float ahi, float alo, int ap, float bhi, float blo, int bp,
                                         const float* center, const float* scale, const float* quat,
                                         float3 o, float3 d, const msplat_opts& opt, float kappa) {
  float diff = (ahi - bhi) + (alo - blo);
  if (fabsf(diff) > kEpsKey * (1.f + fabsf(ahi))) return diff < 0.f;
  HitDF a = hit_test_df(center, scale, quat, ap, o, d, opt, kappa);
  HitDF b = hit_test_df(center, scale, quat, bp, o, d, opt, kappa);
  int sg = df_sign(df_sub(a.tc, b.tc));
  if (sg != 0) return sg < 0;
  return ap < bp;
}

// the per-hit record of hit j (ray `ray`, primitive p) from its contact depth,
// sample count and clip flag: residual, local contact point and direction as
// double-floats, the refined contact depth and half chord, chord start and bin
// width (pass 3 of the fill)
template <bool CONTACT>
__device__ __forceinline__ void hit_record(const Workspace& ws, const float* __restrict__ geo, int64_t j, int p,
                                           float3 o, float3 d, int64_t ray) {
  const int64_t H = ws.hit_cap;
  const float* gp = geo + (int64_t)p * kGeoStride;
  const float* Mh = gp + G_M_HI;
  const float* Ml = gp + G_M_LO;
  float tch = ws.hit_tc_hi[j], tcl = ws.hit_tc_lo[j];
  int kk = ws.hit_k[j];
  bool clipped = kk < 0;
  int K = clipped ? -kk : kk;
  // residual delta = (mu - o) - t_c d and the local contact point
  // p_c = -M delta and direction e = M d, all as double-floats: sample
  // positions feed an encoding of frequency up to 2^(L-1) pi, so their
  // float32 rounding would be amplified into the gradients
  const float dd[3] = {d.x, d.y, d.z};
  const float oo[3] = {o.x, o.y, o.z};
  df tc = {tch, tcl};
  df dl[3];
  for (int k = 0; k < 3; ++k) dl[k] = df_sub(two_sum(gp[G_MU + k], -oo[k]), df_mulf(tc, dd[k]));
  df pcv[3], ev[3];
  for (int r = 0; r < 3; ++r) {
    df pc = {0.f, 0.f}, e = {0.f, 0.f};
    for (int c = 0; c < 3; ++c) {
      const df m = {Mh[3 * r + c], Ml[3 * r + c]};
      pc = df_add(pc, df_mul(m, dl[c]));
      e = df_add(e, df_mulf(m, dd[c]));
    }
    pcv[r] = df_neg(pc);
    ev[r] = e;
  }
  // The sort key t_c is accurate to float32 only; samples are placed
  // relative to t_c, so refine it to double-float accuracy: one Newton step
  // on (p_c + dt e) . e = 0, i.e. dt = -(p_c . e) / |e|^2.
  df aa = {0.f, 0.f}, pe = {0.f, 0.f};
  for (int r = 0; r < 3; ++r) {
    aa = df_add(aa, df_mul(ev[r], ev[r]));
    pe = df_add(pe, df_mul(pcv[r], ev[r]));
  }
  const float dtc = -pe.hi / aa.hi;
  tc = df_add(tc, df_from(dtc));
  ws.hit_tc_hi[j] = tc.hi;
  ws.hit_tc_lo[j] = tc.lo;
  if constexpr (CONTACT) {
    // the contact-point primitive (Sec. 3.2): one interaction at the clamped
    // contact depth t* = max(t_c, 0) (Eq. 2); the network reads the residual
    // delta = mu - (o + t* d) (double-float, in the position arrays) and the
    // ray direction (in the direction arrays); the optical depth is
    // sigma * G * thickness with the Gaussian falloff G = exp(-|y|^2 / 2),
    // y = kappa M delta (the 1-sigma frame), and the thickness sqrt(2 pi) / |kappa M d|
    const df ts = df_sign(tc) > 0 ? tc : df{0.f, 0.f};
    float y2 = 0.f;
    for (int k = 0; k < 3; ++k) dl[k] = df_sub(two_sum(gp[G_MU + k], -oo[k]), df_mulf(ts, dd[k]));
    for (int r = 0; r < 3; ++r) {
      df yr = {0.f, 0.f};
      for (int c = 0; c < 3; ++c) yr = df_add(yr, df_mul(df{Mh[3 * r + c], Ml[3 * r + c]}, dl[c]));
      const float y = kContactKappa * yr.hi;
      y2 += y * y;
    }
    for (int r = 0; r < 3; ++r) {
      ws.hit_pc[r * H + j] = dl[r].hi;
      ws.hit_pc_lo[r * H + j] = dl[r].lo;
      ws.hit_e[r * H + j] = dd[r];
      ws.hit_e_lo[r * H + j] = 0.f;
    }
    const float thick = 2.50662827463100050f / (kContactKappa * sqrtf(aa.hi));   // sqrt(2 pi)
    ws.hit_dlt[j] = __expf(-0.5f * y2) * thick;
    ws.hit_dlt_lo[j] = 0.f;
    ws.hit_sa[j] = 0.f;
    ws.hit_sa_lo[j] = 0.f;
    ws.hit_k[j] = 1;
    ws.hit_ray[j] = (int32_t)ray;
    return;
  }
  df gg = {1.f, 0.f};
  for (int r = 0; r < 3; ++r) {
    pcv[r] = df_add(pcv[r], df_mulf(ev[r], dtc));
    gg = df_sub(gg, df_mul(pcv[r], pcv[r]));
    ws.hit_pc[r * H + j] = pcv[r].hi;
    ws.hit_pc_lo[r * H + j] = pcv[r].lo;
    ws.hit_e[r * H + j] = ev[r].hi;
    ws.hit_e_lo[r * H + j] = ev[r].lo;
  }
  // half chord eta = sqrt((1 - |p_c|^2) / |e|^2) from the refined contact point
  const df etad = df_sqrt(df_div(gg, aa));
  ws.hit_eta[j] = etad.hi;
  df sa, dlt;
  const df Kd = {(float)K, 0.f};
  if (clipped) {
    sa = df_neg(tc);
    dlt = df_div(df_add(tc, etad), Kd);
  } else {
    sa = df_neg(etad);
    dlt = df_div(df_mulf(etad, 2.f), Kd);
  }
  ws.hit_sa[j] = sa.hi;
  ws.hit_sa_lo[j] = sa.lo;
  ws.hit_dlt[j] = dlt.hi;
  ws.hit_dlt_lo[j] = dlt.lo;
  ws.hit_k[j] = K | (clipped ? kClippedBit : 0);
  ws.hit_ray[j] = (int32_t)ray;
}

// entries of the lanes' hits j (act) in their primitives' lists: the lanes
// are grouped by primitive (ballots only), then every group's first lane
// reserves the group's slots with one atomic, all groups at once (a
// reservation per group in turn would wait for each atomic's return); ranks
// within a group by lane
__device__ __forceinline__ void list_by_primitive(const Workspace& ws, bool act, int p, int64_t j, int lane) {
  uint64_t pending = __ballot(act);
  int leader_of = lane, rank = 0, cnt = 0;
  while (pending) {
    const int leader = __builtin_ctzll(pending);
    const int lp = __shfl(p, leader, 64);
    const bool mine = act && p == lp;
    const uint64_t same = __ballot(mine);
    if (mine) {
      leader_of = leader;
      rank = __popcll(same & ((1ull << lane) - 1ull));
    }
    if (lane == leader) cnt = __popcll(same);
    pending &= ~same;
  }
  int base = 0;
  if (act && lane == leader_of) base = atomicAdd(&ws.prim_cursor[p], cnt);
  base = __shfl(base, leader_of, 64);
  if (act) ws.phit[base + rank] = (int32_t)j;
}

// A group's hits sorted in registers: up to kGroupNR * 64 of them, as 64-bit
// keys (ray lane << 58 | order key << 26 | index of the hit in the packet's
// staging order), element e in lane e % 64 of register e / 64
constexpr int kGroupNR = 8;
constexpr int kGroupMax = kGroupNR * kWave;
constexpr int kPackIdxBits = 26;

// orderable bits of a float key (as kp_pack)
__device__ __forceinline__ uint32_t key_bits(float key) {
  uint32_t u = __float_as_uint(key + 0.f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key_float(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

// Fill: every ray's hits, depth-ordered (primitive, contact depth, sample
// count and clip flag, half chord, ray).  A packet of 64 rays owns the
// contiguous range of hit slots [ray_off[first ray], ray_off[last ray + 1]),
// and a group of its consecutive rays the contiguous part of that range that
// the group's rays own.  The packet is cut into the fewest groups of 64 / G
// rays (G a power of two) whose hits number at most kGroupMax each; the hits
// are appended in hit-test order (the lanes of one group that hit one
// candidate write consecutive slots) to a staging copy, then every group's
// hits are sorted in registers by (ray, depth key, test order) and written
// in slot order, one slot per lane, so that memory is touched in contiguous
// runs.  Keys closer than the float32 test can separate are re-ordered per
// ray with the double-float comparison.  A packet with a ray of more than
// kGroupMax hits falls back to appending into each ray's own segment and an
// insertion sort there.  The per-hit records follow in hit_record_kernel.
template <bool TILE>
__global__ __launch_bounds__(256) void bin_fill_kernel(
    const float* __restrict__ ray_o, const float* __restrict__ ray_d,
    const float* __restrict__ center, const float* __restrict__ scale,
    const float* __restrict__ quat, const float* __restrict__ geo, int64_t R, int P,
    msplat_opts opt, float kappa, Workspace ws) {
  int64_t packet = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  int lane = lane_id();
  int64_t ray = packet * kWave + lane;
  if (packet * kWave >= R) return;
  bool valid = ray < R;
  float3 o = valid ? ld3(ray_o, ray) : make_float3(0.f, 0.f, 0.f);
  float3 d = valid ? ld3(ray_d, ray) : make_float3(0.f, 0.f, 1.f);
  Cone cone = packet_cone(valid, o, d);
  if (TILE && opt.tile_rays) {
    // the caller's virtual ray of this packet (the ray through its tile's centre)
    const float* v = opt.tile_rays + 6 * packet;
    cone.vo = make_float3(v[0], v[1], v[2]);
    cone.vd = make_float3(v[3], v[4], v[5]);
  }
  const int64_t H = ws.hit_cap;
  int64_t off = valid ? ws.ray_off[ray] : 0;
  const int64_t last = min(packet * kWave + kWave, R);
  const int64_t pkt_off = __builtin_amdgcn_readfirstlane((int)ws.ray_off[packet * kWave]);
  const int total = __builtin_amdgcn_readfirstlane((int)(ws.ray_off[last] - pkt_off));
  // start of each lane's segment relative to the packet's (rays past the end: total)
  const int rel = valid ? (int)(off - pkt_off) : total;
  // hit test of this lane's ray against primitive p (wave-uniform): hit or
  // not, with the decided K (negative: chord clipped at t = 0), t_c and eta
  auto test = [&](int p, float& tch, float& tcl, int& kk, float& eta) __attribute__((always_inline)) -> bool {
    if (!valid) return false;
    const float* gp = geo + (int64_t)p * kGeoStride;
    int K = 0;
    HitF h = hit_test_f32(gp, o, d, opt, &K);
    bool hit = h.hit;
    bool clipped = h.clipped;
    eta = h.eta;
    if (h.uncertain) {
      HitDF hd = hit_test_df(center, scale, quat, p, o, d, opt, kappa);
      hit = hd.hit;
      K = hd.K;
      clipped = hd.clipped;
      eta = hd.eta.hi;
    }
    tch = h.tc_hi;
    tcl = h.tc_lo;
    kk = clipped ? -K : K;
    return hit;
  };
  // the packet's candidates in tile order (sorted along the virtual ray), if
  // they fit the registers
  TileList tl;
  int nc = 0;
  bool in_order = false;
  if constexpr (TILE) {
    if (tile_collect(cone, geo, P, lane, tl, nc)) {
      if (nc <= kWave) reg_sort<1>(tl.v, lane);
      else if (nc <= 2 * kWave) reg_sort<2>(tl.v, lane);
      else if (nc <= 4 * kWave) reg_sort<4>(tl.v, lane);
      else reg_sort<8>(tl.v, lane);
      in_order = true;
    }
  }
  // the fewest groups (gs = 64 / G rays each) with at most kGroupMax hits each
  int gs = kWave;
  for (; gs >= 1; gs >>= 1) {
    const int g0 = (lane % (kWave / gs)) * gs;   // lanes 0 .. G-1 check group lane
    const int start = __shfl(rel, g0, kWave);
    const int end = g0 + gs < kWave ? __shfl(rel, g0 + gs, kWave) : total;
    if (wave_max(end - start) <= kGroupMax) break;
  }

  if (gs >= 1) {
    // ---- group-wise path ----
    // staging copy of the unsorted hits and their keys: planes of hit_gv
    // (written by the backward only)
    int32_t* st_prim = reinterpret_cast<int32_t*>(ws.hit_gv);
    float* st_tch = ws.hit_gv + H;
    float* st_tcl = ws.hit_gv + 2 * H;
    int32_t* st_k = reinterpret_cast<int32_t*>(ws.hit_gv + 3 * H);
    float* st_eta = ws.hit_gv + 4 * H;
    uint32_t* st_key_hi = reinterpret_cast<uint32_t*>(ws.hit_gv + 5 * H);
    uint32_t* st_key_lo = reinterpret_cast<uint32_t*>(ws.hit_gv + 6 * H);
    const int my_g0 = (lane / gs) * gs;                      // first lane of this lane's group
    const uint64_t gmask = gs == kWave ? ~0ull : (((1ull << gs) - 1ull) << my_g0);
    const uint64_t below = (1ull << lane) - 1ull;
    const int gbase = __shfl(rel, my_g0, kWave);             // the group's first slot
    int cursor = 0;                                          // hits of this lane's group so far
    auto append = [&](int p, float okey) __attribute__((always_inline)) {
      float tch, tcl, eta;
      int kk;
      const bool hit = test(p, tch, tcl, kk, eta);
      const uint64_t mask = __ballot(hit);
      if (mask == 0) return;
      if (hit) {
        const int e = gbase + cursor + __popcll(mask & gmask & below);
        const int64_t sidx = pkt_off + e;
        st_prim[sidx] = p;
        st_tch[sidx] = tch;
        st_tcl[sidx] = tcl;
        st_k[sidx] = kk;
        st_eta[sidx] = eta;
        const uint64_t key =
            ((uint64_t)lane << 58) | ((uint64_t)key_bits(TILE ? okey : tch) << kPackIdxBits) | (uint64_t)e;
        st_key_hi[sidx] = (uint32_t)(key >> 32);
        st_key_lo[sidx] = (uint32_t)key;
      }
      cursor += __popcll(mask & gmask);
    };
    if (in_order) {
      // candidates already in tile order: the test order is the key
      for (int i = 0; i < nc; ++i) append(tile_prim(tl, i), 0.f);
    } else {
      for (int base = 0; base < P; base += kWave) {
        int pl = base + lane;
        bool cand = false;
        if (pl < P) {
          const float* gp = geo + (int64_t)pl * kGeoStride;
          cand = cone_may_hit(cone, gp[G_MU], gp[G_MU + 1], gp[G_MU + 2], gp[G_RAD]);
        }
        uint64_t mask = __ballot(cand);
        while (mask) {
          int bit = __builtin_ctzll(mask);
          mask &= mask - 1;
          const int p = __builtin_amdgcn_readfirstlane(base + bit);
          float vk = 0.f;
          if constexpr (TILE) vk = virtual_depth(geo + (int64_t)p * kGeoStride, cone.vo, cone.vd);
          append(p, vk);
        }
      }
    }
    // (every group's count equals what the count pass found: the same pairs were tested)
    __threadfence_block();
    uint64_t close = 0;   // exact order: ray lanes with two keys closer than float32 separates
    for (int g0 = 0; g0 < kWave; g0 += gs) {
      const int gb = __shfl(rel, g0, kWave);
      const int gn = (g0 + gs < kWave ? __shfl(rel, g0 + gs, kWave) : total) - gb;
      if (gn == 0) continue;
      uint64_t L[kGroupNR];
#pragma unroll
      for (int r = 0; r < kGroupNR; ++r) {
        const int pos = r * kWave + lane;
        L[r] = ~0ull;
        if (pos < gn)
          L[r] = ((uint64_t)st_key_hi[pkt_off + gb + pos] << 32) | (uint64_t)st_key_lo[pkt_off + gb + pos];
      }
      if (gn <= kWave) reg_sort<1>(L, lane);
      else if (gn <= 2 * kWave) reg_sort<2>(L, lane);
      else if (gn <= 4 * kWave) reg_sort<4>(L, lane);
      else reg_sort<8>(L, lane);
      if constexpr (!TILE) {
#pragma unroll
        for (int r = 0; r < kGroupNR; ++r) {
          if (r * kWave >= gn) break;   // (wave-uniform)
          const uint64_t nx0 = __shfl_down(L[r], 1, kWave);
          const uint64_t nx1 = __shfl(L[r + 1 < kGroupNR ? r + 1 : r], 0, kWave);
          const uint64_t nx = lane < kWave - 1 ? nx0 : nx1;
          const int pos = r * kWave + lane;
          if (pos + 1 < gn && (L[r] >> 58) == (nx >> 58)) {
            const float a = key_float((uint32_t)(L[r] >> kPackIdxBits));
            const float b = key_float((uint32_t)(nx >> kPackIdxBits));
            if (b - a <= 2.f * kEpsKey * (1.f + fabsf(a))) close |= 1ull << (L[r] >> 58);
          }
        }
      }
      // the group's sorted hits into its slots, one slot per lane
#pragma unroll
      for (int r = 0; r < kGroupNR; ++r) {
        if (r * kWave >= gn) break;   // (wave-uniform)
        const int pos = r * kWave + lane;
        if (pos < gn) {
          const int64_t src = pkt_off + (int64_t)(L[r] & ((1ull << kPackIdxBits) - 1ull));
          const int64_t j = pkt_off + gb + pos;
          ws.hit_prim[j] = st_prim[src];
          ws.hit_tc_hi[j] = st_tch[src];
          ws.hit_tc_lo[j] = st_tcl[src];
          ws.hit_k[j] = st_k[src];
          ws.hit_eta[j] = st_eta[src];
          ws.hit_ray[j] = (int32_t)(packet * kWave + (int64_t)(L[r] >> 58));
        }
      }
    }
    if constexpr (!TILE) {
#pragma unroll
      for (int sh = 32; sh >= 1; sh >>= 1) close |= __shfl_xor(close, sh, kWave);
      __threadfence_block();
      if ((close >> lane) & 1ull) {
        // insertion sort of this ray's (nearly sorted) segment with the
        // double-float comparison of close keys
        const int n = (int)(ws.ray_off[ray + 1] - off);
        for (int i = 1; i < n; ++i) {
          int64_t ji = off + i;
          int p = ws.hit_prim[ji];
          float th = ws.hit_tc_hi[ji], tlo = ws.hit_tc_lo[ji], et = ws.hit_eta[ji];
          int kk = ws.hit_k[ji];
          int j = i - 1;
          while (j >= 0) {
            int64_t jj = off + j;
            int pj = ws.hit_prim[jj];
            if (!key_less(th, tlo, p, ws.hit_tc_hi[jj], ws.hit_tc_lo[jj], pj, center, scale, quat, o, d, opt, kappa))
              break;
            ws.hit_prim[jj + 1] = pj;
            ws.hit_tc_hi[jj + 1] = ws.hit_tc_hi[jj];
            ws.hit_tc_lo[jj + 1] = ws.hit_tc_lo[jj];
            ws.hit_eta[jj + 1] = ws.hit_eta[jj];
            ws.hit_k[jj + 1] = ws.hit_k[jj];
            --j;
          }
          int64_t jd = off + j + 1;
          ws.hit_prim[jd] = p;
          ws.hit_tc_hi[jd] = th;
          ws.hit_tc_lo[jd] = tlo;
          ws.hit_eta[jd] = et;
          ws.hit_k[jd] = kk;
        }
      }
    }
    return;
  }

  // ---- per-ray path (a ray with more than kGroupMax hits) ----
  int n = 0;
  // hit test of this lane's ray against primitive p (wave-uniform); a hit is
  // appended to the ray's segment with its decided K, clip flag and eta
  auto test_append = [&](int p) __attribute__((always_inline)) {
    float tch, tcl, eta;
    int kk;
    if (test(p, tch, tcl, kk, eta)) {
      int64_t j = off + n;
      ws.hit_prim[j] = p;
      ws.hit_tc_hi[j] = tch;
      ws.hit_tc_lo[j] = tcl;
      ws.hit_k[j] = kk;
      ws.hit_eta[j] = eta;
      ++n;
    }
  };
  // tile order: every ray tests the sorted candidates in order, so its hits
  // come out sorted (a packet with more candidates than the registers hold
  // falls back to the per-ray sort below, on the same keys)
  if (in_order)
    for (int i = 0; i < nc; ++i) test_append(tile_prim(tl, i));
  // pass 1: unsorted hits (primitive order)
  for (int base = 0; !in_order && base < P; base += kWave) {
    int pl = base + lane;
    bool cand = false;
    if (pl < P) {
      const float* gp = geo + (int64_t)pl * kGeoStride;
      cand = cone_may_hit(cone, gp[G_MU], gp[G_MU + 1], gp[G_MU + 2], gp[G_RAD]);
    }
    uint64_t mask = __ballot(cand);
    while (mask) {
      int bit = __builtin_ctzll(mask);
      mask &= mask - 1;
      test_append(__builtin_amdgcn_readfirstlane(base + bit));
    }
  }
  // (lanes of rays past the end have n = 0 and stay for the wave-wide steps below)
  // pass 2: insertion sort of this ray's segment by (t_c, prim), or in tile
  // order by (virtual-ray depth, prim)
  for (int i = 1; !in_order && i < n; ++i) {
    int64_t ji = off + i;
    int p = ws.hit_prim[ji];
    float th = ws.hit_tc_hi[ji], tlo = ws.hit_tc_lo[ji], et = ws.hit_eta[ji];
    uint64_t vk = 0;
    if constexpr (TILE) vk = kp_pack(virtual_depth(geo + (int64_t)p * kGeoStride, cone.vo, cone.vd), p);
    int kk = ws.hit_k[ji];
    int j = i - 1;
    while (j >= 0) {
      int64_t jj = off + j;
      int pj = ws.hit_prim[jj];
      bool before;
      if constexpr (TILE)
        before = vk < kp_pack(virtual_depth(geo + (int64_t)pj * kGeoStride, cone.vo, cone.vd), pj);
      else
        before = key_less(th, tlo, p, ws.hit_tc_hi[jj], ws.hit_tc_lo[jj], pj, center, scale, quat, o, d, opt, kappa);
      if (!before) break;
      ws.hit_prim[jj + 1] = pj;
      ws.hit_tc_hi[jj + 1] = ws.hit_tc_hi[jj];
      ws.hit_tc_lo[jj + 1] = ws.hit_tc_lo[jj];
      ws.hit_eta[jj + 1] = ws.hit_eta[jj];
      ws.hit_k[jj + 1] = ws.hit_k[jj];
      --j;
    }
    int64_t jd = off + j + 1;
    ws.hit_prim[jd] = p;
    ws.hit_tc_hi[jd] = th;
    ws.hit_tc_lo[jd] = tlo;
    ws.hit_eta[jd] = et;
    ws.hit_k[jd] = kk;
  }
  for (int i = 0; i < n; ++i) ws.hit_ray[off + i] = (int32_t)ray;
}

// Per-hit records (one thread per hit slot, in slot order) and the
// per-primitive hit lists.
template <bool CONTACT>
__global__ __launch_bounds__(256) void hit_record_kernel(const float* __restrict__ ray_o,
                                                         const float* __restrict__ ray_d,
                                                         const float* __restrict__ geo, Workspace ws,
                                                         int64_t num_hits) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = j < num_hits;
  int p = -1;
  if (act) {
    p = ws.hit_prim[j];
    const int64_t ray = ws.hit_ray[j];
    hit_record<CONTACT>(ws, geo, j, p, ld3(ray_o, ray), ld3(ray_d, ray), ray);
  }
  list_by_primitive(ws, act, p, j, lane_id());
}

// ------------------------------------------------------------ compositor --

// optical depth kept as a double-float (compensated) sum
__device__ __forceinline__ float depth_total(float hi, float lo, float x) { return hi + (lo + x); }

// The compositor and its adjoint run one thread per ray, 256 rays per
// workgroup.  The hits of a workgroup's rays form one contiguous range of
// slots, [ray_off[r0], ray_off[r0 + 256]); it is staged through LDS in chunks
// with coalesced loads and stores, and each thread walks its own ray's hits
// there in order.  (Walking them in global memory, each step of a wave
// touches a new cache line of every hit array, and with thousands of waves in
// flight the lines are evicted before the neighbouring rays' steps reuse
// them: about five times the hit bytes came from HBM.)
constexpr int kCompRays = 256;

// slots per chunk: the LDS footprint is chunk x (words per slot) x 4 bytes
__host__ __device__ constexpr int comp_chunk(int words) { return words <= 12 ? 1024 : 512; }

__global__ __launch_bounds__(kCompRays) void composite_kernel(Workspace ws, int64_t R, msplat_opts opt,
                                                               float* __restrict__ rgb,
                                                               float* __restrict__ trans,
                                                               float* __restrict__ feat, int cf) {
  extern __shared__ __attribute__((aligned(16))) float sm[];
  const int nc = 3 + cf;
  const int C = comp_chunk(5 + nc);
  // in: optical depth, sample count, colour and feature sums; out: optical
  // depth before the hit (hi, lo), composited count
  float* s_tau = sm;
  int32_t* s_k = reinterpret_cast<int32_t*>(sm + C);
  float* s_c = sm + 2 * C;
  float* s_sbh = s_c + nc * C;
  float* s_sbl = s_sbh + C;
  int32_t* s_nu = reinterpret_cast<int32_t*>(s_sbl + C);
  const int64_t r0 = (int64_t)blockIdx.x * kCompRays;
  const int64_t ray = r0 + threadIdx.x;
  const bool act = ray < R;
  const int64_t h0 = ws.ray_off[r0];
  const int64_t h1 = ws.ray_off[min(r0 + kCompRays, R)];
  const int64_t a = act ? ws.ray_off[ray] : h1, b = act ? ws.ray_off[ray + 1] : h1;
  const int64_t H = ws.hit_cap;
  float c0 = 0.f, c1 = 0.f, c2 = 0.f;
  float f[kMaxOut - 4];
  for (int k = 0; k < kMaxOut - 4; ++k) f[k] = 0.f;
  float shi = 0.f, slo = 0.f;
  bool stopped = false;
  for (int64_t cb = h0; cb < h1; cb += C) {
    const int cn = (int)min((int64_t)C, h1 - cb);
    for (int i = threadIdx.x; i < cn; i += kCompRays) {
      s_tau[i] = ws.hit_tau[cb + i];
      s_k[i] = ws.hit_k[cb + i];
      for (int c = 0; c < nc; ++c) s_c[c * C + i] = ws.hit_cloc[c * H + cb + i];
    }
    __syncthreads();
    const int j0 = (int)(max(a, cb) - cb), j1 = (int)(min(b, cb + cn) - cb);
    for (int j = j0; j < j1; ++j) {
      if (stopped) {
        s_nu[j] = 0;
        continue;
      }
      s_sbh[j] = shi;
      s_sbl[j] = slo;
      const float tau = s_tau[j];
      const float tb = __expf(-(shi + slo));
      if (opt.t_stop > 0.f && __expf(-depth_total(shi, slo, tau)) < opt.t_stop) {
        s_nu[j] = -1;     // cut inside this hit: resolved per sample by the fixup pass
        stopped = true;
        continue;
      }
      s_nu[j] = s_k[j] & kKMask;
      c0 = __builtin_fmaf(tb, s_c[0 * C + j], c0);
      c1 = __builtin_fmaf(tb, s_c[1 * C + j], c1);
      c2 = __builtin_fmaf(tb, s_c[2 * C + j], c2);
      for (int k = 0; k < cf; ++k) f[k] = __builtin_fmaf(tb, s_c[(3 + k) * C + j], f[k]);
      df sm2 = two_sum(shi, tau);
      slo += sm2.lo;
      shi = sm2.hi;
    }
    __syncthreads();
    // (the optical depth before a hit is written where the walk reached it:
    // every hit with a non-zero composited count)
    for (int i = threadIdx.x; i < cn; i += kCompRays) {
      const int nu = s_nu[i];
      ws.hit_nused[cb + i] = nu;
      if (nu != 0) {
        ws.hit_sb_hi[cb + i] = s_sbh[i];
        ws.hit_sb_lo[cb + i] = s_sbl[i];
      }
    }
    __syncthreads();
  }
  if (!act) return;
  float t = __expf(-(shi + slo));
  if (stopped) {
    // partial sums; the fixup pass adds the cut hit and the background
    rgb[3 * ray] = c0;
    rgb[3 * ray + 1] = c1;
    rgb[3 * ray + 2] = c2;
    atomicAdd(&ws.counters->num_terminated, 1);
  } else {
    rgb[3 * ray] = c0 + t * opt.background[0];
    rgb[3 * ray + 1] = c1 + t * opt.background[1];
    rgb[3 * ray + 2] = c2 + t * opt.background[2];
    trans[ray] = t;
    ws.ray_tf[ray] = t;
  }
  for (int k = 0; k < cf; ++k) feat[ray * cf + k] = f[k];
}

// LDS words per slot of the adjoint: in: composited count, optical depth
// before the hit (hi, lo), colour (and, with a feature gradient, feature)
// sums, (with slot features) the slot product and optical depth; out: three
// backward scalars
__host__ __device__ constexpr int adj_words(int nc_read, bool slot) { return 3 + nc_read + (slot ? 2 : 0) + 3; }

// per-ray adjoint: transmittance before each hit and g . (what follows it);
// the chunks are walked from the last to the first
__global__ __launch_bounds__(kCompRays) void composite_adjoint_kernel(
    Workspace ws, int64_t R, msplat_opts opt, const float* __restrict__ grad_rgb,
    const float* __restrict__ grad_trans, const float* __restrict__ grad_feat, int cf,
    const float* __restrict__ trans) {
  extern __shared__ __attribute__((aligned(16))) float sm[];
  const int ncr = 3 + (grad_feat ? cf : 0);   // colour (and feature) sums read
  const bool slot = ws.slot_on != 0;
  const int C = comp_chunk(adj_words(ncr, slot));
  int32_t* s_nu = reinterpret_cast<int32_t*>(sm);
  float* s_sbh = sm + C;
  float* s_sbl = s_sbh + C;
  float* s_c = s_sbl + C;
  float* s_q = s_c + ncr * C;           // (slot features only)
  float* s_tau = s_q + (slot ? C : 0);
  float* s_gsa = s_tau + (slot ? C : 0);
  float* s_tb = s_gsa + C;
  float* s_gt = s_tb + C;
  const int64_t r0 = (int64_t)blockIdx.x * kCompRays;
  const int64_t ray = r0 + threadIdx.x;
  const bool act = ray < R;
  const int64_t h0 = ws.ray_off[r0];
  const int64_t h1 = ws.ray_off[min(r0 + kCompRays, R)];
  const int64_t a = act ? ws.ray_off[ray] : h1, b = act ? ws.ray_off[ray + 1] : h1;
  const int64_t H = ws.hit_cap;
  float g0 = 0.f, g1 = 0.f, g2 = 0.f, tf = 0.f, gt = 0.f;
  if (act) {
    g0 = grad_rgb[3 * ray];
    g1 = grad_rgb[3 * ray + 1];
    g2 = grad_rgb[3 * ray + 2];
    tf = trans[ray];
    gt = grad_trans ? grad_trans[ray] : 0.f;
  }
  // d(rgb)/d(tau_k) = T_{k+1} c_k - sum_{j>k} w_j c_j - T_final bg, and
  // d(T_final)/d(tau_k) = -T_final: the suffix starts with T_final (g.bg + g_T)
  // suffix sum over the later hits, kept compensated (double-float)
  df acc = df_from(tf * (g0 * opt.background[0] + g1 * opt.background[1] + g2 * opt.background[2] + gt));
  const int64_t nchunks = (h1 - h0 + C - 1) / C;
  for (int64_t ci = nchunks - 1; ci >= 0; --ci) {
    const int64_t cb = h0 + ci * C;
    const int cn = (int)min((int64_t)C, h1 - cb);
    for (int i = threadIdx.x; i < cn; i += kCompRays) {
      const int nu = ws.hit_nused[cb + i];
      s_nu[i] = nu;
      if (nu > 0) {
        s_sbh[i] = ws.hit_sb_hi[cb + i];
        s_sbl[i] = ws.hit_sb_lo[cb + i];
        for (int c = 0; c < ncr; ++c) s_c[c * C + i] = ws.hit_cloc[c * H + cb + i];
        if (slot) {
          s_q[i] = ws.hit_q[cb + i];
          s_tau[i] = ws.hit_tau[cb + i];
        }
      }
    }
    __syncthreads();
    const int j0 = (int)(max(a, cb) - cb), j1 = (int)(min(b, cb + cn) - cb);
    for (int j = j1 - 1; j >= j0; --j) {
      if (s_nu[j] <= 0) continue;
      s_gsa[j] = acc.hi + acc.lo;
      const float tb = __expf(-(s_sbh[j] + s_sbl[j]));
      float gc = g0 * s_c[0 * C + j] + g1 * s_c[1 * C + j] + g2 * s_c[2 * C + j];
      if (grad_feat)
        for (int k = 0; k < cf; ++k) gc += grad_feat[ray * cf + k] * s_c[(3 + k) * C + j];
      // slot features: a colour channel constant over the hit, composited with
      // the hit's opacity 1 - exp(-tau), whose upstream product is q
      if (slot) gc += s_q[j] * -expm1f(-s_tau[j]);
      s_tb[j] = tb;
      s_gt[j] = tb * gc;
      acc = df_add(acc, two_prod(tb, gc));
    }
    __syncthreads();
    for (int i = threadIdx.x; i < cn; i += kCompRays) {
      if (s_nu[i] > 0) {
        ws.hit_gsa[cb + i] = s_gsa[i];
        ws.hit_tb[cb + i] = s_tb[i];
        ws.hit_gtot[cb + i] = s_gt[i];
      }
    }
    __syncthreads();
  }
}

// dL/dM and dL/dv accumulated per primitive -> dL/d(center, scale, quat)
// Per-hit geometry adjoint over the primitive-grouped hit list.  A hit's samples sit at
// p_c + s_k e with s_k = (t_a - t_c) + (k + u_k) Delta; the backward kernel
// leaves per hit the sums over its samples of dL/dp, s_k dL/dp, dL/ds_k,
// omega_k dL/ds_k (omega_k = (k + u_k)/K) and of the dL/dDelta terms.  Here
// they are carried through t_a, Delta (chord ends t_c -+ eta, eta =
// sqrt(g/a)), p_c = o_l + t_c d_l and e = M d to dL/dM and dL/dv (v: the
// frame's origin offset), which the finalize kernel maps to (mu, s, q).
__device__ __forceinline__ void hit_geometry_terms(const Workspace& ws, const float* __restrict__ ray_d, int hit,
                                                   int64_t pos, int p, float (&acc)[12]) {
  const int64_t H = ws.hit_cap;
  const float* gp = ws.geo + (int64_t)p * kGeoStride;
  float gv[9], pc[3], ee[3];
  for (int k = 0; k < 9; ++k) gv[k] = ws.hit_gv[k * H + pos];
  for (int a = 0; a < 3; ++a) {
    pc[a] = ws.hit_pc[a * H + hit];
    ee[a] = ws.hit_e[a * H + hit];
  }
  const int kraw = ws.hit_k[hit];
  const bool clipped = (kraw & kClippedBit) != 0;
  const float Kf = (float)(kraw & kKMask);
  const float eta = ws.hit_eta[hit];
  const int ray = ws.hit_ray[hit];
  float dtb = gv[7] + gv[8] / Kf;
  float dta = gv[6] - gv[7] - gv[8] / Kf;
  float lam = clipped ? dtb : dtb + dta;
  float zet = clipped ? dtb : dtb - dta;
  float a2 = ee[0] * ee[0] + ee[1] * ee[1] + ee[2] * ee[2];
  float kap = eta > 0.f ? zet / (eta * a2) : 0.f;
  float dd[3] = {ray_d[3 * ray], ray_d[3 * ray + 1], ray_d[3 * ray + 2]};
  // delta_c = mu - o - t_c d = -R diag(s) p_c
  float dc[3];
  for (int r = 0; r < 3; ++r) {
    dc[r] = 0.f;
    for (int c = 0; c < 3; ++c) dc[r] -= gp[G_R + 3 * r + c] * gp[G_S + c] * pc[c];
  }
  for (int r = 0; r < 3; ++r) {
    float gm = lam * ee[r] / a2 + kap * pc[r];
    float c1 = gm - gv[r];
    float c2 = gv[3 + r] - (lam * pc[r] + zet * eta * ee[r]) / a2;
    for (int c = 0; c < 3; ++c) acc[3 * r + c] = c1 * dc[c] + c2 * dd[c];
    acc[9 + r] = c1;
  }
}

// Contact-point primitive (one interaction per hit): the backward kernel
// leaves per hit dL/d(delta) (gv 0-2) and dL/d(dlt) (gv 8), dlt = G * thickness
// the optical-depth factor.  With the support frame M (semi-axes kappa s),
// e = M d, a = |e|^2, y = kappa M delta, rho = dL/d(dlt) * dlt:
//   dL/dy = -rho y; dL/d(delta) in total: g = gv + kappa M^T dL/dy;
//   through t* = t_c = (e . M v) / a (v = mu - o; zero derivative where
//   t* is clamped at 0): lambda = -(d . g) / a;
//   dL/dM = (kappa dL/dy + lambda e) (x) delta + (lambda M delta - rho e / a) (x) d;
//   dL/dmu = g + lambda M^T e.
// acc: dL/dM (9), dL/dmu (3).
__device__ __forceinline__ void contact_geometry_terms(const Workspace& ws, const float* __restrict__ ray_d,
                                                       int hit, int64_t pos, int p, float (&acc)[12]) {
  const int64_t H = ws.hit_cap;
  const float* gp = ws.geo + (int64_t)p * kGeoStride;
  float M[9];
  for (int k = 0; k < 9; ++k) M[k] = gp[G_M_HI + k] + gp[G_M_LO + k];
  const int ray = ws.hit_ray[hit];
  const float dd[3] = {ray_d[3 * ray], ray_d[3 * ray + 1], ray_d[3 * ray + 2]};
  float dl[3], gdl[3];
  for (int a = 0; a < 3; ++a) {
    dl[a] = ws.hit_pc[a * H + hit] + ws.hit_pc_lo[a * H + hit];
    gdl[a] = ws.hit_gv[a * H + pos];
  }
  const float rho = ws.hit_gv[8 * H + pos] * ws.hit_dlt[hit];
  float e[3], md[3];
  for (int r = 0; r < 3; ++r) {
    e[r] = M[3 * r] * dd[0] + M[3 * r + 1] * dd[1] + M[3 * r + 2] * dd[2];
    md[r] = M[3 * r] * dl[0] + M[3 * r + 1] * dl[1] + M[3 * r + 2] * dl[2];
  }
  const float a2 = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
  const float k2 = kContactKappa * kContactKappa;
  // kappa dL/dy = -rho kappa^2 M delta
  float ky[3], g[3];
  for (int r = 0; r < 3; ++r) ky[r] = -rho * k2 * md[r];
  for (int c = 0; c < 3; ++c) g[c] = gdl[c] + M[c] * ky[0] + M[3 + c] * ky[1] + M[6 + c] * ky[2];
  const float lam = ws.hit_tc_hi[hit] > 0.f ? -(dd[0] * g[0] + dd[1] * g[1] + dd[2] * g[2]) / a2 : 0.f;
  for (int r = 0; r < 3; ++r) {
    const float u = ky[r] + lam * e[r];
    const float w = lam * md[r] - rho * e[r] / a2;
    for (int c = 0; c < 3; ++c) acc[3 * r + c] = u * dl[c] + w * dd[c];
  }
  for (int c = 0; c < 3; ++c) acc[9 + c] = g[c] + lam * (M[c] * e[0] + M[3 + c] * e[1] + M[6 + c] * e[2]);
}

// One thread per entry of the primitive-grouped hit list (all loads of a hit
// are issued at once; no thread walks a chain of hits).  A workgroup whose
// hits share one primitive adds its sum with one set of atomics; otherwise
// each wave whose hits share one does; otherwise each thread.
template <bool CONTACT>
__global__ __launch_bounds__(256) void hit_geometry_kernel(Workspace ws, const float* __restrict__ ray_d,
                                                           int64_t num_hits) {
  __shared__ float part[4][12];
  __shared__ int wp[4];
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float c[12];
  for (int k = 0; k < 12; ++k) c[k] = 0.f;
  int p = -1;
  if (i < num_hits) {
    const int hit = ws.phit[i];
    p = ws.hit_prim[hit];
    if (ws.hit_nused[hit] > 0) {   // (else no samples ran)
      if constexpr (CONTACT) contact_geometry_terms(ws, ray_d, hit, i, p, c);
      else hit_geometry_terms(ws, ray_d, hit, i, p, c);
    }
  }
  // the wave's primitive, or -2 if its hits belong to several (-1: no hits)
  const int pw0 = __builtin_amdgcn_readfirstlane(p);
  const int pw = __all(p == pw0 || p < 0) ? pw0 : -2;
  if (lane == 0) wp[wv] = pw;
  __syncthreads();
  int pb = wp[0];
  for (int w = 1; w < 4; ++w) {
    const int o = wp[w];
    if (o == -1) continue;
    pb = (pb == -1) ? o : (pb == o ? pb : -2);
  }
  if (pb == -2 || pw == -2) {
    // several primitives in this workgroup: per wave, or per thread
    if (pw >= 0) {
      for (int k = 0; k < 12; ++k) {
        float v = wave_sum(c[k]);
        if (lane == 0 && v != 0.f) atomicAdd(ws.geo_grad + (int64_t)pw * 12 + k, v);
      }
    } else if (pw == -2 && p >= 0) {
      for (int k = 0; k < 12; ++k)
        if (c[k] != 0.f) atomicAdd(ws.geo_grad + (int64_t)p * 12 + k, c[k]);
    }
    return;
  }
  if (pb < 0) return;   // no hits in this workgroup
  for (int k = 0; k < 12; ++k) {
    float v = wave_sum(c[k]);
    if (lane == 0) part[wv][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 12) {
    const float v = part[0][threadIdx.x] + part[1][threadIdx.x] + part[2][threadIdx.x] + part[3][threadIdx.x];
    if (v != 0.f) atomicAdd(ws.geo_grad + (int64_t)pb * 12 + threadIdx.x, v);
  }
}

// acc: dL/dM (9) and either u with dL/dmu = M^T u (chord primitives) or
// dL/dmu itself (direct_center: the contact-point primitive); the stored
// semi-axes are kappa times the scale input (kappa = 1 for chord primitives)
__global__ void geo_finalize_kernel(const float* __restrict__ geo, const float* __restrict__ acc,
                                    int P, float* __restrict__ g_center, float* __restrict__ g_scale,
                                    float* __restrict__ g_quat, bool direct_center, float kappa) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const float* gp = geo + (int64_t)i * kGeoStride;
  const float* A = acc + (int64_t)i * 12;
  float M[9], GM[9], u[3];
  for (int k = 0; k < 9; ++k) {
    M[k] = gp[G_M_HI + k] + gp[G_M_LO + k];
    GM[k] = A[k];
  }
  for (int k = 0; k < 3; ++k) u[k] = A[9 + k];
  // dL/dmu = M^T u
  for (int c = 0; c < 3; ++c)
    g_center[3 * i + c] = direct_center ? u[c] : M[c] * u[0] + M[3 + c] * u[1] + M[6 + c] * u[2];
  // M[a][b] = R[b][a] / s[a]
  float G[9];   // dL/dR
  for (int a2 = 0; a2 < 3; ++a2) {
    float s = gp[G_S + a2];
    float ds = 0.f;
    for (int b2 = 0; b2 < 3; ++b2) {
      ds += GM[3 * a2 + b2] * M[3 * a2 + b2];
      G[3 * b2 + a2] = GM[3 * a2 + b2] / s;
    }
    g_scale[3 * i + a2] = -kappa * ds / s;
  }
  float w = gp[G_QN], x = gp[G_QN + 1], y = gp[G_QN + 2], z = gp[G_QN + 3];
  float dw = 2.f * (-z * G[1] + y * G[2] + z * G[3] - x * G[5] - y * G[6] + x * G[7]);
  float dx = 2.f * (y * G[1] + z * G[2] + y * G[3] - 2.f * x * G[4] - w * G[5] + z * G[6] + w * G[7] -
                    2.f * x * G[8]);
  float dy = 2.f * (-2.f * y * G[0] + x * G[1] + w * G[2] + x * G[3] + z * G[5] - w * G[6] + z * G[7] -
                    2.f * y * G[8]);
  float dz = 2.f * (-2.f * z * G[0] - w * G[1] + x * G[2] + w * G[3] - 2.f * z * G[4] + y * G[5] + x * G[6] +
                    y * G[7]);
  float dot = w * dw + x * dx + y * dy + z * dz;
  float inv = gp[G_INVQ];
  g_quat[4 * i] = (dw - w * dot) * inv;
  g_quat[4 * i + 1] = (dx - x * dot) * inv;
  g_quat[4 * i + 2] = (dy - y * dot) * inv;
  g_quat[4 * i + 3] = (dz - z * dot) * inv;
}

__global__ void fill_kernel(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

}  // namespace

// ------------------------------------------------------------ launchers --

hipError_t launch_fill(void* p, size_t bytes, uint32_t value, hipStream_t s) {
  int64_t n = (int64_t)(bytes / 4);
  if (n == 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t*)p, n, value);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) { return launch_fill(p, bytes, 0u, s); }

hipError_t launch_preprocess(const Workspace& ws, const float* center, const float* scale,
                             const float* quat, int P, int kind, hipStream_t s) {
  hipLaunchKernelGGL(preprocess_kernel, dim3((P + 127) / 128), dim3(128), 0, s, center, scale, quat,
                     ws.geo, P, kind == MSPLAT_CONTACT ? kContactKappa : 1.f);
  return hipGetLastError();
}

static inline unsigned packet_blocks(int64_t R) {
  int64_t packets = (R + kWave - 1) / kWave;
  return (unsigned)((packets + 3) / 4);
}

hipError_t launch_bin_count(const Workspace& ws, const float* ray_o, const float* ray_d,
                             const float* center, const float* scale, const float* quat, int64_t R,
                             int P, const msplat_opts& o, int kind, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  const size_t hist_bytes = P <= kBinHistMax ? (size_t)P * 4 : 0;
  hipLaunchKernelGGL(bin_count_kernel, dim3(packet_blocks(R)), dim3(256), hist_bytes, s, ray_o, ray_d, center,
                     scale, quat, (const float*)ws.geo, R, P, o, kind == MSPLAT_CONTACT ? kContactKappa : 1.f,
                     ws.ray_off, ws.prim_nhit, ws.counters);
  return hipGetLastError();
}

hipError_t launch_scans(const Workspace& ws, int64_t R, const NetShape& net, hipStream_t s) {
  const int P = net.P;
  // ray_off[0] = 0 and ray_off[1..R] hold counts: inclusive scan of [1..R]
  int64_t n = R;
  int32_t* data = ws.ray_off + 1;
  int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb > 0) {
    hipLaunchKernelGGL(scan_blocks_kernel, dim3((unsigned)nb), dim3(256), 0, s, data, n, ws.scan_tmp);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(256), 0, s, ws.scan_tmp, nb,
                       ws.scan_tmp + nb);
    hipLaunchKernelGGL(scan_add_kernel, dim3((unsigned)nb), dim3(256), 0, s, data, n,
                       (const int32_t*)ws.scan_tmp);
  }
  hipLaunchKernelGGL(prim_scan_kernel, dim3(1), dim3(256), 0, s, (const int32_t*)ws.prim_nhit,
                     ws.prim_off, ws.prim_cursor, ws.wi_off, P, (const int32_t*)ws.ray_off, R,
                     ws.counters, ws.hit_cap, net, ws.hits_per_item);
  return hipGetLastError();
}

hipError_t launch_bin_fill(const Workspace& ws, const float* ray_o, const float* ray_d,
                           const float* center, const float* scale, const float* quat, int64_t R,
                           int P, const msplat_opts& o, int kind, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  const float kappa = kind == MSPLAT_CONTACT ? kContactKappa : 1.f;
  if (o.order == 1)
    hipLaunchKernelGGL(bin_fill_kernel<true>, dim3(packet_blocks(R)), dim3(256), 0, s, ray_o, ray_d, center,
                       scale, quat, (const float*)ws.geo, R, P, o, kappa, ws);
  else
    hipLaunchKernelGGL(bin_fill_kernel<false>, dim3(packet_blocks(R)), dim3(256), 0, s, ray_o, ray_d, center,
                       scale, quat, (const float*)ws.geo, R, P, o, kappa, ws);
  return hipGetLastError();
}

hipError_t launch_hit_records(const Workspace& ws, const float* ray_o, const float* ray_d, int64_t num_hits,
                              int kind, hipStream_t s) {
  if (num_hits <= 0) return hipSuccess;
  const dim3 grid((unsigned)((num_hits + 255) / 256));
  if (kind == MSPLAT_CONTACT)
    hipLaunchKernelGGL(hit_record_kernel<true>, grid, dim3(256), 0, s, ray_o, ray_d, (const float*)ws.geo, ws,
                       num_hits);
  else
    hipLaunchKernelGGL(hit_record_kernel<false>, grid, dim3(256), 0, s, ray_o, ray_d, (const float*)ws.geo, ws,
                       num_hits);
  return hipGetLastError();
}

hipError_t launch_group_scan(const Workspace& ws, int P, int ghits, hipStream_t s) {
  if (ghits < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(group_scan_kernel, dim3(1), dim3(256), 0, s, (const int32_t*)ws.prim_off, P, ghits,
                     ws.gw_off);
  return hipGetLastError();
}

hipError_t launch_composite(const Workspace& ws, int64_t R, const msplat_opts& o, float* rgb,
                            float* trans, float* feat, int cf, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  const int words = 5 + 3 + cf;
  const size_t lds = (size_t)comp_chunk(words) * words * 4;
  hipLaunchKernelGGL(composite_kernel, dim3((unsigned)((R + kCompRays - 1) / kCompRays)), dim3(kCompRays), lds, s,
                     ws, R, o, rgb, trans, feat, cf);
  return hipGetLastError();
}

hipError_t launch_composite_adjoint(const Workspace& ws, int64_t R, const msplat_opts& o,
                                    const float* grad_rgb, const float* grad_trans,
                                    const float* grad_feat, int cf, const float* trans,
                                    hipStream_t s) {
  if (R <= 0) return hipSuccess;
  const int words = adj_words(3 + (grad_feat ? cf : 0), ws.slot_on != 0);
  const size_t lds = (size_t)comp_chunk(words) * words * 4;
  hipLaunchKernelGGL(composite_adjoint_kernel, dim3((unsigned)((R + kCompRays - 1) / kCompRays)), dim3(kCompRays),
                     lds, s, ws, R, o, grad_rgb, grad_trans, grad_feat, cf, trans);
  return hipGetLastError();
}

hipError_t launch_hit_geometry(const Workspace& ws, const float* ray_d, int64_t num_hits, int kind, hipStream_t s) {
  if (num_hits <= 0) return hipSuccess;
  const dim3 grid((unsigned)((num_hits + 255) / 256));
  if (kind == MSPLAT_CONTACT)
    hipLaunchKernelGGL(hit_geometry_kernel<true>, grid, dim3(256), 0, s, ws, ray_d, num_hits);
  else
    hipLaunchKernelGGL(hit_geometry_kernel<false>, grid, dim3(256), 0, s, ws, ray_d, num_hits);
  return hipGetLastError();
}

hipError_t launch_geo_finalize(const Workspace& ws, int P, float* g_center, float* g_scale,
                               float* g_quat, int kind, hipStream_t s) {
  const bool contact = kind == MSPLAT_CONTACT;
  hipLaunchKernelGGL(geo_finalize_kernel, dim3((P + 127) / 128), dim3(128), 0, s,
                     (const float*)ws.geo, (const float*)ws.geo_grad, P, g_center, g_scale, g_quat, contact,
                     contact ? kContactKappa : 1.f);
  return hipGetLastError();
}

}  // namespace msplat
