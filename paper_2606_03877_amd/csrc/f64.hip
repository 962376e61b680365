// Float64 forward render, used only by the finite-difference gradient checker.
//
// One thread per ray: test every primitive (Sec. 3.2, Eq. 1-2, in float64),
// keep the hits sorted by (t_c, primitive) in a bounded private list, then
// walk them front to back, evaluating each primitive's network at the K
// stratified samples of its chord on the vector units and compositing with
// early termination (Sec. 3.3).  No culling, no grouping: it favours
// simplicity over speed and shares the sampling rules (offsets from the PCG
// hash, Delta = chord / K, the cut after the first sample below T_stop) with
// the float32 path.
#include "common.h"

namespace msplat {

namespace {

constexpr int kMaxHitsF64 = 48;

__device__ __forceinline__ void rotmat64(const double q[4], double r[9]) {
  double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
  r[0] = 1 - 2 * (y * y + z * z); r[1] = 2 * (x * y - w * z); r[2] = 2 * (x * z + w * y);
  r[3] = 2 * (x * y + w * z); r[4] = 1 - 2 * (x * x + z * z); r[5] = 2 * (y * z - w * x);
  r[6] = 2 * (x * z - w * y); r[7] = 2 * (y * z + w * x); r[8] = 1 - 2 * (x * x + y * y);
}

struct Frame64 {
  double ol[3], dl[3];
};

// local ray (o_l, d_l) in primitive p's frame
__device__ __forceinline__ Frame64 frame64(const double* center, const double* scale, const double* quat,
                                           int p, const double o[3], const double d[3]) {
  double q[4] = {quat[4 * p], quat[4 * p + 1], quat[4 * p + 2], quat[4 * p + 3]};
  double r[9];
  rotmat64(q, r);
  Frame64 f;
  for (int a = 0; a < 3; ++a) {
    double so = 0, sd = 0;
    for (int b = 0; b < 3; ++b) {
      so += r[3 * b + a] * (o[b] - center[3 * p + b]);
      sd += r[3 * b + a] * d[b];
    }
    f.ol[a] = so / scale[3 * p + a];
    f.dl[a] = sd / scale[3 * p + a];
  }
  return f;
}

// FNV-style mixing of the discrete decisions of a ray into one word
__device__ __forceinline__ uint32_t mix(uint32_t h, uint32_t v) { return (h ^ v) * 16777619u; }

template <int L, int W, int D, int NOUT>
__device__ void mlp64(const double* __restrict__ th, const double p[3], double out[NOUT], uint32_t& dec) {
  constexpr int IN = 3 + 6 * L;
  double x[IN];
  for (int a = 0; a < 3; ++a) x[a] = p[a];
  for (int l = 0; l < L; ++l)
    for (int a = 0; a < 3; ++a) {
      double arg = (double)(1 << l) * p[a];
      x[3 + 6 * l + a] = sinpi(arg);
      x[6 + 6 * l + a] = cospi(arg);
    }
  double h[W], h2[W];
  int off = 0;
  for (int n = 0; n < W; ++n) {
    double s = th[off + IN * W + n];
    for (int k = 0; k < IN; ++k) s += th[off + n * IN + k] * x[k];
    h[n] = s > 0 ? s : 0.0;
    if (s > 0) dec = mix(dec, (uint32_t)n + 1u);
  }
  off += IN * W + W;
  for (int j = 1; j < D; ++j) {
    for (int n = 0; n < W; ++n) {
      double s = th[off + W * W + n];
      for (int k = 0; k < W; ++k) s += th[off + n * W + k] * h[k];
      h2[n] = s > 0 ? s : 0.0;
      if (s > 0) dec = mix(dec, (uint32_t)(j * W + n) + 1u);
    }
    for (int n = 0; n < W; ++n) h[n] = h2[n];
    off += W * W + W;
  }
  for (int n = 0; n < NOUT; ++n) {
    double s = th[off + W * NOUT + n];
    for (int k = 0; k < W; ++k) s += th[off + n * W + k] * h[k];
    out[n] = s;
  }
}

template <int L, int W, int D, int NOUT>
__global__ __launch_bounds__(64) void forward_f64_kernel(
    const double* __restrict__ center, const double* __restrict__ scale, const double* __restrict__ quat,
    const double* __restrict__ mlp, int n_params, int P, const double* __restrict__ ray_o,
    const double* __restrict__ ray_d, int64_t R, msplat_opts opt, double* __restrict__ rgb,
    double* __restrict__ trans, double* __restrict__ feat, uint32_t* __restrict__ decisions,
    int32_t* __restrict__ overflow) {
  int64_t ray = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ray >= R) return;
  double o[3] = {ray_o[3 * ray], ray_o[3 * ray + 1], ray_o[3 * ray + 2]};
  double d[3] = {ray_d[3 * ray], ray_d[3 * ray + 1], ray_d[3 * ray + 2]};
  double ht[kMaxHitsF64], ha[kMaxHitsF64], hb[kMaxHitsF64];
  int hp[kMaxHitsF64];
  int n = 0;
  for (int p = 0; p < P; ++p) {
    Frame64 f = frame64(center, scale, quat, p, o, d);
    double a = f.dl[0] * f.dl[0] + f.dl[1] * f.dl[1] + f.dl[2] * f.dl[2];
    double tc = -(f.ol[0] * f.dl[0] + f.ol[1] * f.dl[1] + f.ol[2] * f.dl[2]) / a;
    double g = 1.0;
    for (int k = 0; k < 3; ++k) {
      double pc = f.ol[k] + tc * f.dl[k];
      g -= pc * pc;
    }
    if (!(g > 0)) continue;
    double eta = sqrt(g / a);
    if (!(tc + eta > 0)) continue;
    if (n == kMaxHitsF64) {
      atomicOr(overflow, 1);
      break;
    }
    int i = n++;
    while (i > 0 && ht[i - 1] > tc) {   // stable: equal keys keep primitive order
      ht[i] = ht[i - 1];
      ha[i] = ha[i - 1];
      hb[i] = hb[i - 1];
      hp[i] = hp[i - 1];
      --i;
    }
    ht[i] = tc;
    ha[i] = tc - eta > 0 ? tc - eta : 0.0;
    hb[i] = tc + eta;
    hp[i] = p;
  }
  constexpr int CF = NOUT - 4;
  double c[3] = {0, 0, 0}, fe[CF > 0 ? CF : 1];
  for (int k = 0; k < CF; ++k) fe[k] = 0;
  double S = 0.0;
  bool stop = false;
  uint32_t seed_hash = pcg_hash(opt.jitter_seed);
  uint32_t dec = 2166136261u;
  for (int i = 0; i < n && !stop; ++i) {
    int p = hp[i];
    dec = mix(dec, 0x80000000u | (uint32_t)p);
    Frame64 f = frame64(center, scale, quat, p, o, d);
    double Lh = hb[i] - ha[i];
    int K;
    if (opt.samples_fixed > 0) {
      K = opt.samples_fixed;
    } else {
      K = (int)ceil((double)opt.samples_per_unit * Lh);
      K = K < opt.samples_min ? opt.samples_min : (K > opt.samples_max ? opt.samples_max : K);
    }
    double dlt = Lh / K;
    const double* th = mlp + (int64_t)p * n_params;
    for (int k = 0; k < K; ++k) {
      double u = opt.jitter ? (double)sample_offset(seed_hash, (uint32_t)ray, (uint32_t)i, (uint32_t)k) : 0.5;
      double tk = ha[i] + (k + u) * dlt;
      double pk[3] = {f.ol[0] + tk * f.dl[0], f.ol[1] + tk * f.dl[1], f.ol[2] + tk * f.dl[2]};
      double out[NOUT];
      mlp64<L, W, D, NOUT>(th, pk, out, dec);
      double sig = out[3] > 0 ? out[3] + log1p(exp(-out[3])) : log1p(exp(out[3]));
      double tau = sig * dlt;
      double tb = exp(-S);
      if (opt.t_stop > 0.f && tb < (double)opt.t_stop) {
        dec = mix(dec, 0x40000000u | (uint32_t)k);
        stop = true;
        break;
      }
      double w = tb * (-expm1(-tau));
      for (int r = 0; r < 3; ++r) c[r] += w / (1.0 + exp(-out[r]));
      for (int r = 0; r < CF; ++r) fe[r] += w * out[4 + r];
      S += tau;
    }
  }
  double t = exp(-S);
  for (int r = 0; r < 3; ++r) rgb[3 * ray + r] = c[r] + t * (double)opt.background[r];
  trans[ray] = t;
  for (int r = 0; r < CF; ++r) feat[ray * CF + r] = fe[r];
  if (decisions) decisions[ray] = dec;
}

}  // namespace

hipError_t launch_forward_f64(const NetShape& n, const msplat_opts& o, const double* center,
                              const double* scale, const double* quat, const double* mlp,
                              const double* ray_o, const double* ray_d, int64_t R, double* rgb,
                              double* trans, double* feat, uint32_t* decisions, void* ws,
                              uint64_t ws_bytes, int max_hits_per_ray, hipStream_t s) {
  (void)ws_bytes;
  (void)max_hits_per_ray;
  if (R <= 0) return hipSuccess;
  int32_t* overflow = reinterpret_cast<int32_t*>(ws);
  hipError_t e = launch_zero(overflow, 256, s);
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)((R + 63) / 64)), block(64);
#define X(L_, W_, D_, O_)                                                                                   \
  if (n.L == L_ && n.W == W_ && n.D == D_ && n.NOUT == O_) {                                              \
    hipLaunchKernelGGL((forward_f64_kernel<L_, W_, D_, O_>), grid, block, 0, s, center, scale, quat, mlp, \
                       n.n_params, n.P, ray_o, ray_d, R, o, rgb, trans, feat, decisions, overflow);       \
    return hipGetLastError();                                                                             \
  }
  X(4, 32, 2, 4)
  X(6, 64, 3, 4)
  X(6, 64, 3, 20)
#undef X
  return hipErrorInvalidValue;
}

int f64_max_hits() { return kMaxHitsF64; }

}  // namespace msplat
