// Grouped per-primitive MLP kernels (Sec. 3.2 network, Sec. 3.3 compositing).
//
// Hits are grouped by primitive; one workgroup takes up to kHitsPerItem hits
// of one primitive, stages that primitive's packed weights in LDS once, and
// its four waves each walk a contiguous share of the hits' samples in blocks
// of 32 samples (matrix columns).  Per block: positional encoding straight
// into the B operand, the layer chain on the matrix cores with activations
// kept in registers, then the output activations and the hit-local front-to-
// back compositing (segmented scans across the block's columns, carried from
// block to block).  Only per-hit sums leave the kernel: the colour and
// feature sum with hit-local transmittance, and the hit's optical depth.  The
// per-ray compositor then chains the hits; a second launch of the same kernel
// ("fixup") re-evaluates the single hit in which a ray's transmittance falls
// below the threshold and cuts it at the exact sample.
#include "mlp_kernels.h"

namespace msplat {

namespace {

// ---------------------------------------------------------------- packing --

template <class N>
__global__ void pack_weights_kernel(const float* __restrict__ mlp, uint8_t* __restrict__ wpack,
                                    int64_t wpack_bytes, int P) {
  constexpr int NG16 = N::total_bytes() / 16;
  int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)P * NG16) return;
  int p = (int)(gid / NG16);
  int grp = (int)(gid % NG16);
  int byte = grp * 16;
  const float* th = mlp + (int64_t)p * N::n_params();
  uint8_t* dst = wpack + (int64_t)p * wpack_bytes + byte;
  float vals[8];
  int nv = 4;
  bool bf = false;
  // locate the section
  bool done = false;
#pragma unroll
  for (int j = 0; j < N::NL; ++j) {
    if (!done && byte >= N::fwdA_off(j) && byte < N::fwdA_off(j) + N::fwdA_bytes(j)) {
      int q = (byte - N::fwdA_off(j)) / 16;          // [rb][grp][lane]
      int lane = q % 64;
      int gi = (q / 64) % N::groups(N::fks(j));
      int rb = q / 64 / N::groups(N::fks(j));
      int n = 32 * rb + lane % 32;
      int g = lane / 32;
      if (N::BF16) {
        bf = true;
        nv = 8;
        for (int e = 0; e < 8; ++e) vals[e] = net_weight<N>(th, j, n, N::in_feat(j, g, 8 * gi + e));
      } else {
        for (int e = 0; e < 4; ++e) {
          int s = 4 * gi + e;
          vals[e] = s < N::fks(j) ? net_weight<N>(th, j, n, N::in_feat(j, g, s)) : 0.f;
        }
      }
      done = true;
    }
    if (!done && j > 0 && byte >= N::bias_off(j) && byte < N::bias_off(j) + N::bias_bytes(j)) {
      int fidx = (byte - N::bias_off(j)) / 4;        // [rb][g][16]
      for (int e = 0; e < 4; ++e) {
        int ff = fidx + e;
        int r = ff % 16, g = (ff / 16) % 2, rb = ff / 32;
        int n = phi_std(g, 16 * rb + r);
        vals[e] = n < N::fout(j) ? th[N::off_b(j) + n] : 0.f;
      }
      done = true;
    }
    if (!done && byte >= N::bwdA_off(j) && byte < N::bwdA_off(j) + N::bwdA_bytes(j)) {
      int q = (byte - N::bwdA_off(j)) / 16;
      int lane = q % 64;
      int gi = (q / 64) % N::groups(N::bks(j));
      int rb = q / 64 / N::groups(N::bks(j));
      int rho = 32 * rb + lane % 32;                  // input row in D layout
      int f;
      if (j == 0) {
        int gr, tr;
        phi_std_inv(rho, gr, tr);
        f = N::in_feat(0, gr, tr);
        if (f == N::IN) f = -1;                       // no gradient for the constant
      } else {
        f = rho < N::W ? rho : -1;
      }
      int g = lane / 32;
      if (N::BF16) {
        bf = true;
        nv = 8;
        for (int e = 0; e < 8; ++e) {
          int n = phi_std(g, 8 * gi + e);
          vals[e] = net_weight<N>(th, j, n, f);
        }
      } else {
        for (int e = 0; e < 4; ++e) {
          int s = 4 * gi + e;
          int n = phi_std(g, s);
          vals[e] = s < N::bks(j) ? net_weight<N>(th, j, n, f) : 0.f;
        }
      }
      done = true;
    }
  }
  if (bf) {
    bf16x8 v;
    for (int e = 0; e < 8; ++e) v[e] = (__bf16)vals[e];
    *reinterpret_cast<bf16x8*>(dst) = v;
  } else {
    f32x4 v;
    for (int e = 0; e < 4; ++e) v[e] = vals[e];
    *reinterpret_cast<f32x4*>(dst) = v;
  }
  (void)nv;
}

// full network of one 32-sample block; returns the output layer's D registers
template <class N>
__device__ __forceinline__ f32x16 forward_block(const uint8_t* __restrict__ lds, int lane, const float p[3]) {
  using BT = typename Operands<N>::BT;
  int g = lane / 32;
  float ev[N::ENC_KS * N::KSTEP];
  encode_slots<N>(p, g, ev);
  BT B0[rup(N::ENC_KS, N::KGRP)];
  if constexpr (N::BF16) {
#pragma unroll
    for (int s = 0; s < N::ENC_KS; ++s) {
      bf16x8 v;
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (__bf16)ev[8 * s + e];
      B0[s] = v;
    }
  } else {
#pragma unroll
    for (int s = 0; s < rup(N::ENC_KS, N::KGRP); ++s) B0[s] = s < N::ENC_KS ? ev[s] : 0.f;
  }
  f32x16 acc[N::RBH];
  layer_fwd<N, 0, N::ENC_KS>(lds, lane, B0, acc);
  BT Bh[rup(N::HID_KS, N::KGRP)];
#pragma unroll
  for (int j = 1; j < N::NL - 1; ++j) {
    relu_to_B<N>(acc, Bh);
    // J must be a compile-time constant: dispatch on j
    if (j == 1) layer_fwd<N, 1, N::HID_KS>(lds, lane, Bh, acc);
    if constexpr (N::NL - 1 > 2) if (j == 2) layer_fwd<N, (N::NL - 1 > 2 ? 2 : 1), N::HID_KS>(lds, lane, Bh, acc);
    if constexpr (N::NL - 1 > 3) if (j == 3) layer_fwd<N, (N::NL - 1 > 3 ? 3 : 1), N::HID_KS>(lds, lane, Bh, acc);
  }
  relu_to_B<N>(acc, Bh);
  f32x16 out[1];
  layer_fwd<N, N::NL - 1, N::HID_KS>(lds, lane, Bh, out);
  return out[0];
}

// ------------------------------------------------------------- forward --

struct FwdArgs {
  Workspace ws;
  msplat_opts opt;
  int mode;           // 0: all hits, hit-local sums; 1: fixup of cut hits
  int P;
  float* rgb;
  float* trans;
  float* feat;
};

template <class N>
__global__ __launch_bounds__(256) void mlp_forward_kernel(FwdArgs args) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  const Workspace& ws = args.ws;
  const int lane = threadIdx.x % 64;
  const int wv = threadIdx.x / 64;
  const int col = lane % 32;
  const int g = lane / 32;
  const int wi = blockIdx.x;
  const int p = find_prim(ws.wi_off, args.P, wi);
  const int first = ws.prim_off[p] + (wi - ws.wi_off[p]) * kHitsPerItem;
  const int nh = min(kHitsPerItem, ws.prim_off[p + 1] - first);
  const int64_t H = ws.hit_cap;
  if (args.mode == 1) {
    int flag = 0;
    if ((int)threadIdx.x < nh) flag = ws.hit_nused[ws.phit[first + threadIdx.x]] == -1;
    if (!__syncthreads_or(flag)) return;
  }
  // stage the primitive's packed forward operands
  {
    const uint4* src = reinterpret_cast<const uint4*>(ws.wpack + (int64_t)p * ws.wpack_bytes);
    uint4* dst = reinterpret_cast<uint4*>(lds);
    for (int i = threadIdx.x; i < N::fwd_bytes() / 16; i += blockDim.x) dst[i] = src[i];
  }
  __syncthreads();
  // this wave's hits
  const int h0 = (nh * wv) / 4, h1 = (nh * (wv + 1)) / 4;
  const int c = h1 - h0;
  int my_hit = 0, my_k = 0;
  if (lane < c) {
    my_hit = ws.phit[first + h0 + lane];
    int kk = ws.hit_k[my_hit] & kKMask;
    my_k = (args.mode == 0 || ws.hit_nused[my_hit] == -1) ? kk : 0;
  }
  int incl = wave_incl_scan(my_k);
  int my_off = incl - my_k;
  const int ns = __shfl(incl, 63, 64);
  const int nblk = (ns + 31) / 32;
  const uint32_t seed_hash = pcg_hash(args.opt.jitter_seed);
  const float t_stop = args.opt.t_stop;
  // carries between blocks (values of column 31 of the previous block)
  float cr_tau = 0.f, cr_tu = 0.f, cr_cnt = 0.f, cr_c[3] = {0.f, 0.f, 0.f};
  float cr_q[N::OUT_SLOTS];
#pragma unroll
  for (int r = 0; r < N::OUT_SLOTS; ++r) cr_q[r] = 0.f;

  for (int b = 0; b < nblk; ++b) {
    const int x = 32 * b + col;
    const bool valid = x < ns;
    int slot = 0;
    for (int l = 1; l < c; ++l)
      if (__shfl(my_off, l, 64) <= x) slot = l;
    const int hit = __shfl(my_hit, slot, 64);
    const int K = __shfl(my_k, slot, 64);
    const int k = valid ? x - __shfl(my_off, slot, 64) : 0;
    // sample position in the primitive's frame: p = p_c + (t_k - t_c) e
    const int ray = ws.hit_ray[hit];
    float u = 0.5f;
    if (args.opt.jitter) u = sample_offset(seed_hash, (uint32_t)ray, (uint32_t)(hit - ws.ray_off[ray]), (uint32_t)k);
    const float dlt = ws.hit_dlt[hit];
    const float sk = __builtin_fmaf((float)k + u, dlt, ws.hit_sa[hit]);
    float pl[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) pl[a] = __builtin_fmaf(sk, ws.hit_e[a * H + hit], ws.hit_pc[a * H + hit]);
    f32x16 o = forward_block<N>(lds, lane, pl);
    // density of the column (held by half 0), shared with half 1
    float tau0 = valid ? softplusf_(o[3]) * dlt : 0.f;
    const float tau = __shfl(tau0, col, 64);
    const bool head = (k == 0);
    SegScan sc(head, col);
    float tincl = sc.incl(tau);
    if (!sc.seen_head) tincl += cr_tau;
    float texcl = __shfl_up(tincl, 1, 32);
    if (head) texcl = 0.f;
    else if (col == 0) texcl = cr_tau;
    bool used = valid;
    float sb_hi = 0.f, sb_lo = 0.f;
    if (args.mode == 1) {
      sb_hi = ws.hit_sb_hi[hit];
      sb_lo = ws.hit_sb_lo[hit];
      used = valid && __expf(-(sb_hi + (sb_lo + texcl))) >= t_stop;
    }
    float alpha = -expm1f(-tau);
    float w = used ? __expf(-texcl) * alpha : 0.f;
    // colour sums (half 0) and feature sums (both halves)
    float cs[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      float v = sc.incl(w * sigmoidf_(o[r]));
      if (!sc.seen_head) v += cr_c[r];
      cs[r] = v;
    }
    float qs[N::OUT_SLOTS];
#pragma unroll
    for (int r = 0; r < N::OUT_SLOTS; ++r) {
      if constexpr (N::CF > 0) {
        float v = sc.incl(w * o[r]);
        if (!sc.seen_head) v += cr_q[r];
        qs[r] = v;
      } else {
        qs[r] = 0.f;
      }
    }
    float tu = 0.f, cnt = 0.f;
    if (args.mode == 1) {
      tu = sc.incl(used ? tau : 0.f);
      cnt = sc.incl(used ? 1.f : 0.f);
      if (!sc.seen_head) {
        tu += cr_tu;
        cnt += cr_cnt;
      }
    }
    // the lane holding a hit's last sample writes the hit's sums
    if (valid && k == K - 1) {
      if (args.mode == 0) {
        if (g == 0) {
          ws.hit_tau[hit] = tincl;
#pragma unroll
          for (int r = 0; r < 3; ++r) ws.hit_cloc[r * H + hit] = cs[r];
        }
#pragma unroll
        for (int r = 0; r < N::OUT_SLOTS; ++r) {
          int f = phi_std(g, r) - 4;
          if (N::CF > 0 && f >= 0 && f < N::CF) ws.hit_cloc[(3 + f) * H + hit] = qs[r];
        }
      } else {
        float tb = __expf(-(sb_hi + sb_lo));
        float tf = __expf(-(sb_hi + (sb_lo + tu)));
        if (g == 0) {
          ws.hit_tau[hit] = tu;
          ws.hit_nused[hit] = (int)cnt;
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            ws.hit_cloc[r * H + hit] = cs[r];
            args.rgb[3 * ray + r] += tb * cs[r] + tf * args.opt.background[r];
          }
          args.trans[ray] = tf;
          ws.ray_tf[ray] = tf;
        }
#pragma unroll
        for (int r = 0; r < N::OUT_SLOTS; ++r) {
          int f = phi_std(g, r) - 4;
          if (N::CF > 0 && f >= 0 && f < N::CF) {
            ws.hit_cloc[(3 + f) * H + hit] = qs[r];
            args.feat[(int64_t)ray * N::CF + f] += tb * qs[r];
          }
        }
      }
    }
    // carry column 31 into the next block
    cr_tau = __shfl(tincl, 31, 32);
    cr_tu = __shfl(tu, 31, 32);
    cr_cnt = __shfl(cnt, 31, 32);
#pragma unroll
    for (int r = 0; r < 3; ++r) cr_c[r] = __shfl(cs[r], 31, 32);
#pragma unroll
    for (int r = 0; r < N::OUT_SLOTS; ++r) cr_q[r] = __shfl(qs[r], 31, 32);
  }
}

}  // namespace

// ------------------------------------------------------------ dispatch --

template <class N>
static hipError_t pack_impl(const Workspace& ws, const float* mlp, int P, hipStream_t s) {
  int64_t n = (int64_t)P * (N::total_bytes() / 16);
  hipLaunchKernelGGL(pack_weights_kernel<N>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, mlp,
                     ws.wpack, ws.wpack_bytes, P);
  return hipGetLastError();
}

template <class N>
static hipError_t fwd_impl(const Workspace& ws, const msplat_opts& o, int items, int mode, int P,
                           float* rgb, float* trans, float* feat, hipStream_t s) {
  if (items <= 0) return hipSuccess;
  FwdArgs a{ws, o, mode, P, rgb, trans, feat};
  size_t lds = N::fwd_bytes();
  hipLaunchKernelGGL(mlp_forward_kernel<N>, dim3(items), dim3(256), lds, s, a);
  return hipGetLastError();
}

#define MSPLAT_NETS(X)                 \
  X(4, 32, 2, 4, false)                \
  X(4, 32, 2, 4, true)                 \
  X(6, 64, 3, 4, false)                \
  X(6, 64, 3, 4, true)                 \
  X(6, 64, 3, 20, false)               \
  X(6, 64, 3, 20, true)

#define MSPLAT_MATCH(L_, W_, D_, O_, B_) \
  if (n.L == L_ && n.W == W_ && n.D == D_ && n.NOUT == O_ && (n.prec == MSPLAT_BF16) == B_)

bool mlp_supported(const NetShape& n) {
#define X(L_, W_, D_, O_, B_) MSPLAT_MATCH(L_, W_, D_, O_, B_) return true;
  MSPLAT_NETS(X)
#undef X
  return false;
}

int64_t mlp_wpack_bytes(const NetShape& n) {
#define X(L_, W_, D_, O_, B_) MSPLAT_MATCH(L_, W_, D_, O_, B_) return Net<L_, W_, D_, O_, B_>::total_bytes();
  MSPLAT_NETS(X)
#undef X
  return 0;
}

hipError_t launch_pack_weights(const NetShape& n, const Workspace& ws, const float* mlp, hipStream_t s) {
#define X(L_, W_, D_, O_, B_) MSPLAT_MATCH(L_, W_, D_, O_, B_) return pack_impl<Net<L_, W_, D_, O_, B_>>(ws, mlp, n.P, s);
  MSPLAT_NETS(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_mlp_forward(const NetShape& n, const Workspace& ws, const msplat_opts& o, int items,
                              int mode, float* rgb, float* trans, float* feat, hipStream_t s) {
#define X(L_, W_, D_, O_, B_) \
  MSPLAT_MATCH(L_, W_, D_, O_, B_) return fwd_impl<Net<L_, W_, D_, O_, B_>>(ws, o, items, mode, n.P, rgb, trans, feat, s);
  MSPLAT_NETS(X)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace msplat
