// Grouped per-primitive MLP kernels (Sec. 3.2 network, Sec. 3.3 compositing).
//
// Hits are grouped by primitive; one workgroup takes a run of consecutive
// hits of one primitive's list (items_per_group work items of hits_per_item
// hits, at most 64 per wave), stages that primitive's packed weights in LDS
// once (wide networks read them from L2), and its waves (eight; four for
// wide networks) each walk the samples of their hits (dealt by sample count)
// in blocks of 32 samples (matrix columns).  Per block: positional encoding straight
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
  int byte = (int)(gid % NG16) * 16;
  const float* th = mlp + (int64_t)p * N::n_params();
  uint8_t* dst = wpack + (int64_t)p * wpack_bytes + byte;
  float vals[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  bool is_bias = false;
  int part = 0;   // 0: value (or hi part), 1: lo part of a split operand
#pragma unroll
  for (int j = 0; j < N::NL; ++j) {
    const bool in_f = byte >= N::fwdA_off(j) && byte < N::fwdA_off(j) + N::fwdA_bytes(j);
    const bool in_b = byte >= N::bwdA_off(j) && byte < N::bwdA_off(j) + N::bwdA_bytes(j);
    if (in_f || in_b) {
      const int single = in_f ? N::fwdA_single(j) : N::bwdA_single(j);
      const int rel = byte - (in_f ? N::fwdA_off(j) : N::bwdA_off(j));
      part = rel / single;
      const int q = (rel % single) / 16;          // [rb][group][lane]
      const int ng = N::groups(in_f ? N::fks(j) : N::bks(j));
      const int nk = in_f ? N::fks(j) : N::bks(j);
      const int lane = q % 64, gi = (q / 64) % ng, rb = q / 64 / ng;
      const int g = lane / 32;
      int f_row = -1;
      if (in_b) {                                  // transposed: rows are input features
        int rho = 32 * rb + lane % 32;
        if (j == 0) {
          int gr, tr;
          phi_std_inv(rho, gr, tr);
          f_row = N::in_feat(0, gr, tr);
          if (f_row == N::IN) f_row = -1;          // no gradient for the constant
        } else {
          f_row = rho < N::W ? rho : -1;
        }
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        if (!N::BF16 && e >= 4) break;
        const int t = N::BF16 ? 8 * gi + e : 4 * gi + e;       // slot of lane half g
        const int s = N::BF16 ? gi : t;                        // k-step
        if (s >= nk) continue;
        vals[e] = in_f ? net_weight<N>(th, j, 32 * rb + lane % 32, N::in_feat(j, g, t))
                       : net_weight<N>(th, j, phi_std(g, t), f_row);
      }
    }
    if (j > 0 && byte >= N::bias_off(j) && byte < N::bias_off(j) + N::bias_bytes(j)) {
      is_bias = true;
      const int fidx = (byte - N::bias_off(j)) / 4;            // [rb][g][16]
      for (int e = 0; e < 4; ++e) {
        int ff = fidx + e;
        int r = ff % 16, g = (ff / 16) % 2, rb = ff / 32;
        int n = phi_std(g, 16 * rb + r);
        vals[e] = n < N::fout(j) ? th[N::off_b(j) + n] : 0.f;
      }
    }
  }
  if (N::BF16 && !is_bias) {
    bf16x8 v;
    for (int e = 0; e < 8; ++e) {
      __bf16 h = (__bf16)vals[e];
      v[e] = part == 0 ? h : (__bf16)(vals[e] - (float)h);
    }
    *reinterpret_cast<bf16x8*>(dst) = v;
  } else {
    f32x4 v;
    for (int e = 0; e < 4; ++e) v[e] = vals[e];
    *reinterpret_cast<f32x4*>(dst) = v;
  }
}

// full network of one 32-sample block; returns the output layer's D registers
template <class N, int J, int LAYOUT>
__device__ __forceinline__ f32x16 hidden_chain(const uint8_t* __restrict__ wb, const uint8_t* __restrict__ wlo,
                                               int lane, f32x16 (&acc)[N::RBH]) {
  Act<N, rup(N::HID_KS, N::KGRP)> Bh;
  relu_to_B<N>(acc, Bh);
  if constexpr (J < N::NL - 1) {
    layer_fwd<N, J, N::HID_KS, LAYOUT>(wb, wlo, lane, Bh, acc);
    return hidden_chain<N, J + 1, LAYOUT>(wb, wlo, lane, acc);
  } else {
    f32x16 out[1];
    layer_fwd<N, J, N::HID_KS, LAYOUT>(wb, wlo, lane, Bh, out);
    return out[0];
  }
}

template <class N, int LAYOUT>
__device__ __forceinline__ f32x16 forward_block(const uint8_t* __restrict__ wb, const uint8_t* __restrict__ wlo,
                                                int lane, const float ph[3], const float pl[3], const float dd[3]) {
  int g = lane / 32;
  float ev[N::ENC_KS * N::KSTEP];
  encode_input<N>(ph, pl, dd, g, ev);
  Act<N, rup(N::ENC_KS, N::KGRP)> B0;
  enc_to_B<N>(ev, B0);
  f32x16 acc[N::RBH];
  // matrix-core stretch: issue ahead of the other waves' vector work
  mfma_priority<N, 1>();
  layer_fwd<N, 0, N::ENC_KS, LAYOUT>(wb, wlo, lane, B0, acc);
  const f32x16 o = hidden_chain<N, 1, LAYOUT>(wb, wlo, lane, acc);
  mfma_priority<N, 0>();
  return o;
}

// How the forward kernel reads a primitive's operands: 1, all staged in LDS
// (networks up to 64 wide, and wider plain-BF16 ones, whose operands fit);
// 2, the split form's hi sections and biases staged in LDS and the lo
// sections read from L2 (wide split networks: both halves do not fit);
// 0, everything from L2 (wide FP32).
constexpr int kFwdLdsMax = 160 * 1024;
template <class N>
constexpr int fwd_stage() {
  return N::fwd_bytes() <= kFwdLdsMax ? 1 : ((N::SPLIT && N::fwd_hi_bytes() <= kFwdLdsMax) ? 2 : 0);
}
template <class N>
constexpr int fwd_staged_bytes() {
  return fwd_stage<N>() == 1 ? N::fwd_bytes() : (fwd_stage<N>() == 2 ? N::fwd_hi_bytes() : 0);
}

// ------------------------------------------------------------- forward --

struct FwdArgs {
  Workspace ws;
  msplat_opts opt;
  int mode;           // 0: all hits, hit-local sums; 1: fixup of cut hits
  int P;
  int ghits;          // hits per workgroup (a run of one primitive's list), <= 64 per wave
  float* rgb;
  float* trans;
  float* feat;
};

// waves per workgroup: eight for networks whose weights are staged in LDS
// (one copy serves eight waves, and LDS then admits two workgroups, four
// waves per SIMD), four for wide networks
template <class N>
constexpr int fwd_waves() { return N::WIDE ? 4 : 8; }
// waves per SIMD the register allocation must leave room for (two
// workgroups of eight; wide networks take the whole register file)
template <class N>
constexpr int fwd_min_waves() { return N::WIDE ? 1 : 4; }
// LDS: the staged operands, then the deal table (64 ints per wave)
template <class N>
constexpr int fwd_deal_off() { return (fwd_staged_bytes<N>() + 15) / 16 * 16; }
template <class N>
constexpr int fwd_lds_bytes() { return fwd_deal_off<N>() + 256 * fwd_waves<N>(); }

template <class N>
__global__ __launch_bounds__(64 * fwd_waves<N>(), fwd_min_waves<N>()) void mlp_forward_kernel(FwdArgs args) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  const Workspace& ws = args.ws;
  const int lane = threadIdx.x % 64;
  const int wv = threadIdx.x / 64;
  const int col = lane % 32;
  const int g = lane / 32;
  // a run of up to args.ghits consecutive hits of one primitive's list
  const int bid = blockIdx.x;
  if (bid >= ws.gw_off[args.P]) return;   // (the grid is an upper bound)
  const int p = find_prim(ws.gw_off, args.P, bid);
  const int first = ws.prim_off[p] + (bid - ws.gw_off[p]) * args.ghits;
  const int nh = min(args.ghits, ws.prim_off[p + 1] - first);
  const int64_t H = ws.hit_cap;
  if (args.mode == 1) {
    int flag = 0;
    if ((int)threadIdx.x < nh) flag = ws.hit_nused[ws.phit[first + threadIdx.x]] == -1;
    if (!__syncthreads_or(flag)) return;
  }
  // the primitive's packed forward operands, staged in LDS as fwd_stage says
  const uint8_t* wglb = ws.wpack + (int64_t)p * ws.wpack_bytes;
  const uint8_t* wts = wglb;
  if constexpr (fwd_stage<N>() == 1) {
    const uint4* src = reinterpret_cast<const uint4*>(wglb);
    uint4* dst = reinterpret_cast<uint4*>(lds);
    for (int i = threadIdx.x; i < N::fwd_bytes() / 16; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
    wts = lds;
  } else if constexpr (fwd_stage<N>() == 2) {
    // each layer's hi section, then the biases
    uint4* dst = reinterpret_cast<uint4*>(lds);
#pragma unroll
    for (int j = 0; j < N::NL; ++j) {
      const uint4* src = reinterpret_cast<const uint4*>(wglb + N::fwdA_off(j));
      for (int i = threadIdx.x; i < N::fwdA_single(j) / 16; i += blockDim.x) dst[N::fwd_hi_off(j) / 16 + i] = src[i];
    }
    const uint4* srcb = reinterpret_cast<const uint4*>(wglb + N::bias_off(0));
    for (int i = threadIdx.x; i < (N::fwd_bytes() - N::bias_off(0)) / 16; i += blockDim.x)
      dst[N::fwd_hi_off(N::NL) / 16 + i] = srcb[i];
    __syncthreads();
    wts = lds;
  }
  // this wave's hits: the run dealt to the waves (the fixup takes the cut
  // hits only)
  constexpr int NWF = fwd_waves<N>();
  int my_k, li;
  {
    const int idx = 64 * wv + lane;
    int key = -1;
    if (idx < nh) {
      const int h = ws.phit[first + idx];
      const int kk = ws.hit_k[h] & kKMask;
      key = ((args.mode == 0 || ws.hit_nused[h] == -1 ? kk : 0) << 9) | (511 - idx);
    }
    li = deal_run<NWF>(key, reinterpret_cast<int*>(lds + fwd_deal_off<N>()), wv, lane, my_k);
  }
  const int my_hit = li < 0 ? 0 : ws.phit[first + li];
  // the hit's ray and its slot along the ray (for the sample offsets), read
  // once here rather than per block
  int my_ray = 0, my_slot = 0;
  if (li >= 0) {
    my_ray = ws.hit_ray[my_hit];
    my_slot = my_hit - ws.ray_off[my_ray];
  }
  const int c = __popcll(__ballot(li >= 0));   // (the wave's hits fill lanes 0..c-1)
  int incl = wave_incl_scan(my_k);
  int my_off = incl - my_k;
  const int ns = __builtin_amdgcn_readlane(incl, 63);
  const int nblk = (ns + 31) / 32;
  const uint32_t seed_hash = pcg_hash(args.opt.jitter_seed);
  const float t_stop = args.opt.t_stop;
  // carries between blocks (values of column 31 of the previous block)
  float cr_tau = 0.f, cr_tu = 0.f, cr_cnt = 0.f, cr_c[3] = {0.f, 0.f, 0.f};
  float cr_q[N::OUT_SLOTS];
#pragma unroll
  for (int r = 0; r < N::OUT_SLOTS; ++r) cr_q[r] = 0.f;

  int lb = 0;   // (scalar) lane of the hit holding the block's first column
  for (int b = 0; b < nblk; ++b) {
    const int x = 32 * b + col;
    const bool valid = x < ns;
    // the hit of this column: the last of the wave's hits whose samples
    // start at or before it (hit records read from lanes into scalar
    // registers).  The hits sit in lanes 0..c-1 in sample order: the cursor
    // lb moves to the hit holding the block's first column, then the hits
    // starting inside the block are taken.
    const int x0 = 32 * b;
    while (lb + 1 < c && __builtin_amdgcn_readlane(my_off, lb + 1) <= x0) ++lb;
    int hit = __builtin_amdgcn_readlane(my_hit, lb), K = __builtin_amdgcn_readlane(my_k, lb);
    int hoff = __builtin_amdgcn_readlane(my_off, lb);
    int ray = __builtin_amdgcn_readlane(my_ray, lb), slot = __builtin_amdgcn_readlane(my_slot, lb);
    for (int l = lb + 1; l < c; ++l) {
      const int ol = __builtin_amdgcn_readlane(my_off, l);
      if (ol >= x0 + 32) break;
      if (ol <= x) {
        hit = __builtin_amdgcn_readlane(my_hit, l);
        K = __builtin_amdgcn_readlane(my_k, l);
        hoff = ol;
        ray = __builtin_amdgcn_readlane(my_ray, l);
        slot = __builtin_amdgcn_readlane(my_slot, l);
      }
    }
    const int k = valid ? x - hoff : 0;
    // sample position in the primitive's frame: p = p_c + (t_k - t_c) e
    float u = 0.5f;
    if (args.opt.jitter) u = sample_offset(seed_hash, (uint32_t)ray, (uint32_t)slot, (uint32_t)k);
    const float dlt = ws.hit_dlt[hit];
    float ph[3], pl[3], dd[3];
    sample_input<N>(ws, hit, k, u, ph, pl, dd);
    f32x16 o = forward_block<N, fwd_stage<N>() == 2 ? kHiStaged : kPacked>(wts, wglb, lane, ph, pl, dd);
    // density of the column (held by half 0), shared with half 1
    float tau0 = valid ? softplusf_(o[3]) * dlt : 0.f;
    const float tau = from_lower_half(tau0);
    const bool head = (k == 0);
    SegScan sc(head, col);
    float tincl = sc.incl(tau);
    if (!sc.seen_head) tincl += cr_tau;
    float texcl = col_below(tincl, col);
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
    // (the optical depths are the same in both halves; colour and feature
    // sums are per half)
    cr_tau = col31_same(tincl);
    cr_tu = col31_same(tu);
    cr_cnt = col31_same(cnt);
#pragma unroll
    for (int r = 0; r < 3; ++r) cr_c[r] = col31(cs[r], g);
#pragma unroll
    for (int r = 0; r < N::OUT_SLOTS; ++r) cr_q[r] = col31(qs[r], g);
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
static hipError_t fwd_impl(const Workspace& ws, const msplat_opts& o, int64_t num_hits, int group, int mode,
                           int P, float* rgb, float* trans, float* feat, hipStream_t s) {
  if (num_hits <= 0) return hipSuccess;
  if (group < 1 || ws.hits_per_item < 1) return hipErrorInvalidValue;
  static_assert(fwd_lds_bytes<N>() <= kFwdLdsMax, "LDS budget of one workgroup");
  // a workgroup's run: `group` work items, at most 64 hits per wave
  const int ghits = min(group * ws.hits_per_item, 64 * fwd_waves<N>());
  FwdArgs a{ws, o, mode, P, ghits, rgb, trans, feat};
  if (mode == 0) {   // (the fixup pass reuses the offsets of the full pass)
    hipError_t e = launch_group_scan(ws, P, ghits, s);
    if (e != hipSuccess) return e;
  }
  size_t lds = fwd_lds_bytes<N>();
  if (lds > 64 * 1024) {
    static bool attr = false;   // (per network type)
    if (!attr) {
      hipError_t e = hipFuncSetAttribute((const void*)mlp_forward_kernel<N>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      attr = true;
    }
  }
  // at most ceil(hits / ghits) runs plus one partial run per primitive; the
  // workgroups past the last run return at once
  const int64_t groups = (num_hits + ghits - 1) / ghits + P;
  hipLaunchKernelGGL(mlp_forward_kernel<N>, dim3((unsigned)groups), dim3(64 * fwd_waves<N>()), lds, s, a);
  return hipGetLastError();
}

#ifndef MSPLAT_WIDE_TU
bool mlp_supported(const NetShape& n) {
#define X(L_, W_, D_, O_, P_, K_) MSPLAT_MATCH(L_, W_, D_, O_, P_, K_) return true;
  MSPLAT_NETS(X)
#undef X
  return false;
}

int64_t mlp_wpack_bytes(const NetShape& n) {
#define X(L_, W_, D_, O_, P_, K_) MSPLAT_MATCH(L_, W_, D_, O_, P_, K_) return MSPLAT_NET(L_, W_, D_, O_, P_, K_)::total_bytes();
  MSPLAT_NETS(X)
#undef X
  return 0;
}

hipError_t launch_pack_weights_wide(const NetShape& n, const Workspace& ws, const float* mlp, hipStream_t s);
hipError_t launch_mlp_forward_wide(const NetShape& n, const Workspace& ws, const msplat_opts& o, int64_t num_hits,
                                   int group, int mode, float* rgb, float* trans, float* feat, hipStream_t s);
hipError_t launch_pack_weights_narrow(const NetShape& n, const Workspace& ws, const float* mlp, hipStream_t s);
hipError_t launch_mlp_forward_narrow(const NetShape& n, const Workspace& ws, const msplat_opts& o,
                                     int64_t num_hits, int group, int mode, float* rgb, float* trans, float* feat,
                                     hipStream_t s);

hipError_t launch_pack_weights(const NetShape& n, const Workspace& ws, const float* mlp, hipStream_t s) {
  return wide_net(n.W) ? launch_pack_weights_wide(n, ws, mlp, s) : launch_pack_weights_narrow(n, ws, mlp, s);
}

hipError_t launch_mlp_forward(const NetShape& n, const Workspace& ws, const msplat_opts& o, int64_t num_hits,
                              int group, int mode, float* rgb, float* trans, float* feat, hipStream_t s) {
  return wide_net(n.W) ? launch_mlp_forward_wide(n, ws, o, num_hits, group, mode, rgb, trans, feat, s)
                       : launch_mlp_forward_narrow(n, ws, o, num_hits, group, mode, rgb, trans, feat, s);
}
#endif

hipError_t MSPLAT_TU_FN(launch_pack_weights)(const NetShape& n, const Workspace& ws, const float* mlp,
                                             hipStream_t s) {
#define X(L_, W_, D_, O_, P_, K_) MSPLAT_MATCH(L_, W_, D_, O_, P_, K_) return pack_impl<MSPLAT_NET(L_, W_, D_, O_, P_, K_)>(ws, mlp, n.P, s);
  MSPLAT_TU_NETS(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t MSPLAT_TU_FN(launch_mlp_forward)(const NetShape& n, const Workspace& ws, const msplat_opts& o,
                                            int64_t num_hits, int group, int mode, float* rgb, float* trans,
                                            float* feat, hipStream_t s) {
#define X(L_, W_, D_, O_, P_, K_)                                                                     \
  MSPLAT_MATCH(L_, W_, D_, O_, P_, K_)                                                                \
  return fwd_impl<MSPLAT_NET(L_, W_, D_, O_, P_, K_)>(ws, o, num_hits, group, mode, n.P, rgb, trans, feat, s);
  MSPLAT_TU_NETS(X)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace msplat
