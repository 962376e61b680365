// Fused adjoint of the per-primitive MLP, of the hit-local compositing and of
// the sample geometry (the paper prints no backward; this is the exact
// derivative of the forward in mlp.hip with the discrete decisions fixed).
//
// Work decomposition as in the forward: one workgroup per run of up to 64
// hits per wave of one primitive's list, its operands (forward and
// transposed) staged in LDS as far as they fit beside the exchange planes,
// the run dealt to the waves by sample count, each wave walking its hits'
// samples in 32-column blocks.
// Per block the wave
//   1. recomputes the network, keeping the hi parts of the layer inputs in
//      registers (nothing is stored to memory between forward and backward);
//   2. forms dL/d(raw outputs) from the compositing adjoint: with per-hit
//      transmittance T_b, suffix g.S_after and total g.(hit colour) from the
//      per-ray adjoint, dtau_k = T_{k+1} g.c_k - sum_{j>k} w_j g.c_j - g.S_after;
//   3. runs the transposed chain delta_{j-1} = W_j^T delta_j * relu' on the
//      matrix cores, registers to registers;
//   4. reduces the sample-position adjoints of its samples into per-hit sums
//      (segmented scans), which the hit's last sample stores; a kernel of its
//      own (geometry.hip) chains them through the contact point, the chord
//      and the frame M = diag(s)^-1 R^T.
// Weight gradients are contractions over samples: the waves of a workgroup
// publish delta_j and the layer inputs of their blocks to LDS, then each wave
// accumulates its units of dW_j (a 16-row strip by a few 16-column tiles)
// over all the workgroup's samples in registers.  Those sums are added to
// global memory once per workgroup.
#include "mlp_kernels.h"

namespace msplat {

namespace {

template <class N>
struct Bwd {
  static constexpr int mx(int a, int b) { return a > b ? a : b; }
  static constexpr int ESZ = N::BF16 ? 2 : 4;       // exchange element bytes
  static constexpr int HROWS = mx(rup(N::IN + 1, 16), rup(N::W, 16));
  static constexpr int DROWS = mx(rup(N::W, 16), rup(N::NOUT, 16));
  // The split form contracts the weight gradient from the hi parts of both
  // operands (delta and layer input), one product per pair: a single rounding
  // of each factor, not compounded through the chain, keeps dW within about
  // 6e-4 of the FP64 result at the sizes tested; the transposed chain keeps
  // all three products.  (true: also delta_lo x_hi, with its own LDS plane.)
  // The contact-point primitive has one sample per hit, so a weight-gradient
  // entry sums few samples and their roundings do not average out: its
  // (small) networks contract all three products, delta hi x input hi, delta
  // lo x input hi and delta hi x input lo, with planes for both lo parts.
  static constexpr bool DWS = N::SPLIT && N::CONTACT;
  static constexpr bool DWX = N::SPLIT && N::CONTACT;
  // exchange planes of nw waves (32 samples each; rows padded by 16 bytes,
  // which keeps the 16-row operand reads free of bank conflicts): layer
  // inputs (the split form contracts the weight gradient with their hi part
  // only), deltas (hi), and the deltas' lo parts
  static constexpr int xsp(int nw) { return 32 * nw + (N::BF16 ? 8 : 4); }
  static constexpr int planes(int nw) { return (HROWS * (DWX ? 2 : 1) + DROWS * (DWS ? 2 : 1)) * xsp(nw) * ESZ; }
  // Weights staged in LDS beside the planes.  Where they do not all fit, the
  // first layer's forward operands (requested ahead of the encoding, which
  // covers their latency) are read from global memory instead, L2-resident
  // while a primitive's work items run; wide networks read there all but the
  // hi sections staged for their recompute (HS below).
  static constexpr int LDS_MAX = 160 * 1024 - 256;   // (less the static arrays)
  static constexpr int staged(int nw, int skip) { return rup(planes(nw), 256) + N::total_bytes() - skip; }
  // Waves per workgroup.  The bfloat16 forms of networks up to 64 wide run
  // eight where their weights fit beside eight waves' planes (two waves per
  // SIMD sharing one LDS copy of the weights, so that one wave's LDS and
  // barrier waits overlap the other's work); otherwise four; the float32
  // form (whose exchange planes are twice as wide) two.
  static constexpr bool FIT8 = N::BF16 && !N::WIDE && staged(8, N::fwdA_bytes(0)) <= LDS_MAX;
  static constexpr int NW = N::BF16 ? (FIT8 ? 8 : 4) : 2;
  static constexpr int XS = 32 * NW;                // samples per exchange round
  static constexpr int XSP = xsp(NW);               // padded row (elements)
  // plane offsets: at the bottom of LDS, where (up to 64 KiB) an access is a
  // base register plus an immediate offset; the staged weights follow
  static constexpr int XH_OFF = 0;
  static constexpr int XD_OFF = XH_OFF + HROWS * XSP * ESZ;
  static constexpr int XDL_OFF = XD_OFF + DROWS * XSP * ESZ;                   // lo parts (split form)
  static constexpr int XHL_OFF = XDL_OFF + (DWS ? DROWS * XSP * ESZ : 0);      // inputs' lo parts
  static constexpr int PLANES = planes(NW);
  static constexpr int W_OFF = rup(PLANES, 256);
  static constexpr bool G0 = !N::WIDE && staged(NW, 0) > LDS_MAX;
  static constexpr int SKIP = G0 ? N::fwdA_bytes(0) : 0;   // = fwdA_off(1): staged from here
  static constexpr bool GW = N::WIDE || staged(NW, SKIP) > LDS_MAX;
  // Wide bfloat16 networks: the hi sections of the forward operands of the
  // first HS layers (as many as fit) are staged beside the planes; the
  // recompute reads them there (read in both passes, by every block), the
  // rest from global memory.
  static constexpr int hs_fit(int s) { return s < N::NL && W_OFF + N::fwd_hi_off(s + 1) <= LDS_MAX ? hs_fit(s + 1) : s; }
  static constexpr int HS = N::WIDE && N::BF16 ? hs_fit(0) : 0;
  static constexpr int FL = HS > 0 ? kHiPrefix + HS : kPacked;   // the recompute's operand layout
  static constexpr int LDS = GW ? (HS > 0 ? W_OFF + N::fwd_hi_off(HS) : PLANES) : staged(NW, SKIP);
  static_assert(LDS <= 160 * 1024, "LDS budget of one workgroup");
  // weight-gradient tiles (16 x 16) of layer j
  static constexpr int inp(int j) { return j == 0 ? N::IN + 1 : N::W; }
  static constexpr int RT(int j) { return (N::fout(j) + 15) / 16; }
  static constexpr int CT(int j) { return (inp(j) + 15) / 16; }
  static constexpr int CTB(int j) { return CT(j) + (j > 0 ? 1 : 0); }
  // ownership: the tiles of layer j are cut into units of one row tile and
  // CPG(j) consecutive column tiles (CG(j) units per row tile, enough for
  // every wave to own one where the layer has fewer row tiles than waves);
  // wave q owns units q, q + NW, ...
  static constexpr int mn(int a, int b) { return a < b ? a : b; }
  static constexpr int CG(int j) { return mn(CTB(j), (NW + RT(j) - 1) / RT(j)); }
  static constexpr int CPG(int j) { return (CTB(j) + CG(j) - 1) / CG(j); }
  static constexpr int UNITS(int j) { return RT(j) * CG(j); }
  static constexpr int OWN(int j) { return (UNITS(j) + NW - 1) / NW; }
  static constexpr int TOFF(int j) { return j == 0 ? 0 : TOFF(j - 1) + OWN(j - 1) * CPG(j - 1); }
  static constexpr int TT = TOFF(N::NL);
  // a pass accumulates the weight gradients of layers LO..HI
  static constexpr int tiles(int lo, int hi) { return TOFF(hi + 1) - TOFF(lo); }
  static constexpr int toff(int lo, int j) { return TOFF(j) - TOFF(lo); }
};


// D registers -> B operand (no activation), first NSLOT slots
template <class N, int NSLOT, int RB>
__device__ __forceinline__ void d_to_B(const f32x16 (&acc)[RB],
                                       Act<N, rup(rup(NSLOT, N::KSTEP) / N::KSTEP, N::KGRP)>& B) {
  constexpr int KS = rup(NSLOT, N::KSTEP) / N::KSTEP;
  act_fill<N, rup(KS, N::KGRP)>(B, [&](int t) { return t < NSLOT ? acc[t / 16][t % 16] : 0.f; });
}

// transposed layer: out[rb] = W_j^T delta (rows = input slots of layer j),
// with the next row block's operands requested ahead as in layer_fwd
template <class N, int J>
__device__ __forceinline__ void layer_bwd(const uint8_t* __restrict__ wb, int lane,
                                          const Act<N, rup(N::bks(J), N::KGRP)>& B,
                                          f32x16 (&acc)[N::brb(J)]) {
  constexpr int RB = N::brb(J);
  constexpr int NG = N::groups(N::bks(J));
  const uint8_t* A = wb + N::bwdA_off(J);
  RowOps<N, NG, false> ops[2];
  load_row<N, NG, false>(A, A + N::bwdA_single(J), nullptr, 0, lane, ops[0]);
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    if (rb + 1 < RB) load_row<N, NG, false>(A, A + N::bwdA_single(J), nullptr, rb + 1, lane, ops[(rb + 1) & 1]);
    f32x16 c;
#pragma unroll
    for (int e = 0; e < 16; ++e) c[e] = 0.f;
    row_mfma<N, NG, false>(ops[rb & 1], B, c);
    acc[rb] = c;
    __builtin_amdgcn_sched_barrier(0);
  }
}

// publish this wave's 32 columns of a layer input (slots -> canonical rows)
template <class N, int J, int NKS, bool LO = false>
__device__ __forceinline__ void publish_input(uint8_t* __restrict__ lds, const Hi<N, NKS>& a, int g,
                                              int colx) {
  using B = Bwd<N>;
  constexpr int OFF = LO ? B::XHL_OFF : B::XH_OFF;
#pragma unroll
  for (int s = 0; s < NKS; ++s) {
#pragma unroll
    for (int e = 0; e < N::KSTEP; ++e) {
      int t = N::KSTEP * s + e;
      if (N::BF16 ? (t >= (J == 0 ? N::ENC_KS * 8 : N::HID_KS * 8)) : (s >= (J == 0 ? N::ENC_KS : N::HID_KS)))
        continue;
      int f = N::in_feat(J, g, t);
      if (f < 0) continue;
      if constexpr (N::BF16) {
        reinterpret_cast<__bf16*>(lds + OFF)[f * B::XSP + colx] = a.hi[s][e];
      } else {
        reinterpret_cast<float*>(lds + B::XH_OFF)[f * B::XSP + colx] = a.hi[s];
      }
    }
  }
}

// publish this wave's 32 columns of delta_j (D layout -> canonical rows); the
// deltas of columns past the end of the wave's samples are zero.  The
// bfloat16 forms publish the operand already converted for the transposed
// product (hi, and lo in the split form).
template <class N, int J, int NK>
__device__ __forceinline__ void publish_delta(uint8_t* __restrict__ lds, const f32x16 (&dz)[N::frb(J)],
                                              const Act<N, NK>& bd, int g, int colx) {
  using B = Bwd<N>;
#pragma unroll
  for (int rb = 0; rb < N::frb(J); ++rb) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int t = 16 * rb + r;
      const int n = phi_std(g, t);
      if (n >= N::fout(J)) continue;
      if constexpr (N::BF16) {
        if (t / 8 >= NK) continue;   // (rows past the operand's slots are padding)
        reinterpret_cast<__bf16*>(lds + B::XD_OFF)[n * B::XSP + colx] = bd.hi[t / 8][t % 8];
        if constexpr (B::DWS)
          reinterpret_cast<__bf16*>(lds + B::XDL_OFF)[n * B::XSP + colx] = bd.lo[t / 8][t % 8];
      } else {
        reinterpret_cast<float*>(lds + B::XD_OFF)[n * B::XSP + colx] = dz[rb][r];
      }
    }
  }
}

// bfloat16 forms: accumulate one unit of dW_J (and db_J) over the round, row
// tile rt (wave-uniform) by the column tiles [C0, C0 + CPG).  C0 is a
// compile-time constant, so which tiles are inputs, which one is the bias
// (ones) and which lie past the layer is fixed per instantiation: no branch
// inside the k-step loop, every LDS address the lane's offset plus constants.
template <class N, int J, int C0>
__device__ __forceinline__ void dw_unit(const uint8_t* __restrict__ lds, f32x4* __restrict__ acc, int rt,
                                        int lane) {
  using B = Bwd<N>;
  constexpr int CPG = B::CPG(J);
  const int r16 = lane % 16, kg = lane / 16;
  const int lo16 = r16 * B::XSP + 8 * kg;
  const __bf16* pd = reinterpret_cast<const __bf16*>(lds + B::XD_OFF) + 16 * rt * B::XSP + lo16;
  const __bf16* pdl = reinterpret_cast<const __bf16*>(lds + B::XDL_OFF) + 16 * rt * B::XSP + lo16;
  const __bf16* px = reinterpret_cast<const __bf16*>(lds + B::XH_OFF) + 16 * C0 * B::XSP + lo16;
  const __bf16* pxl = reinterpret_cast<const __bf16*>(lds + B::XHL_OFF) + 16 * C0 * B::XSP + lo16;
  bf16x8 ones;
#pragma unroll
  for (int e = 0; e < 8; ++e) ones[e] = (__bf16)(r16 == 0 ? 1.f : 0.f);
  // operands of one 32-sample k-step: delta row strip (hi, lo) and the
  // unit's input tiles; the next k-step's are requested before this one's
  // products
  struct KOps {
    bf16x8 a, al, b[CPG], bl[B::DWX ? CPG : 1];
  };
  auto load = [&](int kk, KOps& o) {
    o.a = *reinterpret_cast<const bf16x8*>(pd + 32 * kk);
    if constexpr (B::DWS) o.al = *reinterpret_cast<const bf16x8*>(pdl + 32 * kk);
#pragma unroll
    for (int c = 0; c < CPG; ++c) {
      if (C0 + c >= B::CT(J)) continue;
      o.b[c] = *reinterpret_cast<const bf16x8*>(px + 16 * c * B::XSP + 32 * kk);
      if constexpr (B::DWX) o.bl[c] = *reinterpret_cast<const bf16x8*>(pxl + 16 * c * B::XSP + 32 * kk);
    }
  };
  KOps ko[2];
  load(0, ko[0]);
#pragma unroll
  for (int kk = 0; kk < B::XS / 32; ++kk) {
    if (kk + 1 < B::XS / 32) load(kk + 1, ko[(kk + 1) & 1]);
    const KOps& o = ko[kk & 1];
#pragma unroll
    for (int c = 0; c < CPG; ++c) {
      if (C0 + c < B::CT(J)) {
        acc[c] = mfma16(o.a, o.b[c], acc[c]);
        if constexpr (B::DWS) acc[c] = mfma16(o.al, o.b[c], acc[c]);
        if constexpr (B::DWX) acc[c] = mfma16(o.a, o.bl[c], acc[c]);
      } else if (C0 + c < B::CTB(J)) {
        // bias tile: the row sums of delta (lo: delta_lo x 1)
        acc[c] = mfma16(o.a, ones, acc[c]);
        if constexpr (B::DWS) acc[c] = mfma16(o.al, ones, acc[c]);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// the unit's column group cg (wave-uniform) selects the instantiation
template <class N, int J, int CG0>
__device__ __forceinline__ void dw_unit_of(const uint8_t* __restrict__ lds, f32x4* __restrict__ acc, int rt,
                                           int cg, int lane) {
  if constexpr (CG0 < Bwd<N>::CG(J)) {
    if (cg == CG0) dw_unit<N, J, CG0 * Bwd<N>::CPG(J)>(lds, acc, rt, lane);
    else dw_unit_of<N, J, CG0 + 1>(lds, acc, rt, cg, lane);
  }
}

// accumulate this wave's units of dW_J (and db_J) over the round: unit u =
// q + i NW is row tile u % RT and column tiles [CPG (u / RT), +CPG)
template <class N, int J>
__device__ __forceinline__ void dw_tiles(const uint8_t* __restrict__ lds, f32x4* __restrict__ dj, int q,
                                         int lane) {
  using B = Bwd<N>;
  const int r16 = lane % 16, kg = lane / 16;
#pragma unroll
  for (int i = 0; i < B::OWN(J); ++i) {
    const int u = q + i * B::NW;
    if (u >= B::UNITS(J)) continue;
    if constexpr (N::BF16) {
      dw_unit_of<N, J, 0>(lds, dj + i * B::CPG(J), u % B::RT(J), u / B::RT(J), lane);
    } else {
      const int rt = u % B::RT(J), c0 = (u / B::RT(J)) * B::CPG(J);
      f32x4* acc = dj + i * B::CPG(J);
      const float* xd = reinterpret_cast<const float*>(lds + B::XD_OFF);
      const float* xh = reinterpret_cast<const float*>(lds + B::XH_OFF);
      float one = r16 == 0 ? 1.f : 0.f;
#pragma unroll
      for (int kk = 0; kk < B::XS / 16; ++kk) {
        int so = 16 * kk + 4 * kg;
        f32x4 a = *reinterpret_cast<const f32x4*>(xd + (16 * rt + r16) * B::XSP + so);
#pragma unroll
        for (int c = 0; c < B::CPG(J); ++c) {
          const int ct = c0 + c;
          if (ct >= B::CTB(J)) continue;
          if (ct < B::CT(J)) {
            f32x4 b = *reinterpret_cast<const f32x4*>(xh + (16 * ct + r16) * B::XSP + so);
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[c] = mfma16(a[e], b[e], acc[c]);
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[c] = mfma16(a[e], one, acc[c]);
          }
        }
      }
    }
  }
}

// add this wave's weight-gradient units of layer J (tiles from dj) to the
// global gradient
template <class N, int J>
__device__ __forceinline__ void flush_dw(const f32x4* __restrict__ dj, float* __restrict__ gm, int q,
                                         int lane) {
  using B = Bwd<N>;
  // folded here: the recursive offset helpers are not inlined when called
  // from a run-time expression, and a call costs the kernel its registers
  constexpr int OW = N::off_w(J), OB = N::off_b(J), OB0 = N::off_b(0);
  const int r16 = lane % 16, rq = lane / 16;
#pragma unroll
  for (int i = 0; i < B::OWN(J); ++i) {
    const int u = q + i * B::NW;
    if (u >= B::UNITS(J)) continue;
    const int rt = u % B::RT(J), c0 = (u / B::RT(J)) * B::CPG(J);
#pragma unroll
    for (int c = 0; c < B::CPG(J); ++c) {
      const int ct = c0 + c;
      if (ct >= B::CTB(J)) continue;
      f32x4 v = dj[i * B::CPG(J) + c];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int n = 16 * rt + 4 * rq + r;
        if (n >= N::fout(J) || v[r] == 0.f) continue;
        if (ct < B::CT(J)) {
          int f = 16 * ct + r16;
          if (f >= B::inp(J)) continue;
          int idx = (J == 0 && f == N::IN) ? OB0 + n : OW + n * N::fin(J) + f;
          atomicAdd(gm + idx, v[r]);
        } else if (r16 == 0) {
          atomicAdd(gm + OB + n, v[r]);
        }
      }
    }
  }
}

template <class N, int J, int LO, int HI>
__device__ __forceinline__ void flush_range(const f32x4* __restrict__ dacc, float* __restrict__ gm, int q,
                                            int lane) {
  flush_dw<N, J>(dacc + Bwd<N>::toff(LO, J), gm, q, lane);
  if constexpr (J < HI) flush_range<N, J + 1, LO, HI>(dacc, gm, q, lane);
}

struct BwdArgs {
  Workspace ws;
  msplat_opts opt;
  int P;
  int n_params;
  int ghits;   // hits per workgroup (a run of one primitive's list), <= 64 per wave
  const float* ray_d;
  const float* grad_rgb;
  const float* grad_feat;
  float* g_mlp;
};

// per-sample state kept from the recompute for a pass over layers LO..HI:
// the sample position (the encoding is evaluated again where it is needed),
// the hi part of the inputs of layers max(LO,1)..HI (their ReLU gates and the
// weight-gradient operand), and the gates of the layers above HI as bits
template <class N, int LO, int HI>
struct Keep {
  static constexpr int H0 = LO > 1 ? LO : 1;
  static constexpr int NH = HI - H0 + 1;
  static constexpr int NG = N::NL - 1 - HI;
  float ph[3], pl[3];
  float dd[N::CONTACT ? 3 : 1];   // contact-point primitive: the ray direction
  Hi<N, rup(N::HID_KS, N::KGRP)> ah[NH > 0 ? NH : 1];
  Hi<N, rup(N::HID_KS, N::KGRP)> al[(Bwd<N>::DWX && NH > 0) ? NH : 1];   // lo parts (full-split weight gradient)
  Gates<N> gt[NG > 0 ? NG : 1];
};

template <class N, int LO, int HI, int J>
__device__ __forceinline__ const Hi<N, rup(N::HID_KS, N::KGRP)>& input_hi(const Keep<N, LO, HI>& kp) {
  return kp.ah[J - Keep<N, LO, HI>::H0];
}
template <class N, int LO, int HI, int J>
__device__ __forceinline__ const Hi<N, rup(N::HID_KS, N::KGRP)>& input_lo(const Keep<N, LO, HI>& kp) {
  return kp.al[Bwd<N>::DWX ? J - Keep<N, LO, HI>::H0 : 0];
}

// ReLU gate of slot t of layer J's input (its pre-activation was positive)
template <class N, int LO, int HI, int J>
__device__ __forceinline__ bool gate(const Keep<N, LO, HI>& kp, int t) {
  if constexpr (J <= HI) {
    if constexpr (N::BF16) {
      // the kept input is relu(z) >= +0 rounded to bfloat16: open iff its bits are non-zero
      const uint32_t w = __builtin_bit_cast(uint4, input_hi<N, LO, HI, J>(kp).hi[t / 8])[(t % 8) / 2];
      return (t % 2) ? w > 0xffffu : (uint16_t)w != 0;
    } else {
      return input_hi<N, LO, HI, J>(kp).hi[t] > 0.f;
    }
  }
  else return (kp.gt[J - HI - 1].w[t / 32] >> (t % 32)) & 1u;
}

// forward recompute keeping what the backward needs (wb: the operands as the
// layout FL places them, LDS or global; wg: the packed copy the rest is read
// from)
template <class N, int J, int LO, int HI>
__device__ __forceinline__ void chain_keep(const uint8_t* __restrict__ wb, const uint8_t* __restrict__ wg, int lane,
                                           Keep<N, LO, HI>& kp, f32x16 (&acc)[N::RBH], f32x16& out) {
  constexpr int FL = Bwd<N>::FL;
  Act<N, rup(N::HID_KS, N::KGRP)> x;
  relu_to_B<N>(acc, x);
  if constexpr (J >= Keep<N, LO, HI>::H0 && J <= HI) {
#pragma unroll
    for (int i = 0; i < rup(N::HID_KS, N::KGRP); ++i) {
      kp.ah[J - Keep<N, LO, HI>::H0].hi[i] = x.hi[i];
      if constexpr (Bwd<N>::DWX) kp.al[J - Keep<N, LO, HI>::H0].hi[i] = x.lo[i];
    }
  } else if constexpr (J > HI) {
    gates_of<N>(acc, kp.gt[J - HI - 1]);
  }
  if constexpr (J < N::NL - 1) {
    layer_fwd<N, J, N::HID_KS, FL>(wb, wg, lane, x, acc);
    chain_keep<N, J + 1, LO, HI>(wb, wg, lane, kp, acc, out);
  } else {
    f32x16 o[1];
    layer_fwd<N, J, N::HID_KS, FL>(wb, wg, lane, x, o);
    out = o[0];
  }
}

// (wb0: where the first layer's forward operands are read, which may differ
// from wb; they are requested before the encoding is computed.  wl: the
// staged hi sections where the layout FL has them, else wb)
template <class N, int LO, int HI>
__device__ __forceinline__ f32x16 forward_keep(const uint8_t* __restrict__ wb, const uint8_t* __restrict__ wb0,
                                               const uint8_t* __restrict__ wl, int lane, const float ph[3],
                                               const float pl[3], const float dd[3], Keep<N, LO, HI>& kp) {
  constexpr int FL = Bwd<N>::FL;
  int g = lane / 32;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    kp.ph[a] = ph[a];
    kp.pl[a] = pl[a];
    if constexpr (N::CONTACT) kp.dd[a] = dd[a];
  }
  f32x16 acc[N::RBH];
  {
    FwdOps<N, 0, N::ENC_KS> first;
    fwd_row_load<N, 0, N::ENC_KS, FL>(FL == kPacked ? wb0 : wl, wb0, lane, 0, first);
    float ev[N::ENC_KS * N::KSTEP];
    encode_input<N>(ph, pl, dd, g, ev);
    Act<N, rup(N::ENC_KS, N::KGRP)> a0;
    enc_to_B<N>(ev, a0);
    // matrix-core stretch: issue ahead of the other wave's vector work
    mfma_priority<N, 1>();
    layer_fwd_from<N, 0, N::ENC_KS, FL>(FL == kPacked ? wb0 : wl, wb0, lane, a0, acc, first);
  }
  f32x16 out;
  chain_keep<N, 1, LO, HI>(FL == kPacked ? wb : wl, wb, lane, kp, acc, out);
  mfma_priority<N, 0>();
  return out;
}

// backward through layer J (and below): the transposed product towards layer
// J-1, and, where the pass accumulates layer J's weight gradient, the
// exchange of the block's deltas and inputs with the other waves
template <class N, int J, int LO, int HI>
__device__ __forceinline__ void chain_back(uint8_t* __restrict__ lds, const uint8_t* __restrict__ wb, int lane,
                                           int q, int colx, const Keep<N, LO, HI>& kp,
                                           const f32x16 (&dz)[N::frb(J)], float (&dp)[3],
                                           f32x4* __restrict__ dacc) {
  constexpr bool DW = J >= LO && J <= HI;     // layer J's weight gradient
  constexpr bool DOWN = J > 0 && J - 1 >= LO;  // continue to layer J-1
  const int g = lane / 32;
  float ev[N::ENC_KS * N::KSTEP];
  if constexpr (J == 0) {
    if constexpr (N::CONTACT) encode_contact_slots<N>(kp.ph, kp.pl, kp.dd, g, ev);
    else encode_slots<N>(kp.ph, kp.pl, g, ev);
  }
  // the delta as the transposed product's B operand (also what is published)
  Act<N, rup(N::bks(J), N::KGRP)> Bd;
  if constexpr (DW || DOWN || J == 0) {
    if constexpr (J == N::NL - 1) d_to_B<N, N::OUT_SLOTS, N::frb(J)>(dz, Bd);
    else d_to_B<N, 16 * N::RBH, N::frb(J)>(dz, Bd);
  }
  if constexpr (DW) {
    publish_delta<N, J, rup(N::bks(J), N::KGRP)>(lds, dz, Bd, g, colx);
    if constexpr (J == 0) {
      Act<N, rup(N::ENC_KS, N::KGRP)> a0;
      enc_to_B<N>(ev, a0);
      Hi<N, rup(N::ENC_KS, N::KGRP)> h0;
#pragma unroll
      for (int i = 0; i < rup(N::ENC_KS, N::KGRP); ++i) h0.hi[i] = a0.hi[i];
      publish_input<N, 0, rup(N::ENC_KS, N::KGRP)>(lds, h0, g, colx);
      if constexpr (Bwd<N>::DWX) {
#pragma unroll
        for (int i = 0; i < rup(N::ENC_KS, N::KGRP); ++i) h0.hi[i] = a0.lo[i];
        publish_input<N, 0, rup(N::ENC_KS, N::KGRP), true>(lds, h0, g, colx);
      }
    } else {
      publish_input<N, J, rup(N::HID_KS, N::KGRP)>(lds, input_hi<N, LO, HI, J>(kp), g, colx);
      if constexpr (Bwd<N>::DWX)
        publish_input<N, J, rup(N::HID_KS, N::KGRP), true>(lds, input_lo<N, LO, HI, J>(kp), g, colx);
    }
  }
  // transposed product for the next delta (or the input gradient), overlapping the exchange
  f32x16 da[N::brb(J)];
  mfma_priority<N, 1>();
  if constexpr (DOWN || J == 0) layer_bwd<N, J>(wb, lane, Bd, da);
  if constexpr (DW) {
    __syncthreads();
    dw_tiles<N, J>(lds, dacc + Bwd<N>::toff(LO, J), q, lane);
    __syncthreads();
  }
  mfma_priority<N, 0>();
  if constexpr (DOWN) {
    // relu': the layer input a_J = relu(z_{J-1}) is positive where z_{J-1} is
    f32x16 dzn[N::RBH];
#pragma unroll
    for (int rb = 0; rb < N::RBH; ++rb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) dzn[rb][r] = gate<N, LO, HI, J>(kp, 16 * rb + r) ? da[rb][r] : 0.f;
    }
    chain_back<N, J - 1, LO, HI>(lds, wb, lane, q, colx, kp, dzn, dp, dacc);
  } else if constexpr (J == 0 && N::CONTACT) {
    // dL/d(delta) of the contact point from the input-feature gradient
    // W_0^T delta_0 (the direction d carries no gradient)
#pragma unroll
    for (int a = 0; a < 3; ++a) dp[a] = 0.f;
#pragma unroll
    for (int t = 0; t < 6 * N::L; ++t) {
      const int pr = t / 12, r = t % 12, c = r % 6;
      if (c < 3) continue;
      const float gf = da[t / 16][t % 16];
      const float mul = (float)(1 << (2 * pr)) * (g ? 2.f : 1.f) * 3.14159265358979f;
      // d sin(m x)/dx = m cos(m x); d cos(m x)/dx = -m sin(m x)
      const float dv = r < 6 ? mul * ev[12 * pr + 6 + c] : -mul * ev[12 * pr + c];
      dp[c - 3] += gf * dv;
    }
  } else if constexpr (J == 0) {
    // dL/dp of the sample from the input-feature gradient W_0^T delta_0
#pragma unroll
    for (int a = 0; a < 3; ++a) dp[a] = 0.f;
#pragma unroll
    for (int t = 0; t < N::ENC_SLOTS; ++t) {
      float gf = da[t / 16][t % 16];
      if (t < 3 * N::L) {
        int pr = t / 6, j = t % 6, a = j % 3;
        float mul = (float)(1 << (2 * pr)) * (g ? 2.f : 1.f) * 3.14159265358979f;
        // d sin(m p)/dp = m cos(m p); d cos(m p)/dp = -m sin(m p)
        float dv = j < 3 ? mul * ev[6 * pr + 3 + a] : -mul * ev[6 * pr + a];
        dp[a] += gf * dv;
      } else {
        int a = t - 3 * N::L;
        if (g == 0) dp[a] += gf;
      }
    }
  }
}

// one pass of the backward: recompute the network, chain the adjoint down to
// layer LO and accumulate the weight gradients of layers LO..HI (and, when LO
// is 0, the geometry gradient).  Weights are staged in LDS, or read from
// global memory for wide networks.
template <class N, int LO, int HI>
__global__ __launch_bounds__(64 * Bwd<N>::NW) void mlp_backward_kernel(BwdArgs args) {
  using B = Bwd<N>;
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  __shared__ int rounds_s[B::NW];
  const Workspace& ws = args.ws;
  const int lane = threadIdx.x % 64;
  const int q = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);   // (wave-uniform: scalar)
  const int col = lane % 32;
  const int g = lane / 32;
  const int colx = 32 * q + col;
  const int64_t H = ws.hit_cap;
  const uint32_t seed_hash = pcg_hash(args.opt.jitter_seed);
  // The workgroup takes a run of up to args.ghits consecutive hits of one
  // primitive's list (the hits of `group` work items of the forward, at most
  // 64 per wave): the weights are staged once, the hits are dealt to the
  // waves in one balanced deal, and the weight-gradient sums stay in
  // registers until they are added to the global gradient at the end.
  constexpr int NW = B::NW;
  const int bid = blockIdx.x;
  if (bid >= ws.gw_off[args.P]) return;   // (the grid is an upper bound)
  const int p = find_prim(ws.gw_off, args.P, bid);
  const int first = ws.prim_off[p] + (bid - ws.gw_off[p]) * args.ghits;
  const int nh = min(args.ghits, ws.prim_off[p + 1] - first);
  const uint8_t* wglb = ws.wpack + (int64_t)p * ws.wpack_bytes;
  if constexpr (!B::GW) {
    // packed bytes [SKIP, total) go to LDS at W_OFF (read after the
    // barriers below)
    const uint4* src = reinterpret_cast<const uint4*>(wglb + B::SKIP);
    uint4* dst = reinterpret_cast<uint4*>(lds + B::W_OFF);
    for (int i = threadIdx.x; i < (N::total_bytes() - B::SKIP) / 16; i += blockDim.x) dst[i] = src[i];
  }
  // wts: the base that the packed offsets of the weights are taken from (LDS
  // for the staged sections); wts0: where the first layer's forward operands
  // are read
  if constexpr (B::HS > 0) {
    // the hi sections of layers 0..HS-1 of the forward operands
    uint4* dst = reinterpret_cast<uint4*>(lds + B::W_OFF);
#pragma unroll
    for (int j = 0; j < B::HS; ++j) {
      const uint4* src = reinterpret_cast<const uint4*>(wglb + N::fwdA_off(j));
      for (int i = threadIdx.x; i < N::fwdA_single(j) / 16; i += blockDim.x) dst[N::fwd_hi_off(j) / 16 + i] = src[i];
    }
  }
  const uint8_t* wts = B::GW ? wglb : lds + B::W_OFF - B::SKIP;
  const uint8_t* wts0 = B::G0 ? wglb : wts;
  // ---- deal the run's hits to the waves (the exchange planes are free here)
  int my_k;
  int my_li;
  {
    const int idx = 64 * q + lane;
    int key = -1;
    if (idx < nh) {
      const int h = ws.phit[first + idx];
      const int kk = ws.hit_nused[h] > 0 ? (ws.hit_k[h] & kKMask) : 0;
      key = (kk << 9) | (511 - idx);
    }
    my_li = deal_run<NW>(key, reinterpret_cast<int*>(lds + B::XH_OFF), q, lane, my_k);
  }
  const int my_hit = my_li < 0 ? 0 : ws.phit[first + my_li];
  // the hit's ray and its slot along the ray (for the sample offsets), read
  // once here rather than per block
  int my_ray = 0, my_slot = 0;
  if (my_li >= 0) {
    my_ray = ws.hit_ray[my_hit];
    my_slot = my_hit - ws.ray_off[my_ray];
  }
  const int c = __popcll(__ballot(my_li >= 0));   // (the wave's hits fill lanes 0..c-1)
  int incl = wave_incl_scan(my_k);
  int my_off = incl - my_k;
  const int ns = __builtin_amdgcn_readlane(incl, 63);
  const int nblk = (ns + 31) / 32;
  if (lane == 0) rounds_s[q] = nblk;
  __syncthreads();
  int rounds = 0;
  for (int i = 0; i < NW; ++i) rounds = max(rounds, rounds_s[i]);
  f32x4 dacc[B::tiles(LO, HI)];
#pragma unroll
  for (int i = 0; i < B::tiles(LO, HI); ++i) dacc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  // carries of the hit-local scans from block to block
  float cr_tau = 0.f, cr_P = 0.f, cr_geo[7];
#pragma unroll
  for (int i = 0; i < 7; ++i) cr_geo[i] = 0.f;

  int lb = 0;   // (scalar) lane of the hit holding the block's first column
  for (int b = 0; b < rounds; ++b) {
    const int x = 32 * b + col;
    const bool valid = x < ns;
    // the hit of this column: the last of the wave's hits whose samples
    // start at or before it (hit records read from lanes into scalar
    // registers).  The hits sit in lanes 0..c-1 in sample order: the
    // cursor lb moves to the hit holding the block's first column, then the
    // hits starting inside the block are taken.
    const int x0 = 32 * b;
    while (lb + 1 < c && __builtin_amdgcn_readlane(my_off, lb + 1) <= x0) ++lb;
    int hit = __builtin_amdgcn_readlane(my_hit, lb), K = __builtin_amdgcn_readlane(my_k, lb);
    int hoff = __builtin_amdgcn_readlane(my_off, lb), hli = __builtin_amdgcn_readlane(my_li, lb);
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
        hli = __builtin_amdgcn_readlane(my_li, l);
      }
    }
    const int k = valid ? x - hoff : 0;
    float u = 0.5f;
    if (args.opt.jitter) u = sample_offset(seed_hash, (uint32_t)ray, (uint32_t)slot, (uint32_t)k);
    const float dlt = ws.hit_dlt[hit];
    // the hit's compositing records and the ray's upstream gradient are
    // loaded before the recompute so that their latency overlaps it
    const int nused = valid ? ws.hit_nused[hit] : 0;
    const float tb = valid ? ws.hit_tb[hit] : 0.f;
    const float gtot = valid ? ws.hit_gtot[hit] : 0.f;
    const float gsa = valid ? ws.hit_gsa[hit] : 0.f;
    // slot features enter like a colour channel constant over the hit
    const float gq = (ws.slot_on && valid) ? ws.hit_q[hit] : 0.f;
    float gr[3] = {0.f, 0.f, 0.f};
    if (valid) {
#pragma unroll
      for (int r = 0; r < 3; ++r) gr[r] = args.grad_rgb[3 * ray + r];
    }
    float ph[3], pl[3], dd[3];
    sample_input<N>(ws, hit, k, u, ph, pl, dd);
    const bool last = valid && k == K - 1;
    Keep<N, LO, HI> kp;
    f32x16 o = forward_keep<N, LO, HI>(wts, wts0, lds + B::W_OFF, lane, ph, pl, dd, kp);

    // ---- compositing adjoint of the column ----
    const bool used = valid && k < nused;
    float cc[3], sig = 0.f, sgm = 0.f;
#pragma unroll
    for (int r = 0; r < 3; ++r) cc[r] = sigmoidf_(o[r]);
    if (g == 0) {
      sig = softplusf_(o[3]);
      sgm = sigmoidf_(o[3]);
    }
    float tau0 = valid ? sig * dlt : 0.f;
    const float tau = from_lower_half(tau0);
    // g . (colour, features) of the sample: half 0 holds RGB, both halves features
    float gcf = g == 0 ? gr[0] * cc[0] + gr[1] * cc[1] + gr[2] * cc[2] : 0.f;
    float gfv[N::OUT_SLOTS];
#pragma unroll
    for (int r = 0; r < N::OUT_SLOTS; ++r) {
      gfv[r] = 0.f;
      if constexpr (N::CF > 0) {
        int f = phi_std(g, r) - 4;
        if (valid && f >= 0 && f < N::CF) {
          gfv[r] = args.grad_feat ? args.grad_feat[(int64_t)ray * N::CF + f] : 0.f;
          gcf += gfv[r] * o[r];
        }
      }
    }
    const float gc = gcf + other_half(gcf, g) + gq;
    const bool head = (k == 0);
    SegScan sc(head, col);
    float tincl = sc.incl(tau);
    if (!sc.seen_head) tincl += cr_tau;
    float texcl = col_below(tincl, col);
    if (head) texcl = 0.f;
    else if (col == 0) texcl = cr_tau;
    const float alpha = -expm1f(-tau);
    const float w = used ? tb * __expf(-texcl) * alpha : 0.f;
    float P = sc.incl(w * gc);
    if (!sc.seen_head) P += cr_P;
    const float dtau = used ? (tb * __expf(-tincl) * gc - (gtot - P) - gsa) : 0.f;
    // dL/d(raw outputs) in D layout (row block 0)
    f32x16 dz[1];
#pragma unroll
    for (int r = 0; r < 16; ++r) dz[0][r] = 0.f;
    if (g == 0) {
#pragma unroll
      for (int r = 0; r < 3; ++r) dz[0][r] = w * gr[r] * cc[r] * (1.f - cc[r]);
      dz[0][3] = dtau * dlt * sgm;
    }
#pragma unroll
    for (int r = 0; r < N::OUT_SLOTS; ++r)
      if constexpr (N::CF > 0) {
        int f = phi_std(g, r) - 4;
        if (f >= 0 && f < N::CF) dz[0][r] = w * gfv[r];
      }
    // half 0 holds dtau * sigma (for dL/dDelta); both halves take it
    const float dts = from_lower_half(dtau * sig);
    // carries of the compositing scans into the next block
    // (both halves hold the same scans)
    cr_tau = col31_same(tincl);
    cr_P = col31_same(P);

    // ---- network adjoint and weight gradients ----
    float dp[3] = {0.f, 0.f, 0.f};
    chain_back<N, N::NL - 1, LO, HI>(lds, wts, lane, q, colx, kp, dz, dp, dacc);
    if constexpr (LO > 0) continue;   // this pass has no geometry gradient

    // ---- dL/dp of the sample: the two lane halves hold disjoint encoding slots ----
#pragma unroll
    for (int a = 0; a < 3; ++a) dp[a] += other_half(dp[a], g);
    if (!valid) dp[0] = dp[1] = dp[2] = 0.f;

    // ---- per-hit geometry sums ----
    // Scanned over each hit's samples: dL/dp (3), (k + u) dL/dp (3) and the
    // optical-depth factor's adjoint (1); the contact-point primitive (one
    // sample per hit) needs dL/d(delta) and that factor only.  The other
    // sums the geometry adjoint takes follow per hit, e being fixed per hit:
    // with s_k = s_a + (k + u) Delta and dL/ds_k = e . dL/dp,
    //   sum s_k dL/dp = s_a sum dL/dp + Delta sum (k + u) dL/dp,
    //   sum dL/ds_k = e . sum dL/dp,
    //   sum omega_k dL/ds_k = e . sum (k + u) dL/dp / K.
    constexpr int NS = N::CONTACT ? 4 : 7;
    float sv[NS];
#pragma unroll
    for (int a = 0; a < 3; ++a) sv[a] = dp[a];
    if constexpr (!N::CONTACT) {
      const float ku = (float)k + u;
#pragma unroll
      for (int a = 0; a < 3; ++a) sv[3 + a] = ku * dp[a];
    }
    sv[NS - 1] = dts;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      sv[i] = sc.incl(sv[i]);
      if (!sc.seen_head) sv[i] += cr_geo[i];
    }
    // the lane of the hit's last sample leaves the hit's sums; the chain to
    // the primitive's frame runs per hit in a kernel of its own
    if (last && g == 0) {
      const int pos = first + hli;   // the hit's entry in the grouped list
      float gv[9];
#pragma unroll
      for (int a = 0; a < 3; ++a) gv[a] = sv[a];
      if constexpr (N::CONTACT) {
        gv[3] = gv[4] = gv[5] = gv[6] = gv[7] = 0.f;
      } else {
        const float sa = ws.hit_sa[hit];
        float ee[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          ee[a] = ws.hit_e[a * H + hit];
          gv[3 + a] = sa * sv[a] + dlt * sv[3 + a];
        }
        gv[6] = ee[0] * sv[0] + ee[1] * sv[1] + ee[2] * sv[2];
        gv[7] = (ee[0] * sv[3] + ee[1] * sv[4] + ee[2] * sv[5]) * __builtin_amdgcn_rcpf((float)K);
      }
      gv[8] = sv[NS - 1];
#pragma unroll
      for (int i = 0; i < 9; ++i) ws.hit_gv[i * H + pos] = gv[i];
    }
    // carries of the geometry scans
#pragma unroll
    for (int i = 0; i < NS; ++i) cr_geo[i] = col31_same(sv[i]);
  }

  // ---- flush the weight-gradient strips ----
  flush_range<N, LO, LO, HI>(dacc, args.g_mlp + (int64_t)p * args.n_params, q, lane);
}

}  // namespace

template <class N, int LO, int HI>
static hipError_t bwd_pass(const BwdArgs& a, int64_t groups, hipStream_t s) {
  size_t lds = Bwd<N>::LDS;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)mlp_backward_kernel<N, LO, HI>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL((mlp_backward_kernel<N, LO, HI>), dim3((unsigned)groups), dim3(64 * Bwd<N>::NW), lds, s, a);
  return hipGetLastError();
}

// wide networks: passes over ranges of WSPAN layers, from layer LO up
template <class N, int LO>
static hipError_t wide_passes(const BwdArgs& a, int64_t groups, hipStream_t s) {
  constexpr int HI = LO + N::WSPAN - 1 < N::NL - 1 ? LO + N::WSPAN - 1 : N::NL - 1;
  hipError_t e = bwd_pass<N, LO, HI>(a, groups, s);
  if constexpr (HI + 1 < N::NL) {
    if (e == hipSuccess) return wide_passes<N, HI + 1>(a, groups, s);
  }
  return e;
}

template <class N>
static hipError_t bwd_impl(const Workspace& ws, const msplat_opts& o, int64_t num_hits, int group, int P,
                           int n_params, const float* ray_d, const float* grad_rgb, const float* grad_feat,
                           float* g_mlp, hipStream_t s) {
  if (num_hits <= 0) return hipSuccess;
  if (group < 1 || ws.hits_per_item < 1) return hipErrorInvalidValue;
  // a workgroup's run: `group` work items of the forward, at most 64 hits per wave
  const int ghits = min(group * ws.hits_per_item, 64 * Bwd<N>::NW);
  BwdArgs a{ws, o, P, n_params, ghits, ray_d, grad_rgb, grad_feat, g_mlp};
  hipError_t e = launch_group_scan(ws, P, ghits, s);
  if (e != hipSuccess) return e;
  // at most ceil(hits / ghits) runs plus one partial run per primitive; the
  // workgroups past the last run return at once
  const int64_t groups = (num_hits + ghits - 1) / ghits + P;
  if constexpr (N::WIDE) {
    return wide_passes<N, 0>(a, groups, s);
  } else if constexpr (N::PASSES) {
    // the upper half of the layers, then the lower half with the geometry
    constexpr int M = N::NL / 2;
    hipError_t e = bwd_pass<N, M, N::NL - 1>(a, groups, s);
    return e != hipSuccess ? e : bwd_pass<N, 0, M - 1>(a, groups, s);
  } else {
    return bwd_pass<N, 0, N::NL - 1>(a, groups, s);
  }
}

hipError_t MSPLAT_TU_FN(launch_mlp_backward)(const NetShape& n, const Workspace& ws, const msplat_opts& o,
                                             int64_t num_hits, int group, const float* ray_d,
                                             const float* grad_rgb, const float* grad_feat, float* g_mlp,
                                             hipStream_t s) {
#define X(L_, W_, D_, O_, P_, K_)                                                                   \
  MSPLAT_MATCH(L_, W_, D_, O_, P_, K_)                                                              \
  return bwd_impl<MSPLAT_NET(L_, W_, D_, O_, P_, K_)>(ws, o, num_hits, group, n.P, n.n_params, ray_d, \
                                                      grad_rgb, grad_feat, g_mlp, s);
  MSPLAT_TU_NETS(X)
#undef X
  return hipErrorInvalidValue;
}

#ifndef MSPLAT_WIDE_TU
hipError_t launch_mlp_backward_wide(const NetShape& n, const Workspace& ws, const msplat_opts& o,
                                    int64_t num_hits, int group, const float* ray_d, const float* grad_rgb,
                                    const float* grad_feat, float* g_mlp, hipStream_t s);

hipError_t launch_mlp_backward(const NetShape& n, const Workspace& ws, const msplat_opts& o, int64_t num_hits,
                               int group, const float* ray_d, const float* grad_rgb, const float* grad_feat,
                               float* g_mlp, hipStream_t s) {
  return wide_net(n.W)
             ? launch_mlp_backward_wide(n, ws, o, num_hits, group, ray_d, grad_rgb, grad_feat, g_mlp, s)
             : launch_mlp_backward_narrow(n, ws, o, num_hits, group, ray_d, grad_rgb, grad_feat, g_mlp, s);
}
#endif

}  // namespace msplat
