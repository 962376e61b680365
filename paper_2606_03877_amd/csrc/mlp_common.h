// Shared definitions of the per-primitive MLP kernels: network shape,
// operand packing order and the matrix-core helpers.
//
// Matrix-core layouts (gfx950, wave64), verified on the device:
//   32x32x16 bf16 / 32x32x2 f32: A lane l holds row l%32 and k = kstep*(l/32)+e,
//     B lane l holds column l%32 and the same k, D lane l holds column l%32 and
//     rows 8*(r/4) + 4*(l/32) + r%4 for r = 0..15.
//   16x16x32 bf16 / 16x16x4 f32: A lane l holds row l%16 and k = kstep*(l/16)+e,
//     B lane l holds column l%16, D lane l holds column l%16, rows 4*(l/16)+r.
//
// Samples are the matrix columns (one sample per lane%32) and features the
// rows, so a layer's D registers are directly the next layer's B operand: the
// input feature order of every layer is permuted to the D-register order
// ("slots") and the weights are packed in that order once per call.
#pragma once

#include "common.h"

namespace msplat {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// feature held by D-register slot t (= 16*block + reg) of lane half g
__host__ __device__ constexpr int phi_std(int g, int t) {
  return 32 * (t / 16) + 8 * ((t % 16) / 4) + 4 * g + t % 4;
}
__host__ __device__ inline void phi_std_inv(int rho, int& g, int& t) {
  int rl = rho % 32;
  g = (rl / 4) % 2;
  t = 16 * (rho / 32) + 4 * (rl / 8) + rl % 4;
}
// encoding slot -> canonical input feature.  Canonical order (also the weight
// layout): [p_x, p_y, p_z, then per level l: sin x,y,z, cos x,y,z], then the
// constant 1 that carries the first layer's bias (index 3 + 6L).  Half 0
// takes the even levels and the identity terms, half 1 the odd levels and the
// constant, so both halves run the same instruction stream.
__host__ __device__ constexpr int phi_enc(int L, int g, int t) {
  return t < 3 * L ? 3 + 6 * (2 * (t / 6) + g) + t % 6
                   : (t < 3 * L + 3 ? (g == 0 ? t - 3 * L : (t == 3 * L ? 3 + 6 * L : -1)) : -1);
}

// The contact-point primitive's input [d; delta] (6 values) encoded per
// component with L levels and no identity term (12 L values).  Canonical
// order (also the weight layout): component c, level l, sin then cos at
// index 2 L c + 2 l (+1), then the constant 1 of the first layer's bias at
// 12 L.  Slot t of lane half g: levels 2 (t / 12) + g, within a level the
// six sines then the six cosines; half 1 holds the constant after them.
__host__ __device__ constexpr int phi_enc_contact(int L, int g, int t) {
  return t < 6 * L ? 2 * L * ((t % 12) % 6) + 2 * (2 * (t / 12) + g) + (t % 12) / 6
                   : (t == 6 * L && g == 1 ? 12 * L : -1);
}

__host__ __device__ constexpr int rup(int a, int b) { return (a + b - 1) / b * b; }
// networks wider than this read their weights from global memory (see Net::WIDE)
__host__ __device__ constexpr bool wide_net(int W) { return W > 64; }

// SPLIT_: bfloat16 operands carried as a sum of two bfloat16 values (hi, lo);
// a product of two such operands is taken as hi*hi + hi*lo + lo*hi on the
// matrix cores with float32 accumulation (about 16 significant bits).
// CONTACT_: the contact-point primitive (one interaction per hit, input the
// encoded [d; delta]); otherwise samples of the hit chord, input the encoded
// local position.
template <int L_, int W_, int D_, int NOUT_, bool BF16_, bool SPLIT_ = false, bool CONTACT_ = false>
struct Net {
  static constexpr int L = L_, W = W_, D = D_, NOUT = NOUT_;
  static constexpr bool BF16 = BF16_;
  static constexpr bool SPLIT = SPLIT_;
  static constexpr bool CONTACT = CONTACT_;
  static_assert(BF16 || !SPLIT, "split operands are a bfloat16 form");
  static constexpr int NSPLIT = SPLIT ? 2 : 1;
  static constexpr int IN = CONTACT ? 12 * L : 3 + 6 * L;
  static constexpr int NL = D + 1;
  static constexpr int CF = NOUT - 4;
  static constexpr int NC = NOUT - 1;                 // rgb + features composited
  static constexpr int KSTEP = BF16 ? 8 : 1;          // slots per lane half per k-step
  static constexpr int KGRP = BF16 ? 1 : 4;           // k-steps per 16-byte operand group
  static constexpr int ENC_SLOTS = CONTACT ? 6 * L + 1 : 3 * L + 3;
  static constexpr int ENC_KS = rup(ENC_SLOTS, KSTEP) / KSTEP;
  static constexpr int RBH = W / 32;
  static constexpr int HID_KS = 16 * RBH / KSTEP;
  // D-register slots that hold output rows 0..NOUT-1 (rows 8i..8i+7 use slots 4i..4i+3)
  static constexpr int OUT_SLOTS = 4 * ((NOUT + 7) / 8);
  static constexpr int OUT_KS = rup(OUT_SLOTS, KSTEP) / KSTEP;
  static constexpr int RB0 = (ENC_SLOTS + 15) / 16;   // row blocks of the input-gradient
  // wide networks read their weight operands from global memory (they stay
  // in L2 while a primitive's work items run) instead of staging them in LDS,
  // and split the backward into passes over ranges of layers
  static constexpr bool WIDE = wide_net(W);
  // layers per backward pass of a wide network: each pass recomputes the
  // network and holds its layers' weight-gradient accumulators.  For
  // 39-128x4-20, 3 (two passes) measured 251 ms per backward on a 1080p
  // frame, against 407 ms for one pass per layer and 254 ms for one pass.
  static constexpr int WSPAN = 3;
  // backward split into two passes over halves of the layers (fewer live
  // weight-gradient accumulators, the network recomputed twice); measured
  // slower than one spilling pass for the 64-wide split form, so off
  static constexpr bool PASSES = false;
  static_assert(L % 2 == 0, "encoding split needs an even number of levels");
  static_assert(W % 32 == 0, "hidden width must be a multiple of 32");
  static_assert(NOUT >= 4 && NOUT <= kMaxOut, "4 to kMaxOut outputs (the compositor holds kMaxOut - 4 features)");

  // forward layer j: k-steps, row blocks, padded k-steps
  __host__ __device__ static constexpr int fks(int j) { return j == 0 ? ENC_KS : HID_KS; }
  __host__ __device__ static constexpr int frb(int j) { return j == NL - 1 ? 1 : RBH; }
  __host__ __device__ static constexpr int fin(int j) { return j == 0 ? IN : W; }
  __host__ __device__ static constexpr int fout(int j) { return j == NL - 1 ? NOUT : W; }
  // backward (transposed) layer j: rows = input slots, k = output slots
  __host__ __device__ static constexpr int brb(int j) { return j == 0 ? RB0 : RBH; }
  __host__ __device__ static constexpr int bks(int j) { return j == NL - 1 ? OUT_KS : HID_KS; }
  __host__ __device__ static constexpr int groups(int ks) { return rup(ks, KGRP) / KGRP; }

  // byte sizes of the packed sections (a split section holds all hi parts,
  // then all lo parts)
  __host__ __device__ static constexpr int fwdA_single(int j) { return frb(j) * groups(fks(j)) * 64 * 16; }
  __host__ __device__ static constexpr int bwdA_single(int j) { return brb(j) * groups(bks(j)) * 64 * 16; }
  __host__ __device__ static constexpr int fwdA_bytes(int j) { return NSPLIT * fwdA_single(j); }
  __host__ __device__ static constexpr int bias_bytes(int j) { return j == 0 ? 0 : frb(j) * 2 * 16 * 4; }
  __host__ __device__ static constexpr int bwdA_bytes(int j) { return NSPLIT * bwdA_single(j); }
  __host__ __device__ static constexpr int fwdA_off(int j) {
    return j == 0 ? 0 : fwdA_off(j - 1) + fwdA_bytes(j - 1);
  }
  __host__ __device__ static constexpr int bias_off(int j) {
    return j == 0 ? fwdA_off(NL - 1) + fwdA_bytes(NL - 1) : bias_off(j - 1) + bias_bytes(j - 1);
  }
  __host__ __device__ static constexpr int fwd_bytes() { return bias_off(NL - 1) + bias_bytes(NL - 1); }
  // a forward staging of the hi parts only (split form): the layers' hi
  // sections back to back, then the biases
  __host__ __device__ static constexpr int fwd_hi_off(int j) {
    return j == 0 ? 0 : fwd_hi_off(j - 1) + fwdA_single(j - 1);
  }
  __host__ __device__ static constexpr int fwd_hi_bias(int j) { return fwd_hi_off(NL) + bias_off(j) - bias_off(0); }
  __host__ __device__ static constexpr int fwd_hi_bytes() { return fwd_hi_off(NL) + fwd_bytes() - bias_off(0); }
  __host__ __device__ static constexpr int bwdA_off(int j) {
    return j == 0 ? fwd_bytes() : bwdA_off(j - 1) + bwdA_bytes(j - 1);
  }
  __host__ __device__ static constexpr int total_bytes() { return bwdA_off(NL - 1) + bwdA_bytes(NL - 1); }

  // parameter offsets in the canonical per-primitive vector
  __host__ __device__ static constexpr int off_w(int j) {
    return j == 0 ? 0 : off_w(j - 1) + fin(j - 1) * fout(j - 1) + fout(j - 1);
  }
  __host__ __device__ static constexpr int off_b(int j) { return off_w(j) + fin(j) * fout(j); }
  __host__ __device__ static constexpr int n_params() { return off_w(NL - 1) + fin(NL - 1) * fout(NL - 1) + NOUT; }

  // input feature (canonical index, -1 = padding) of an input slot of layer j
  __host__ __device__ static constexpr int in_feat(int j, int g, int t) {
    return j == 0 ? (t < ENC_SLOTS ? (CONTACT ? phi_enc_contact(L, g, t) : phi_enc(L, g, t)) : -1)
                  : (phi_std(g, t) < W ? phi_std(g, t) : -1);
  }
};

// weight W_j[n][f] of the canonical parameter vector (f = IN of layer 0 is
// the bias carried by the constant feature)
template <class N>
__device__ __forceinline__ float net_weight(const float* th, int j, int n, int f) {
  if (n < 0 || n >= N::fout(j) || f < 0) return 0.f;
  if (j == 0 && f == N::IN) return th[N::off_b(0) + n];
  if (f >= N::fin(j)) return 0.f;
  return th[N::off_w(j) + n * N::fin(j) + f];
}

// Compiled networks: (pe_freqs, hidden width, hidden layers, outputs,
// precision, primitive).  Networks up to 64 wide and wider ones are compiled
// in separate units (the wide kernels with the compiler's default register
// assignment).
#define MSPLAT_NETS_NARROW(X)                                                                            \
  X(4, 32, 2, 4, MSPLAT_FP32, 0) X(4, 32, 2, 4, MSPLAT_BF16, 0) X(4, 32, 2, 4, MSPLAT_BF16X3, 0)          \
  X(6, 64, 3, 4, MSPLAT_FP32, 0) X(6, 64, 3, 4, MSPLAT_BF16, 0) X(6, 64, 3, 4, MSPLAT_BF16X3, 0)          \
  X(6, 64, 3, 20, MSPLAT_FP32, 0) X(6, 64, 3, 20, MSPLAT_BF16, 0) X(6, 64, 3, 20, MSPLAT_BF16X3, 0)       \
  X(6, 32, 2, 4, MSPLAT_FP32, 1) X(6, 32, 2, 4, MSPLAT_BF16X3, 1)
#define MSPLAT_NETS_WIDE(X) \
  X(6, 128, 4, 20, MSPLAT_FP32, 0) X(6, 128, 4, 20, MSPLAT_BF16, 0) X(6, 128, 4, 20, MSPLAT_BF16X3, 0)
#define MSPLAT_NETS(X) MSPLAT_NETS_NARROW(X) MSPLAT_NETS_WIDE(X)

// the networks of this translation unit, and the suffix of its launchers
#ifdef MSPLAT_WIDE_TU
#define MSPLAT_TU_NETS MSPLAT_NETS_WIDE
#define MSPLAT_TU_FN(name) name##_wide
#else
#define MSPLAT_TU_NETS MSPLAT_NETS_NARROW
#define MSPLAT_TU_FN(name) name##_narrow
#endif
#define MSPLAT_NET(L_, W_, D_, O_, P_, K_) \
  Net<L_, W_, D_, O_, (P_) != MSPLAT_FP32, (P_) == MSPLAT_BF16X3, (K_) == 1>
#define MSPLAT_MATCH(L_, W_, D_, O_, P_, K_) \
  if (n.L == L_ && n.W == W_ && n.D == D_ && n.NOUT == O_ && n.prec == (P_) && n.kind == (K_))

__device__ __forceinline__ f32x16 mfma32(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 mfma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// two floats rounded (to nearest even) into one packed bfloat16 pair, the
// first in the low half
__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, bf16x2));
}
// the two floats of a packed pair
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
// hi + lo split of two floats: hi = bf16(x), lo = bf16(x - hi) (x - hi is exact)
__device__ __forceinline__ void split_pk(float a, float b, uint32_t& hi, uint32_t& lo) {
  hi = pk_bf16(a, b);
  lo = pk_bf16(a - bf16_lo(hi), b - bf16_hi(hi));
}

__device__ __forceinline__ uint4 lds16(const uint8_t* p) { return *reinterpret_cast<const uint4*>(p); }
__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }
__device__ __forceinline__ f32x4 as_f32x4(uint4 v) { return __builtin_bit_cast(f32x4, v); }

// Output activations.  The reciprocal is the hardware one (1 ulp): an IEEE
// division costs about ten vector instructions per call.  log(1 + e) for
// e = exp(-|x|) in (0, 1] is the hardware logarithm of 1 + e, or the series
// e - e^2/2 below 1e-4, where forming 1 + e loses the low bits of e (the
// absolute error stays below 1e-7 either way).
__device__ __forceinline__ float sigmoidf_(float x) { return __builtin_amdgcn_rcpf(1.f + __expf(-x)); }
__device__ __forceinline__ float softplusf_(float x) {
  const float e = __expf(-fabsf(x));
  const float l = e < 1e-4f ? e * (1.f - 0.5f * e) : __logf(1.f + e);
  return fmaxf(x, 0.f) + l;
}

}  // namespace msplat
