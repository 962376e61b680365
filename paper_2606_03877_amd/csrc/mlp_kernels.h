// Device building blocks shared by the forward and backward MLP kernels:
// positional encoding into B-operand slots, one dense layer on the matrix
// cores, ReLU/convert of D registers into the next B operand, segmented scans
// over a block's columns, and the work-item to primitive lookup.
#pragma once

#include <type_traits>

#include "mlp_common.h"

namespace msplat {

// ---------------------------------------------------------- forward chain --

// sample position p = p_c + s e with s = s_a + (k + u) Delta, evaluated in
// double-float arithmetic from the hit's double-float record; returns s (float)
__device__ __forceinline__ float sample_position(const Workspace& ws, int hit, int k, float u, float ph[3],
                                                 float pl[3]) {
  const int64_t H = ws.hit_cap;
  const df ku = two_sum((float)k, u);
  const df dlt = {ws.hit_dlt[hit], ws.hit_dlt_lo[hit]};
  const df s = df_add(df{ws.hit_sa[hit], ws.hit_sa_lo[hit]}, df_mul(ku, dlt));
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const df e = {ws.hit_e[a * H + hit], ws.hit_e_lo[a * H + hit]};
    const df p = df_add(df{ws.hit_pc[a * H + hit], ws.hit_pc_lo[a * H + hit]}, df_mul(s, e));
    ph[a] = p.hi;
    pl[a] = p.lo;
  }
  return s.hi;
}

// sin(pi x), cos(pi x) of x = m (hi + lo) for a power of two m: m hi is exact,
// its reduction modulo 2 is exact, and m lo is added to the reduced argument,
// so the result is accurate to float32 rounding of the reduced argument
template <bool FAST>
__device__ __forceinline__ void sincospi_df(float hi, float lo, float m, float& s, float& c) {
  const float xh = hi * m, xl = lo * m;
  if constexpr (FAST) {
    // hardware sine takes turns: x pi = 2 pi (x / 2)
    float h = 0.5f * xh;
    float r = (h - rintf(h)) + 0.5f * xl;
    s = __builtin_amdgcn_sinf(r);
    c = __builtin_amdgcn_cosf(r);
  } else {
    float r = (xh - 2.f * rintf(0.5f * xh)) + xl;
    s = sinpif(r);
    c = cospif(r);
  }
}

// positional encoding of one sample into the lane half's input slots
template <class N>
__device__ __forceinline__ void encode_slots(const float ph[3], const float pl[3], int g,
                                             float (&v)[N::ENC_KS * N::KSTEP]) {
#pragma unroll
  for (int t = 0; t < N::ENC_KS * N::KSTEP; ++t) v[t] = 0.f;
#pragma unroll
  for (int pr = 0; pr < N::L / 2; ++pr) {
    // level 2*pr + g
    float mul = (float)(1 << (2 * pr)) * (g ? 2.f : 1.f);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float s, c;
      sincospi_df<N::BF16>(ph[a], pl[a], mul, s, c);
      v[6 * pr + a] = s;
      v[6 * pr + 3 + a] = c;
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) v[3 * N::L + a] = g == 0 ? ph[a] : (a == 0 ? 1.f : 0.f);
}

// encoding of the contact-point primitive's input [d; delta] into the lane
// half's input slots (d exact, delta as a double-float)
template <class N>
__device__ __forceinline__ void encode_contact_slots(const float dh[3], const float dl[3], const float dd[3], int g,
                                                     float (&v)[N::ENC_KS * N::KSTEP]) {
#pragma unroll
  for (int t = 0; t < N::ENC_KS * N::KSTEP; ++t) v[t] = 0.f;
#pragma unroll
  for (int pr = 0; pr < N::L / 2; ++pr) {
    // level 2*pr + g
    float mul = (float)(1 << (2 * pr)) * (g ? 2.f : 1.f);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      float sn, cs;
      if (c < 3) sincospi_df<N::BF16>(dd[c], 0.f, mul, sn, cs);
      else sincospi_df<N::BF16>(dh[c - 3], dl[c - 3], mul, sn, cs);
      v[12 * pr + c] = sn;
      v[12 * pr + 6 + c] = cs;
    }
  }
  v[6 * N::L] = g == 1 ? 1.f : 0.f;
}

// the first layer's input of one sample: the encoded local position (ph, pl)
// of a chord sample, or the encoded [dd; delta = (ph, pl)] of a contact point
template <class N>
__device__ __forceinline__ void encode_input(const float ph[3], const float pl[3], const float dd[3], int g,
                                             float (&v)[N::ENC_KS * N::KSTEP]) {
  if constexpr (N::CONTACT) encode_contact_slots<N>(ph, pl, dd, g, v);
  else encode_slots<N>(ph, pl, g, v);
}

// The network input of a hit's sample.  Chord primitives: the sample
// position p = p_c + s e in the local frame (double-float, returns s).
// Contact-point primitive (one sample per hit): the residual delta
// (double-float, in the position arrays) and the ray direction d (in the
// direction arrays); returns 0.
template <class N>
__device__ __forceinline__ float sample_input(const Workspace& ws, int hit, int k, float u, float ph[3], float pl[3],
                                              float dd[3]) {
  if constexpr (N::CONTACT) {
    const int64_t H = ws.hit_cap;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      ph[a] = ws.hit_pc[a * H + hit];
      pl[a] = ws.hit_pc_lo[a * H + hit];
      dd[a] = ws.hit_e[a * H + hit];
    }
    return 0.f;
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a) dd[a] = 0.f;
    return sample_position(ws, hit, k, u, ph, pl);
  }
}

template <class N>
struct Operands {
  // bf16: one bf16x8 per k-step; f32: one float per k-step (padded to groups of 4)
  using BT = typename std::conditional<N::BF16, bf16x8, float>::type;
};

// B operands of one layer input: hi parts, and lo parts in the split form
template <class N, int NK>
struct Act {
  typename Operands<N>::BT hi[NK];
  typename Operands<N>::BT lo[N::SPLIT ? NK : 1];
};

// hi parts only (what the backward keeps of a layer input)
template <class N, int NK>
struct Hi {
  typename Operands<N>::BT hi[NK];
};

// LDS (or global) operands of one row block of a layer: the A groups (hi,
// and lo in the split form) and, for the forward of a hidden or output
// layer, the lane's 16 biases
template <class N, int NG, bool BIAS>
struct RowOps {
  uint4 a[NG];
  uint4 al[N::SPLIT ? NG : 1];
  uint4 b[BIAS ? 4 : 1];
};

template <class N, int NG, bool BIAS>
__device__ __forceinline__ void load_row(const uint8_t* __restrict__ A, const uint8_t* __restrict__ Alo,
                                         const uint8_t* __restrict__ bp, int rb, int lane, RowOps<N, NG, BIAS>& o) {
#pragma unroll
  for (int gi = 0; gi < NG; ++gi) {
    const int idx = ((rb * NG + gi) * 64 + lane) * 16;
    o.a[gi] = lds16(A + idx);
    if constexpr (N::SPLIT) o.al[gi] = lds16(Alo + idx);
  }
  if constexpr (BIAS) {
#pragma unroll
    for (int i = 0; i < 4; ++i) o.b[i] = lds16(bp + 16 * i);
  }
}

// c += A_rb x over the row block's groups (three products per pair in the split form)
template <class N, int NG, bool BIAS, int NK>
__device__ __forceinline__ void row_mfma(const RowOps<N, NG, BIAS>& o, const Act<N, NK>& B, f32x16& c) {
#pragma unroll
  for (int gi = 0; gi < NG; ++gi) {
    if constexpr (N::BF16) {
      c = mfma32(as_bf16x8(o.a[gi]), B.hi[gi], c);
      if constexpr (N::SPLIT) {
        c = mfma32(as_bf16x8(o.a[gi]), B.lo[gi], c);
        c = mfma32(as_bf16x8(o.al[gi]), B.hi[gi], c);
      }
    } else {
      f32x4 a4 = as_f32x4(o.a[gi]);
#pragma unroll
      for (int e = 0; e < 4; ++e) c = mfma32(a4[e], B.hi[4 * gi + e], c);
    }
  }
}

// operands of one row block of forward layer J
template <class N, int J, int KS>
using FwdOps = RowOps<N, N::groups(KS), (J > 0)>;

// Where the forward operands are read: kPacked, the packed layout at wb
// (LDS or global); kHiStaged, the hi sections and biases staged at wb in the
// fwd_hi_* layout, the lo sections read from the packed copy at wlo;
// kHiPrefix + S, the hi sections of layers 0..S-1 staged at wb (fwd_hi_off
// offsets), everything else (the other hi sections, all lo sections, the
// biases) read from the packed copy at wlo.
enum FwdLayout { kPacked = 0, kHiStaged = 1, kHiPrefix = 16 };

template <class N, int J, int KS, int LAYOUT = kPacked>
__device__ __forceinline__ void fwd_row_load(const uint8_t* __restrict__ wb, const uint8_t* __restrict__ wlo,
                                             int lane, int rb, FwdOps<N, J, KS>& o) {
  const int bo = ((lane / 32) * 16) * 4 + rb * 128;
  if constexpr (LAYOUT == kHiStaged) {
    load_row<N, N::groups(KS), (J > 0)>(wb + N::fwd_hi_off(J), wlo + N::fwdA_off(J) + N::fwdA_single(J),
                                        wb + N::fwd_hi_bias(J) + bo, rb, lane, o);
  } else if constexpr (LAYOUT >= kHiPrefix) {
    const uint8_t* P = wlo + N::fwdA_off(J);
    if constexpr (J < LAYOUT - kHiPrefix)
      load_row<N, N::groups(KS), (J > 0)>(wb + N::fwd_hi_off(J), P + N::fwdA_single(J), wlo + N::bias_off(J) + bo,
                                          rb, lane, o);
    else
      load_row<N, N::groups(KS), (J > 0)>(P, P + N::fwdA_single(J), wlo + N::bias_off(J) + bo, rb, lane, o);
  } else {
    const uint8_t* A = wb + N::fwdA_off(J);
    load_row<N, N::groups(KS), (J > 0)>(A, A + N::fwdA_single(J), wb + N::bias_off(J) + bo, rb, lane, o);
  }
}

// one dense layer on the matrix cores: acc[rb] = bias + W_j x, given the
// operands of row block 0 (`first`).  `wb` is the primitive's packed
// operands, staged in LDS or in global memory.  The operands of row block
// rb+1 are requested before the products of row block rb, so their latency
// overlaps the matrix cores' work; at most two row blocks' operands are in
// flight (bounds register pressure).
template <class N, int J, int KS, int LAYOUT = kPacked>
__device__ __forceinline__ void layer_fwd_from(const uint8_t* __restrict__ wb, const uint8_t* __restrict__ wlo,
                                               int lane, const Act<N, rup(KS, N::KGRP)>& B,
                                               f32x16 (&acc)[N::frb(J)], const FwdOps<N, J, KS>& first) {
  constexpr int RB = N::frb(J);
  constexpr int NG = N::groups(KS);
  constexpr bool BIAS = J > 0;
  FwdOps<N, J, KS> ops[2];
  ops[0] = first;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    if (rb + 1 < RB) fwd_row_load<N, J, KS, LAYOUT>(wb, wlo, lane, rb + 1, ops[(rb + 1) & 1]);
    const FwdOps<N, J, KS>& o = ops[rb & 1];
    f32x16 c;
    if constexpr (BIAS) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        f32x4 b = as_f32x4(o.b[i]);
#pragma unroll
        for (int e = 0; e < 4; ++e) c[4 * i + e] = b[e];
      }
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) c[e] = 0.f;
    }
    row_mfma<N, NG, BIAS>(o, B, c);
    acc[rb] = c;
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <class N, int J, int KS, int LAYOUT = kPacked>
__device__ __forceinline__ void layer_fwd(const uint8_t* __restrict__ wb, const uint8_t* __restrict__ wlo,
                                          int lane, const Act<N, rup(KS, N::KGRP)>& B,
                                          f32x16 (&acc)[N::frb(J)]) {
  FwdOps<N, J, KS> first;
  fwd_row_load<N, J, KS, LAYOUT>(wb, wlo, lane, 0, first);
  layer_fwd_from<N, J, KS, LAYOUT>(wb, wlo, lane, B, acc, first);
}
template <class N, int J, int KS>
__device__ __forceinline__ void layer_fwd(const uint8_t* __restrict__ wb, int lane,
                                          const Act<N, rup(KS, N::KGRP)>& B, f32x16 (&acc)[N::frb(J)]) {
  layer_fwd<N, J, KS, kPacked>(wb, wb, lane, B, acc);
}

// k-step s of a bfloat16 B operand from its 8 slot values, converted in pairs
template <class N, int NK>
__device__ __forceinline__ void act_set8(Act<N, NK>& a, int s, const float (&x)[8]) {
  uint4 h, l;
  split_pk(x[0], x[1], h.x, l.x);
  split_pk(x[2], x[3], h.y, l.y);
  split_pk(x[4], x[5], h.z, l.z);
  split_pk(x[6], x[7], h.w, l.w);
  a.hi[s] = as_bf16x8(h);
  if constexpr (N::SPLIT) a.lo[s] = as_bf16x8(l);
}
template <class N, int NK>
__device__ __forceinline__ void act_set8_hi(Act<N, NK>& a, int s, const float (&x)[8]) {
  uint4 h;
  h.x = pk_bf16(x[0], x[1]);
  h.y = pk_bf16(x[2], x[3]);
  h.z = pk_bf16(x[4], x[5]);
  h.w = pk_bf16(x[6], x[7]);
  a.hi[s] = as_bf16x8(h);
}
// B operand of NKS k-steps from slot values v(t) (t = KSTEP s + e)
template <class N, int NK, class F>
__device__ __forceinline__ void act_fill(Act<N, NK>& a, F v) {
#pragma unroll
  for (int s = 0; s < NK; ++s) {
    if constexpr (N::BF16) {
      float x[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = v(8 * s + e);
      if constexpr (N::SPLIT) act_set8<N, NK>(a, s, x);
      else act_set8_hi<N, NK>(a, s, x);
    } else {
      a.hi[s] = v(s);
    }
  }
}

// max(x, 0) as an integer maximum of the bit pattern (negative floats, -0
// included, are negative integers): one instruction, where a float maximum
// also canonicalises its operand
__device__ __forceinline__ float relu(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

// ReLU and conversion of a hidden layer's D registers into the next B operand
template <class N>
__device__ __forceinline__ void relu_to_B(const f32x16 (&acc)[N::RBH],
                                          Act<N, rup(N::HID_KS, N::KGRP)>& B) {
  act_fill<N, rup(N::HID_KS, N::KGRP)>(B, [&](int t) { return t < 16 * N::RBH ? relu(acc[t / 16][t % 16]) : 0.f; });
}

// ReLU gates of a hidden layer's D registers as bits (slot t = 16 rb + r)
template <class N>
struct Gates {
  uint32_t w[(16 * N::RBH + 31) / 32];
};
template <class N>
__device__ __forceinline__ void gates_of(const f32x16 (&acc)[N::RBH], Gates<N>& m) {
#pragma unroll
  for (int i = 0; i < (16 * N::RBH + 31) / 32; ++i) m.w[i] = 0u;
#pragma unroll
  for (int rb = 0; rb < N::RBH; ++rb) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      int t = 16 * rb + r;
      if (acc[rb][r] > 0.f) m.w[t / 32] |= 1u << (t % 32);
    }
  }
}

// encoding slots of one sample into the first layer's B operand
template <class N>
__device__ __forceinline__ void enc_to_B(const float (&ev)[N::ENC_KS * N::KSTEP],
                                         Act<N, rup(N::ENC_KS, N::KGRP)>& B) {
  act_fill<N, rup(N::ENC_KS, N::KGRP)>(B, [&](int t) { return t < N::ENC_KS * N::KSTEP ? ev[t] : 0.f; });
}

// ------------------------------------------------------ cross-lane moves --
//
// A block's 32 columns sit in lanes 0-31 and again in lanes 32-63 (the two
// lane halves hold different rows of the same samples).  The moves below run
// on the vector ALU (DPP row shifts and broadcasts, the 32-lane half swap and
// lane reads into scalar registers) instead of the LDS permute path, whose
// latency a single wave per SIMD cannot hide.

template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, true);
}
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(dpp_i<CTRL, ROWS>(__float_as_int(v)));
}
// value of the lane D below within the 16-lane row (0 where that leaves the row)
template <int D>
__device__ __forceinline__ float row_shr(float v) { return dpp_f<0x110 + D>(v); }
template <int D>
__device__ __forceinline__ int row_shr_i(int v) { return dpp_i<0x110 + D>(v); }
// lanes of rows 1 and 3 (columns 16-31 of each half) receive lane 15 of the
// row below; rows 0 and 2 receive 0
__device__ __forceinline__ float row_bcast15(float v) { return dpp_f<0x142, 0xA>(v); }
__device__ __forceinline__ int row_bcast15_i(int v) { return dpp_i<0x142, 0xA>(v); }

// both halves receive the lower half's value of the same column
__device__ __forceinline__ float from_lower_half(float v) {
  auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]);
}
// each half receives the other half's value of the same column
__device__ __forceinline__ float other_half(float v, int g) {
  auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(g ? r[0] : r[1]);
}
// column 31 of the lane's own half
__device__ __forceinline__ float col31(float v, int g) {
  float lo = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(v), 31));
  float hi = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(v), 63));
  return g ? hi : lo;
}
// column 31 where both halves hold the same values
__device__ __forceinline__ float col31_same(float v) {
  return __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(v), 31));
}

// ------------------------------------------------------ segmented scans --

// segmented inclusive scan over the 32 columns of a lane half: four shift
// steps inside each 16-lane row, then the rows of columns 16-31 add the
// running sum of column 15 where no segment head lies between
struct SegScan {
  uint32_t mask;   // bit i < 4: add the column 2^i below at step i; bit 4: add column 15
  bool seen_head;  // a segment head lies at or before this column
  __device__ __forceinline__ SegScan(bool head, int col) {
    int f = head;
    mask = 0;
    const int c16 = col & 15;
    int fp;
    fp = row_shr_i<1>(f);
    if (c16 >= 1) { if (!f) mask |= 1u; f |= fp; }
    fp = row_shr_i<2>(f);
    if (c16 >= 2) { if (!f) mask |= 2u; f |= fp; }
    fp = row_shr_i<4>(f);
    if (c16 >= 4) { if (!f) mask |= 4u; f |= fp; }
    fp = row_shr_i<8>(f);
    if (c16 >= 8) { if (!f) mask |= 8u; f |= fp; }
    fp = row_bcast15_i(f);
    if (col >= 16) { if (!f) mask |= 16u; f |= fp; }
    seen_head = f != 0;
  }
  __device__ __forceinline__ float incl(float v) const {
    float vp;
    vp = row_shr<1>(v);
    if (mask & 1u) v += vp;
    vp = row_shr<2>(v);
    if (mask & 2u) v += vp;
    vp = row_shr<4>(v);
    if (mask & 4u) v += vp;
    vp = row_shr<8>(v);
    if (mask & 8u) v += vp;
    vp = row_bcast15(v);
    if (mask & 16u) v += vp;
    return v;
  }
};

// the column below's value within the lane half (column 0 receives 0)
__device__ __forceinline__ float col_below(float v, int col) {
  float a = row_shr<1>(v), b = row_bcast15(v);
  return (col & 15) ? a : (col ? b : 0.f);
}

// wave priority over a matrix-core stretch: raised, the wave's matrix
// instructions issue ahead of the other waves' vector work on its SIMD.
// Wide networks run one wave per SIMD, where it only lengthens live ranges.
template <class N, int P>
__device__ __forceinline__ void mfma_priority() {
  if constexpr (!N::WIDE) __builtin_amdgcn_s_setprio(P);
}

// bitonic sort of one value per lane over the wave, largest in lane 0
__device__ __forceinline__ int wave_sort_desc(int v, int lane) {
#pragma unroll
  for (int kk = 2; kk <= 64; kk <<= 1) {
#pragma unroll
    for (int j = kk >> 1; j > 0; j >>= 1) {
      const int o = __shfl_xor(v, j, 64);
      const bool keep_max = ((lane & kk) == 0) == ((lane & j) == 0);
      v = keep_max ? max(v, o) : min(v, o);
    }
  }
  return v;
}

// A run of up to 64 NW hits dealt to the NW waves of a workgroup so that the
// waves' sample counts balance (a workgroup lasts as long as its busiest
// wave).  Thread (wave w, lane l) brings the key of run hit i = 64 w + l:
// (k_i << 9) | (511 - i), k_i its sample count, or -1 past the run.  Wave w
// sorts its 64 keys, largest first; rank r of that list goes to wave
// (snake(r) + w) mod NW, snake(r) running 0..NW-1 and back over each row of
// NW ranks; the table `tab` (64 NW ints of LDS) carries them; each wave
// sorts what it received.  Returns the run index of the hit in lane `lane`
// of wave `w` (-1: none; the hits fill lanes 0..c-1) and its count in k.
// Every thread of the workgroup calls it (it holds a barrier).
template <int NW>
__device__ __forceinline__ int deal_run(int key, int* tab, int w, int lane, int& k) {
  static_assert(64 * NW <= 512, "run indices fit 9 bits");
  tab[64 * w + lane] = wave_sort_desc(key, lane);
  __syncthreads();
  constexpr int PER = 64 / NW;   // keys a wave takes from each wave's list
  const int qc = lane / PER, j = lane % PER;
  const int sp = (w - qc + NW) % NW;
  const int r = j * NW + ((j & 1) ? NW - 1 - sp : sp);
  const int got = wave_sort_desc(tab[64 * qc + r], lane);
  k = got < 0 ? 0 : got >> 9;
  return got < 0 ? -1 : 511 - (got & 511);
}

__device__ __forceinline__ int find_prim(const int32_t* __restrict__ wi_off, int P, int wi) {
  int lo = 0, hi = P;   // wi_off[lo] <= wi < wi_off[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (wi_off[mid] <= wi) lo = mid; else hi = mid;
  }
  return lo;
}


}  // namespace msplat
