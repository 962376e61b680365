// Device building blocks shared by the forward and backward MLP kernels:
// positional encoding into B-operand slots, one dense layer on the matrix
// cores, ReLU/convert of D registers into the next B operand, segmented scans
// over a block's columns, and the work-item to primitive lookup.
#pragma once

#include <type_traits>

#include "mlp_common.h"

namespace msplat {

// ---------------------------------------------------------- forward chain --

// positional encoding of one sample into the lane half's input slots
template <class N>
__device__ __forceinline__ void encode_slots(const float p[3], int g, float (&v)[N::ENC_KS * N::KSTEP]) {
#pragma unroll
  for (int t = 0; t < N::ENC_KS * N::KSTEP; ++t) v[t] = 0.f;
#pragma unroll
  for (int pr = 0; pr < N::L / 2; ++pr) {
    // level 2*pr + g
    float mul = (float)(1 << (2 * pr)) * (g ? 2.f : 1.f);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float s, c;
      sincospi_<N::BF16>(p[a] * mul, s, c);
      v[6 * pr + a] = s;
      v[6 * pr + 3 + a] = c;
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) v[3 * N::L + a] = g == 0 ? p[a] : (a == 0 ? 1.f : 0.f);
}

template <class N>
struct Operands {
  // bf16: one bf16x8 per k-step; f32: one float per k-step (padded to groups of 4)
  using BT = typename std::conditional<N::BF16, bf16x8, float>::type;
};

// one dense layer on the matrix cores: acc[rb] = bias + W_j x
template <class N, int J, int KS>
__device__ __forceinline__ void layer_fwd(const uint8_t* __restrict__ lds, int lane,
                                          const typename Operands<N>::BT (&B)[rup(KS, N::KGRP)],
                                          f32x16 (&acc)[N::frb(J)]) {
  constexpr int RB = N::frb(J);
  constexpr int NG = N::groups(KS);
  const uint8_t* A = lds + N::fwdA_off(J);
  int g = lane / 32;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    f32x16 c;
    if constexpr (J > 0) {
      const uint8_t* bp = lds + N::bias_off(J) + ((rb * 2 + g) * 16) * 4;
      f32x4 b0 = as_f32x4(lds16(bp)), b1 = as_f32x4(lds16(bp + 16)), b2 = as_f32x4(lds16(bp + 32)),
            b3 = as_f32x4(lds16(bp + 48));
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        c[e] = b0[e];
        c[4 + e] = b1[e];
        c[8 + e] = b2[e];
        c[12 + e] = b3[e];
      }
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) c[e] = 0.f;
    }
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
      uint4 raw = lds16(A + ((rb * NG + gi) * 64 + lane) * 16);
      if constexpr (N::BF16) {
        c = mfma32(as_bf16x8(raw), B[gi], c);
      } else {
        f32x4 a4 = as_f32x4(raw);
#pragma unroll
        for (int e = 0; e < 4; ++e) c = mfma32(a4[e], B[4 * gi + e], c);
      }
    }
    acc[rb] = c;
  }
}

// ReLU and conversion of a hidden layer's D registers into the next B operand
template <class N>
__device__ __forceinline__ void relu_to_B(const f32x16 (&acc)[N::RBH],
                                          typename Operands<N>::BT (&B)[rup(N::HID_KS, N::KGRP)]) {
#pragma unroll
  for (int rb = 0; rb < N::RBH; ++rb) {
    if constexpr (N::BF16) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        bf16x8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (__bf16)fmaxf(acc[rb][8 * h + e], 0.f);
        B[2 * rb + h] = v;
      }
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r) B[16 * rb + r] = fmaxf(acc[rb][r], 0.f);
    }
  }
}

// ------------------------------------------------------ segmented scans --

// step masks of a segmented inclusive scan over the 32 columns of a lane half
struct SegScan {
  uint32_t mask;   // bit i: add the value from column - 2^i at step i
  bool seen_head;  // a segment head lies at or before this column
  __device__ __forceinline__ SegScan(bool head, int col) {
    bool f = head;
    mask = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      int d = 1 << i;
      int fp = __shfl_up((int)f, d, 32);
      if (col >= d) {
        if (!f) mask |= 1u << i;
        f = f || fp;
      }
    }
    seen_head = f;
  }
  __device__ __forceinline__ float incl(float v) const {
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      float vp = __shfl_up(v, 1 << i, 32);
      if (mask & (1u << i)) v += vp;
    }
    return v;
  }
};

__device__ __forceinline__ int find_prim(const int32_t* __restrict__ wi_off, int P, int wi) {
  int lo = 0, hi = P;   // wi_off[lo] <= wi < wi_off[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (wi_off[mid] <= wi) lo = mid; else hi = mid;
  }
  return lo;
}


}  // namespace msplat
