// closure.hpp -- per-node MLP closure: feature map and the wave-level BF16 MFMA
// evaluation shared by the fused stream-collide kernel and the stand-alone
// evaluation kernel.
//
// Network: x (27) -> relu(W1 x + b1) (64) -> relu(W2 h1 + b2) (64) -> W3 h2 + b3 (6).
// A wavefront evaluates it for its 64 nodes at once as three products with the
// 64 nodes as the N dimension, on v_mfma_f32_32x32x16_bf16:
//   layer 1: [64 x 32] (W1, K padded 27 -> 32) x [32 x 64 nodes]
//   layer 2: [64 x 64] x [64 x 64 nodes]
//   layer 3: [32 x 64] (W3, 6 rows used) x [64 x 64 nodes]
// Lane layouts (checked on gfx950): A lane l holds row l%32, k = 8(l/32)+i;
// B lane l holds column l%32, k = 8(l/32)+i; accumulator element j of lane l
// is row 8(j/4) + 4(l/32) + j%4, column l%32.  So the ReLU'd accumulators of
// one layer are used in place as the B operand of the next, provided the next
// layer's weights are packed with the hidden units in the order unit(q, h, i)
// below.  Inputs reach the MFMA layout through a per-wave LDS tile; the six
// outputs of a node are gathered back to its lane with one cross-half swap.
// Weights and biases live in LDS (PACKED_BYTES per block), fp32 accumulation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "d3q27.hpp"
#include "fpc_collide.hpp"

namespace fpc {
namespace cl {

constexpr int NIN = 27, NH = 64, NOUT = 6, NPARAM = 6342;
constexpr int OFF_W1 = 0, OFF_B1 = NH * NIN, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NOUT * NH;
constexpr int NFRAG = 16;                        // A fragments: 4 (layer 1), 8 (layer 2), 4 (layer 3)
constexpr int AFRAG_BYTES = NFRAG * 64 * 16;     // 64 lanes x 8 bf16 each
constexpr int NBIAS = 5;                         // bias blocks: L1 mb0/mb1, L2 mb0/mb1, L3
constexpr int BIAS_BYTES = NBIAS * 2 * 16 * 4;   // per block: 2 lane halves x 16 floats
constexpr int PACKED_BYTES = AFRAG_BYTES + BIAS_BYTES;
constexpr int XROW = 40;                         // bf16 per LDS feature row (32 used; padded)
constexpr int XTILE = 64 * XROW;                 // bf16 per wave

// Hidden unit carried by slot i of lane half h in K-block q (16 rows) of layers
// 2 and 3: the row that element j = 8 (q%2) + i of the previous layer's
// accumulator block q/2 holds.
__host__ __device__ constexpr int unit(int q, int h, int i) {
  return 32 * (q / 2) + 16 * (q % 2) + 8 * (i / 4) + 4 * h + (i % 4);
}

// Feature normalisation 3^((a+b+c)/2) = 1 / c_s^(order) by moment order.
__host__ __device__ constexpr float order_norm(int order) {
  return order == 0 ? 1.0f : order == 1 ? 1.7320508075688772f : order == 2 ? 3.0f
       : order == 3 ? 5.196152422706632f : order == 4 ? 9.0f : order == 5 ? 15.588457268119896f : 27.0f;
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// features from the primed pre-collision cube (v[c][b][a] = kappa'_abc):
// x_000 = rho - 1, x_100 = x_010 = x_001 = 0 (the first-order central moments
// are -F/2 at every node: no information, only FP32 rounding noise),
// x_abc = (kappa'_abc - rho' E_abc) / rho * 3^((a+b+c)/2), in the paper's
// moment order.
// The factor 3^(order/2) / rho is formed once per order, so each feature takes
// one multiply; 1 / rho is the collision's own (recip_rho), computed once.
template <typename T>
__device__ __forceinline__ void features(const T (&v)[3][3][3], T rhop, T rho, float (&x)[NIN]) {
  constexpr int MM[NIN][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1},
                              {2, 0, 0}, {0, 2, 0}, {0, 0, 2}, {1, 2, 0}, {1, 0, 2}, {2, 1, 0}, {0, 1, 2},
                              {2, 0, 1}, {0, 2, 1}, {1, 1, 1}, {2, 2, 0}, {2, 0, 2}, {0, 2, 2}, {2, 1, 1},
                              {1, 2, 1}, {1, 1, 2}, {1, 2, 2}, {2, 1, 2}, {2, 2, 1}, {2, 2, 2}};
  (void)rho;
  const T ir = recip_rho<T>(rhop);
  T irn[7];
#pragma unroll
  for (int o = 2; o < 7; ++o) irn[o] = ir * T(order_norm(o));
  x[0] = (float)rhop;
  x[1] = x[2] = x[3] = 0.0f;
#pragma unroll
  for (int k = 4; k < NIN; ++k) {
    const int a = MM[k][0], b = MM[k][1], c = MM[k][2];
    const double E = C1[a] * C1[b] * C1[c];
    const T kap = v[c][b][a];
    const T d = (E == 0.0) ? kap : kap - rhop * T(E);
    x[k] = (float)(d * irn[a + b + c]);
  }
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x16 load_bias(const char* w, int blk, int h) {
  const float4* p = (const float4*)(w + AFRAG_BYTES + (blk * 2 + h) * 64);
  const float4 a = p[0], b = p[1], c = p[2], d = p[3];
  f32x16 r;
  r[0] = a.x; r[1] = a.y; r[2] = a.z; r[3] = a.w;
  r[4] = b.x; r[5] = b.y; r[6] = b.z; r[7] = b.w;
  r[8] = c.x; r[9] = c.y; r[10] = c.z; r[11] = c.w;
  r[12] = d.x; r[13] = d.y; r[14] = d.z; r[15] = d.w;
  return r;
}

__device__ __forceinline__ bf16x8 load_afrag(const char* w, int f, int lane) {
  return *(const bf16x8*)(w + (f * 64 + lane) * 16);
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// elements 8 q' .. 8 q' + 7 of an accumulator block, ReLU'd, as a B fragment.
// Rounding to bf16 (nearest even) and ReLU commute for finite values, so each
// pair is converted with one packed conversion and the ReLU is a packed signed
// 16-bit max with 0 on the bf16 bit patterns (negative values, -0 included,
// have the sign bit).
__device__ __forceinline__ bf16x8 relu_bf16(const f32x16& acc, int qp) {
  u32x4 w;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const f32x2 f = {acc[8 * qp + 2 * i], acc[8 * qp + 2 * i + 1]};
    const bf16x2 p = __builtin_convertvector(f, bf16x2);
    w[i] = __builtin_bit_cast(unsigned, __builtin_elementwise_max(__builtin_bit_cast(s16x2, p), s16x2{0, 0}));
  }
  return __builtin_bit_cast(bf16x8, w);
}

// Evaluate the MLP for the 64 nodes of the calling wavefront.  Every lane of
// the wave must call it (MFMA and the LDS tile are wave-wide).  w: packed
// parameters (LDS), xs: this wave's LDS tile of XTILE bf16.
__device__ __forceinline__ void mlp_wave(const float (&x)[NIN], float (&out)[NOUT], const char* __restrict__ w,
                                         __bf16* __restrict__ xs) {
  const int l = threadIdx.x & 63, h = l >> 5, r = l & 31;
  {
    bf16x8 t[4];
#pragma unroll
    for (int k = 0; k < 32; ++k) t[k / 8][k % 8] = (__bf16)(k < NIN ? x[k] : 0.0f);
    wave_lds_sync();  // previous readers of the tile are done
#pragma unroll
    for (int c = 0; c < 4; ++c) *(bf16x8*)(xs + l * XROW + 8 * c) = t[c];
    wave_lds_sync();
  }
  // layer 1 -> B fragments of layer 2: h1[nb][q]
  bf16x8 h1[2][4];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb) {
    const f32x16 bias = load_bias(w, mb, h);
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      f32x16 acc = bias;
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        const bf16x8 b = *(const bf16x8*)(xs + (nb * 32 + r) * XROW + 16 * kb + 8 * h);
        acc = mfma(load_afrag(w, mb * 2 + kb, l), b, acc);
      }
      h1[nb][2 * mb] = relu_bf16(acc, 0);
      h1[nb][2 * mb + 1] = relu_bf16(acc, 1);
    }
  }
  // layer 2 -> B fragments of layer 3
  bf16x8 h2[2][4];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb) {
    const f32x16 bias = load_bias(w, 2 + mb, h);
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      f32x16 acc = bias;
#pragma unroll
      for (int q = 0; q < 4; ++q) acc = mfma(load_afrag(w, 4 + mb * 4 + q, l), h1[nb][q], acc);
      h2[nb][2 * mb] = relu_bf16(acc, 0);
      h2[nb][2 * mb + 1] = relu_bf16(acc, 1);
    }
  }
  // layer 3 (rows 0..5 used)
  f32x16 o[2];
  const f32x16 bias3 = load_bias(w, 4, h);
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    o[nb] = bias3;
#pragma unroll
    for (int q = 0; q < 4; ++q) o[nb] = mfma(load_afrag(w, 12 + q, l), h2[nb][q], o[nb]);
  }
  // node n = 32 nb + r: outputs 0..3 sit in lane r (block nb), outputs 4..5 in
  // lane r + 32 (block nb); swap the halves so that lane n holds all six.
  float recv[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) recv[j] = __shfl_xor(h ? o[0][j] : o[1][j], 32, 64);
  if (h == 0) {
    out[0] = o[0][0]; out[1] = o[0][1]; out[2] = o[0][2]; out[3] = o[0][3];
    out[4] = recv[0]; out[5] = recv[1];
  } else {
    out[0] = recv[0]; out[1] = recv[1]; out[2] = recv[2]; out[3] = recv[3];
    out[4] = o[1][0]; out[5] = o[1][1];
  }
}

}  // namespace cl
}  // namespace fpc
