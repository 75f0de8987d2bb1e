// lbm_internal.hpp -- pieces shared by the translation units of liblbm.so
// (storage forms, the context, error handling, launch shapes).  Not part of
// the public interface (include/lbm.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/lbm.h"
#include "d3q27.hpp"
#include "fpc_collide.hpp"

using namespace fpc;

// ===========================================================================
// storage forms
template <int ST>
struct Stor;

template <>
struct Stor<LBM_F64> {
  using S = double;
  using R = double;
  static __device__ __forceinline__ R dec(S s, int) { return s; }
  // f: exact power of two still carried by r (see inverse_all)
  static constexpr bool stochastic = false;
  static __device__ __forceinline__ S enc(R r, int, double f = 1.0, uint32_t = 0) { return r * f; }
  static __device__ __forceinline__ S enc_nearest(R r, int a, double f = 1.0) { return enc(r, a, f); }
};

template <>
struct Stor<LBM_F32> {
  using S = float;
  using R = float;
  static __device__ __forceinline__ R dec(S s, int) { return s; }
  static constexpr bool stochastic = false;
  static __device__ __forceinline__ S enc(R r, int, double f = 1.0, uint32_t = 0) { return r * (float)f; }
  static __device__ __forceinline__ S enc_nearest(R r, int a, double f = 1.0) { return enc(r, a, f); }
};

// FP16 / BF16 deviation storage.  SR = true: stochastic rounding with the
// gfx950 conversions v_cvt_sr_{f16,bf16}_f32, which compare the dropped bits
// with the high bits of a random word (E[round(x)] = x), so that increments
// smaller than half an ulp (a small body force, slow viscous change) are kept
// on average instead of being rounded away.  SR = false: round to nearest even.
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

template <bool SR>
struct StorF16 {
  using S = _Float16;
  using R = float;
  static constexpr bool stochastic = SR;
  static __device__ __forceinline__ R dec(S s, int a) { return (float)s * (1.0f / dev_scale(a)); }
  static __device__ __forceinline__ S enc(R r, int a, double f = 1.0, uint32_t rnd = 0) {
    const float x = r * (float)(dev_scale(a) * f);
    if (SR) {
      f16x2_t h = {};
      h = __builtin_amdgcn_cvt_sr_f16_f32(h, x, rnd, false);
      return h[0];
    }
    return (_Float16)x;  // round to nearest even (default mode)
  }
  static __device__ __forceinline__ S enc_nearest(R r, int a, double f = 1.0) {
    return (_Float16)(r * (float)(dev_scale(a) * f));
  }
};

template <bool SR>
struct StorBF16 {
  using S = uint16_t;
  using R = float;
  static constexpr bool stochastic = SR;
  static __device__ __forceinline__ R dec(S s, int a) {
    return __uint_as_float((uint32_t)s << 16) * (1.0f / dev_scale(a));
  }
  static __device__ __forceinline__ S enc(R r, int a, double f = 1.0, uint32_t rnd = 0) {
    const float x = r * (float)(dev_scale(a) * f);
    if (SR) {
      bf16x2_t h = {};
      h = __builtin_amdgcn_cvt_sr_bf16_f32(h, x, rnd, false);
      return __builtin_bit_cast(uint16_t, h[0]);
    }
    return __builtin_bit_cast(uint16_t, (__bf16)x);  // v_cvt_pk_bf16_f32: nearest even
  }
  static __device__ __forceinline__ S enc_nearest(R r, int a, double f = 1.0) {
    return __builtin_bit_cast(uint16_t, (__bf16)(r * (float)(dev_scale(a) * f)));
  }
};

template <> struct Stor<LBM_F16DEV> : StorF16<true> {};
template <> struct Stor<LBM_BF16DEV> : StorBF16<true> {};
template <> struct Stor<LBM_F16DEV_RNE> : StorF16<false> {};
template <> struct Stor<LBM_BF16DEV_RNE> : StorBF16<false> {};

// random word of the stored values of one node in one step: a published
// 32-bit integer hash (lowbias32) of the node's byte offset and the step,
// plus a golden-ratio Weyl increment per direction (its high bits, the ones
// the conversions use, are well spread)
__device__ __forceinline__ uint32_t node_hash(uint32_t node, uint32_t step) {
  uint32_t h = node ^ (step * 0x9E3779B1u + 0x7F4A7C15u);
  h ^= h >> 16;
  h *= 0x7FEB352Du;
  h ^= h >> 15;
  h *= 0x846CA68Bu;
  h ^= h >> 16;
  return h;
}

struct Geom {
  int nx, ny, nz;
  int64_t stride;  // values between direction arrays
};

template <typename T>
struct StepArgs {
  Geom g;
  Rates<T> r;
  T F[3];
  uint32_t step;  // completed steps before this one (random words of SR storage)
};

// ===========================================================================
// streaming (Appendix D Step 6), pull form, shared by every kernel that reads a
// time level: f_alpha(x) = f~_alpha(x - e_alpha), periodic wrap, and halfway
// bounce-back across the y walls (the node's own opposite population).
//
// ROW = true: the block is one segment of an x row, so y and z are uniform
// across the wavefront and every row/plane offset lives in scalar registers;
// the only per-lane address terms are the three x offsets.  ROW = false: 2D
// blocks (small nx), y per lane.  Addresses are a uniform 64-bit base per
// direction plus a 32-bit per-lane byte offset (one direction array is
// < 4 GiB, checked at creation).  Returns the byte offset of node (x, y, z).
template <int ST, bool WALLS, bool ROW>
__device__ __forceinline__ uint32_t pull(const typename Stor<ST>::S* __restrict__ src, const Geom& g, int x, int y,
                                         int z, typename Stor<ST>::R (&v)[3][3][3]) {
  using T = typename Stor<ST>::R;
  using S = typename Stor<ST>::S;
  using SS = Stor<ST>;
  constexpr uint32_t SZ = sizeof(S);
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  // rows away from the walls (all but two per plane) take the wall-free gather,
  // whose loads keep the scalar-base form; the branch is wavefront-uniform
  if (ROW && WALLS && y > 0 && y < ny - 1) return pull<ST, false, true>(src, g, x, y, z, v);
  const uint32_t rowb = (uint32_t)nx * SZ;
  const uint32_t planeb = rowb * (uint32_t)ny;
  // byte offsets of the source x, y, z for e = -1, 0, +1 (periodic wrap)
  const uint32_t x0 = (uint32_t)x * SZ;
  const uint32_t xb[3] = {x == nx - 1 ? 0u : x0 + SZ, x0, x == 0 ? rowb - SZ : x0 - SZ};
  const uint32_t y0 = (uint32_t)y * rowb;
  const uint32_t yb[3] = {y == ny - 1 ? 0u : y0 + rowb, y0, y == 0 ? planeb - rowb : y0 - rowb};
  const uint32_t z0 = (uint32_t)z * planeb;
  const uint32_t zb[3] = {z == nz - 1 ? 0u : z0 + planeb, z0, z == 0 ? (uint32_t)(nz - 1) * planeb : z0 - planeb};
  const uint64_t stb = (uint64_t)g.stride * SZ;
  const char* __restrict__ sb = (const char*)src;
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const int ex = EX[a], ey = EY[a], ez = EZ[a];
    // halfway bounce-back: if x - e_alpha is a wall node, take the node's own
    // opposite population (same weight, so the deviation carries over)
    const bool bb = WALLS && ((ey == 1 && y == 0) || (ey == -1 && y == ny - 1));
    const int o = opposite(a);
    T val;
    if (ROW) {
      // bb is uniform here: the base is chosen in scalar registers
      const char* base = bb ? sb + o * stb + (uint64_t)(z0 + y0) : sb + a * stb + (uint64_t)(zb[ez + 1] + yb[ey + 1]);
      const uint32_t off = bb ? x0 : xb[ex + 1];
      val = SS::dec(*(const S*)(base + off), a);  // w_opp = w_alpha, scales equal
    } else if (bb) {
      val = SS::dec(*(const S*)(sb + o * stb + (uint32_t)(z0 + y0 + x0)), o);
    } else {
      val = SS::dec(*(const S*)(sb + a * stb + (uint32_t)(zb[ez + 1] + yb[ey + 1] + xb[ex + 1])), a);
    }
    v[ez + 1][ey + 1][ex + 1] = val;
  }
  return z0 + y0 + x0;
}

// store the post-collision cube (deviations times 2^inv_shift) at byte offset ib
// ROW: the row's byte offset (uniform) is folded into a scalar base that walks
// the 27 direction arrays; the per-lane part is the x offset only.
template <int ST, bool ROW>
__device__ __forceinline__ void push(typename Stor<ST>::S* __restrict__ dst, const Geom& g, int x, int y, int z,
                                     uint32_t ib, const typename Stor<ST>::R (&v)[3][3][3], uint32_t step) {
  using S = typename Stor<ST>::S;
  constexpr uint32_t SZ = sizeof(S);
  const uint64_t stb = (uint64_t)g.stride * SZ;
  const uint32_t h = Stor<ST>::stochastic ? node_hash(ib, step) : 0u;
  const uint32_t xoff = (uint32_t)x * SZ;
  char* base = (char*)dst + (ROW ? (uint64_t)(((uint32_t)z * (uint32_t)g.ny + (uint32_t)y) * (uint32_t)g.nx * SZ) : 0);
  const uint32_t off = ROW ? xoff : ib;
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    *(S*)(base + off) = Stor<ST>::enc(v[EZ[a] + 1][EY[a] + 1][EX[a] + 1], a, inv_factor(a), h + (uint32_t)a * 0x9E3779B9u);
    base += stb;
  }
}

// ===========================================================================
// context
struct lbm_ctx {
  lbm_config cfg;
  int device = 0;
  int64_t n = 0, stride = 0;
  size_t elem = 0;
  void* buf[2] = {nullptr, nullptr};
  int cur = 0;  // buffer holding the current post-collision state
  bool initialised = false;
  int64_t steps = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  double omega[LBM_Q];
  double* scratch = nullptr;  // 4 N doubles for moments / diagnostics
  double* part = nullptr;     // DIAG_BLOCKS * (NP + 1) + NP doubles
  double* host_out = nullptr; // pinned NP doubles
  char err[512] = {0};
  // learned closure (closure.hip): packed BF16 parameters on the device, NULL = plain method
  char* closure = nullptr;
  float closure_inv_w[6] = {0, 0, 0, 0, 0, 0};  // 1 / omega_4..9
};

int set_err(lbm_ctx* c, int code, const char* fmt, ...);
bool step_launch_shape(int nx, int ny, int nz, dim3& block, dim3& grid);
size_t elem_size(int st);
int alloc_scratch(lbm_ctx* c);
// closure.hip: enqueue n steps of the stream-collide kernel with the fused closure
int launch_closure_steps(lbm_ctx* c, int64_t nsteps);

#define HIPCHK(ctx, call)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) return set_err(ctx, LBM_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

#define LAUNCHCHK(ctx)                                                                     \
  do {                                                                                     \
    hipError_t e_ = hipGetLastError();                                                     \
    if (e_ != hipSuccess) return set_err(ctx, LBM_EHIP, "kernel launch: %s", hipGetErrorString(e_)); \
  } while (0)

// dispatch over the storage forms
#define DISPATCH_ST(st, ...)                                   \
  switch (st) {                                                \
    case LBM_F64: { constexpr int ST = LBM_F64; __VA_ARGS__; } break;         \
    case LBM_F32: { constexpr int ST = LBM_F32; __VA_ARGS__; } break;         \
    case LBM_F16DEV: { constexpr int ST = LBM_F16DEV; __VA_ARGS__; } break;   \
    case LBM_BF16DEV: { constexpr int ST = LBM_BF16DEV; __VA_ARGS__; } break; \
    case LBM_F16DEV_RNE: { constexpr int ST = LBM_F16DEV_RNE; __VA_ARGS__; } break; \
    case LBM_BF16DEV_RNE: { constexpr int ST = LBM_BF16DEV_RNE; __VA_ARGS__; } break; \
  }

static inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }
