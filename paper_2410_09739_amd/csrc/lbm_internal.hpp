// lbm_internal.hpp -- host-side pieces shared by the translation units of
// liblbm.so (the context, error handling, dispatch helpers).  Not part of the
// public interface (include/lbm.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lattice.hpp"

// ===========================================================================
// context
struct lbm_ctx {
  lbm_config cfg;
  int device = 0;
  int64_t n = 0;
  Geom g{};     // storage layout of the state buffers
  int64_t values = 0;  // values per state buffer
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
  int closure_grid = 0;                          // blocks of the persistent closure step (0: not sized yet)
};

int set_err(lbm_ctx* c, int code, const char* fmt, ...);
inline Geom geom(const lbm_ctx* c) { return c->g; }
inline bool has_lid(const lbm_ctx* c) {
  return c->cfg.lid_velocity[0] != 0.0 || c->cfg.lid_velocity[1] != 0.0 || c->cfg.lid_velocity[2] != 0.0;
}
// boundary kernel: 0 periodic, 1 walls across y only, 2 walls on any faces / moving lid
inline int bc_kind(const lbm_ctx* c) {
  if (c->cfg.walls_x || c->cfg.walls_z || has_lid(c) || c->cfg.sym_top || c->cfg.les_cs > 0.0) return 2;
  return c->cfg.walls_y ? 1 : 0;
}
template <typename T>
inline Box<T> box_args(const lbm_ctx* c) {
  Box<T> b;
  b.wx = c->cfg.walls_x;
  b.wy = c->cfg.walls_y;
  b.wz = c->cfg.walls_z;
  b.lid_on = has_lid(c) ? 1 : 0;
  for (int d = 0; d < 3; ++d) b.lid6[d] = (T)(6.0 * c->cfg.lid_velocity[d]);
  b.sym = c->cfg.sym_top;
  b.les_on = c->cfg.les_cs > 0.0 ? 1 : 0;
  b.les_c = (T)c->cfg.les_cs;
  b.les_s = (T)c->cfg.les_wall_units;
  b.les_ia = (T)(1.0 / c->cfg.les_aplus);
  return b;
}
// wall mask of the diagnostics: 1 = y, 2 = x, 4 = z, 8 = symmetry plane on top
inline int wall_mask(const lbm_ctx* c) {
  return (c->cfg.walls_y ? 1 : 0) | (c->cfg.walls_x ? 2 : 0) | (c->cfg.walls_z ? 4 : 0) | (c->cfg.sym_top ? 8 : 0);
}
int alloc_scratch(lbm_ctx* c);
// closure.hip: enqueue n steps of the stream-collide kernel with the fused closure
int launch_closure_steps(lbm_ctx* c, int64_t nsteps);
// lbm.hip: every rate of orders 3-6 is exactly 1 (the paper's runs)
bool unit_rates_3_to_6(const lbm_ctx* c);

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
