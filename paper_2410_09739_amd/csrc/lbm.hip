// lbm.hip -- gfx950 kernels and the C ABI of include/lbm.h.
//
// Data layout in HBM: two state buffers (A/B, ping-pong) in the blocked
// layout of lbm_internal.hpp (per row, segments of 64 x-consecutive nodes
// holding their 27 directions one after the other).  A step reads the
// previous post-collision state from one buffer with a pull gather
// (f_alpha(x) = f~_alpha(x - e_alpha), Appendix D Step 6; halfway bounce-back
// takes the node's own opposite population) and writes the new post-collision
// state to the other: 27 reads and 27 writes per node, each value read exactly
// once, no atomics, no LDS.  One wavefront updates one 64-node segment.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>

#include "lbm_internal.hpp"

#include "stream_collide.hpp"

// ===========================================================================
// initialisation: f~(0) = f^eq(rho, u); kappa' = rho' E, mapped back by the
// inverse sweeps (the same ones the collision uses).
template <int ST>
__global__ __launch_bounds__(256) void k_init(const double* __restrict__ rho, const double* __restrict__ u,
                                              typename Stor<ST>::S* __restrict__ dst, int64_t n, Geom g) {
  using T = typename Stor<ST>::R;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T rp = rho ? (T)(rho[i] - 1.0) : T(0);
  const T ux = u ? (T)u[i] : T(0), uy = u ? (T)u[n + i] : T(0), uz = u ? (T)u[2 * n + i] : T(0);
  T v[3][3][3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int a = 0; a < 3; ++a) v[c][b][a] = rp * T(C1[a] * C1[b] * C1[c]);
  inverse_all(v, ux, uy, uz);
  int x, y, z;
  node_xyz(g, i, x, y, z);
#pragma unroll
  for (int a = 0; a < Q; ++a)
    dst[pop_index(g, a, x, y, z)] = Stor<ST>::enc_nearest(v[EZ[a] + 1][EY[a] + 1][EX[a] + 1], a, inv_factor(a));
}

// host order f[a][i] <-> the blocked layout
template <int ST>
__global__ __launch_bounds__(256) void k_set_f(const double* __restrict__ f, typename Stor<ST>::S* __restrict__ dst,
                                               int64_t n, Geom g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int x, y, z;
  node_xyz(g, i, x, y, z);
#pragma unroll
  for (int a = 0; a < Q; ++a)
    dst[pop_index(g, a, x, y, z)] = Stor<ST>::enc_nearest((typename Stor<ST>::R)(f[a * n + i] - weight(a)), a);
}

template <int ST>
__global__ __launch_bounds__(256) void k_get_f(const typename Stor<ST>::S* __restrict__ src, double* __restrict__ f,
                                               int64_t n, Geom g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int x, y, z;
  node_xyz(g, i, x, y, z);
#pragma unroll
  for (int a = 0; a < Q; ++a) f[a * n + i] = weight(a) + (double)Stor<ST>::dec(src[pop_index(g, a, x, y, z)], a);
}

// the populations of listed nodes only (flat indices checked on the host)
template <int ST>
__global__ __launch_bounds__(256) void k_get_f_nodes(const typename Stor<ST>::S* __restrict__ src,
                                                     const int64_t* __restrict__ nodes, int64_t count,
                                                     double* __restrict__ f, Geom g) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  int x, y, z;
  node_xyz(g, nodes[k], x, y, z);
#pragma unroll
  for (int a = 0; a < Q; ++a) f[a * count + k] = weight(a) + (double)Stor<ST>::dec(src[pop_index(g, a, x, y, z)], a);
}

// Step 7 fields from the stored post-collision state: rho = 1 + sum delta,
// rho u = sum delta e - F/2.  FP64 output sums in FP64 whatever the storage
// (as the diagnostics do); FP32 output sums in the storage's arithmetic type.
template <int ST, typename OUT>
__global__ __launch_bounds__(256) void k_moments(const typename Stor<ST>::S* __restrict__ src, OUT* __restrict__ rho,
                                                 OUT* __restrict__ u, int64_t n, Geom g, double Fx, double Fy,
                                                 double Fz) {
  using T = typename Stor<ST>::R;
  using A = typename std::conditional<sizeof(OUT) == sizeof(double), double, T>::type;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int x, y, z;
  node_xyz(g, i, x, y, z);
  A v[3][3][3];
#pragma unroll
  for (int a = 0; a < Q; ++a) v[EZ[a] + 1][EY[a] + 1][EX[a] + 1] = (A)Stor<ST>::dec(src[pop_index(g, a, x, y, z)], a);
  A rp, jx, jy, jz;
  density_momentum(v, rp, jx, jy, jz);
  const double r = 1.0 + (double)rp;
  if (rho) rho[i] = (OUT)r;
  if (u) {
    u[i] = (OUT)(((double)jx - 0.5 * Fx) / r);
    u[n + i] = (OUT)(((double)jy - 0.5 * Fy) / r);
    u[2 * n + i] = (OUT)(((double)jz - 0.5 * Fz) / r);
  }
}

// ===========================================================================
// FP64 diagnostics with a deterministic reduction order:
// fixed grid of DIAG_BLOCKS blocks, grid-stride loops, wave64 shuffles, LDS
// across the 4 waves, then one block over the per-block partials.
constexpr int DIAG_BLOCKS = 1024;
constexpr int DIAG_THREADS = 256;
constexpr int NP = 12;  // partial slots per block

enum { P_MASS, P_MX, P_MY, P_MZ, P_KE, P_WX, P_WY, P_WZ, P_NONFIN, P_ENS, P_MAXU, P_MINRHO };

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

// sums partial values over the block; kind 0 = sum, 1 = max, 2 = min
template <int NV>
__device__ void block_reduce(double (&val)[NV], const int (&kind)[NV], double* out) {
  __shared__ double sh[DIAG_THREADS / 64][NV];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double t = kind[k] == 0 ? wave_sum(val[k]) : kind[k] == 1 ? wave_max(val[k]) : wave_min(val[k]);
    if (lane == 0) sh[wid][k] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double t = sh[0][k];
      for (int w = 1; w < DIAG_THREADS / 64; ++w)
        t = kind[k] == 0 ? t + sh[w][k] : kind[k] == 1 ? fmax(t, sh[w][k]) : fmin(t, sh[w][k]);
      out[k] = t;
    }
  }
}

template <int ST>
__global__ __launch_bounds__(DIAG_THREADS) void k_diag_nodes(const typename Stor<ST>::S* __restrict__ src,
                                                             double* __restrict__ uscr, double* __restrict__ part,
                                                             Geom g, int walls, double Fx, double Fy, double Fz) {
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  double acc[NP];
  const int kind[NP] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 2};
#pragma unroll
  for (int k = 0; k < NP; ++k) acc[k] = 0.0;
  acc[P_MINRHO] = INFINITY;
  for (int64_t i = (int64_t)blockIdx.x * DIAG_THREADS + threadIdx.x; i < n; i += (int64_t)DIAG_BLOCKS * DIAG_THREADS) {
    int x, y, z;
    node_xyz(g, i, x, y, z);
    double d[Q];
    bool finite = true;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      d[a] = (double)Stor<ST>::dec(src[pop_index(g, a, x, y, z)], a);
      finite = finite && isfinite(d[a]);
    }
    double rp = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      rp += d[a];
      jx += EX[a] * d[a];
      jy += EY[a] * d[a];
      jz += EZ[a] * d[a];
    }
    const double r = 1.0 + rp;
    jx -= 0.5 * Fx;
    jy -= 0.5 * Fy;
    jz -= 0.5 * Fz;
    const double ux = jx / r, uy = jy / r, uz = jz / r;
    uscr[i] = ux;
    uscr[n + i] = uy;
    uscr[2 * n + i] = uz;
    acc[P_MASS] += r;
    acc[P_MX] += jx;
    acc[P_MY] += jy;
    acc[P_MZ] += jz;
    const double s2 = ux * ux + uy * uy + uz * uz;
    acc[P_KE] += 0.5 * r * s2;
    acc[P_NONFIN] += finite ? 0.0 : 1.0;
    acc[P_MAXU] = fmax(acc[P_MAXU], sqrt(s2));
    acc[P_MINRHO] = fmin(acc[P_MINRHO], r);
    if (walls & 7) {
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        // links from this node into a wall (the symmetry plane takes no force)
        const bool ly = (walls & 1) && ((EY[a] == -1 && y == 0) || (EY[a] == 1 && y == g.ny - 1 && !(walls & 8)));
        const bool lx = (walls & 2) && ((EX[a] == -1 && x == 0) || (EX[a] == 1 && x == g.nx - 1));
        const bool lz = (walls & 4) && ((EZ[a] == -1 && z == 0) || (EZ[a] == 1 && z == g.nz - 1));
        if (ly || lx || lz) {
          const double fa = weight(a) + d[a];
          acc[P_WX] += 2.0 * fa * EX[a];
          acc[P_WY] += 2.0 * fa * EY[a];
          acc[P_WZ] += 2.0 * fa * EZ[a];
        }
      }
    }
  }
  block_reduce<NP>(acc, kind, part + (int64_t)blockIdx.x * NP);
}

// 1/2 |curl u|^2 with centred differences, d q(i) = (q(i+1) - q(i-1)) / 2.
// Periodic axes wrap; across a half-link wall at rest the ghost value is -u of
// the adjacent node (u = 0 halfway), across the moving lid above y = ny - 1 it
// is 2 U - u (u = U halfway), and across the symmetry plane there the
// tangential components (the only ones differentiated in y) mirror.
// walls: wall mask (1 = y, 2 = x, 4 = z, 8 = symmetry plane on top).
__global__ __launch_bounds__(DIAG_THREADS) void k_diag_enstrophy(const double* __restrict__ u, double* __restrict__ part,
                                                                 Geom g, int walls, double lidx, double lidy,
                                                                 double lidz) {
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  double acc[1] = {0.0};
  const int kind[1] = {0};
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const double lid[3] = {lidx, lidy, lidz};
  for (int64_t i = (int64_t)blockIdx.x * DIAG_THREADS + threadIdx.x; i < n; i += (int64_t)DIAG_BLOCKS * DIAG_THREADS) {
    const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((int64_t)nx * ny));
    auto at = [&](int c, int xx, int yy, int zz) { return u[(int64_t)c * n + ((int64_t)zz * ny + yy) * nx + xx]; };
    // value of component c one node along axis (0 x, 1 y, 2 z) in direction s (+-1)
    auto nb = [&](int c, int axis, int s) -> double {
      int xx = x, yy = y, zz = z;
      if (axis == 0) {
        xx = x + s;
        if (xx < 0 || xx >= nx) {
          if (walls & 2) return -at(c, x, y, z);
          xx = xx < 0 ? nx - 1 : 0;
        }
      } else if (axis == 1) {
        yy = y + s;
        if (yy < 0 || yy >= ny) {
          if (walls & 1) {
            if (yy < 0) return -at(c, x, y, z);
            if (walls & 8) return at(c, x, y, z);  // tangential components mirror
            return 2.0 * lid[c] - at(c, x, y, z);
          }
          yy = yy < 0 ? ny - 1 : 0;
        }
      } else {
        zz = z + s;
        if (zz < 0 || zz >= nz) {
          if (walls & 4) return -at(c, x, y, z);
          zz = zz < 0 ? nz - 1 : 0;
        }
      }
      return at(c, xx, yy, zz);
    };
    auto d = [&](int c, int axis) { return 0.5 * (nb(c, axis, 1) - nb(c, axis, -1)); };
    const double wx = d(2, 1) - d(1, 2), wy = d(0, 2) - d(2, 0), wz = d(1, 0) - d(0, 1);
    acc[0] += 0.5 * (wx * wx + wy * wy + wz * wz);
  }
  block_reduce<1>(acc, kind, part + (int64_t)blockIdx.x);
}

__global__ __launch_bounds__(DIAG_THREADS) void k_diag_final(const double* __restrict__ part,
                                                             const double* __restrict__ part_ens,
                                                             double* __restrict__ out) {
  double acc[NP];
  const int kind[NP] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 2};
#pragma unroll
  for (int k = 0; k < NP; ++k) acc[k] = 0.0;
  acc[P_MINRHO] = INFINITY;
  for (int b = threadIdx.x; b < DIAG_BLOCKS; b += DIAG_THREADS) {
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const double p = k == P_ENS ? part_ens[b] : part[b * NP + k];
      acc[k] = kind[k] == 0 ? acc[k] + p : kind[k] == 1 ? fmax(acc[k], p) : fmin(acc[k], p);
    }
  }
  block_reduce<NP>(acc, kind, out);
}

// ===========================================================================
// host side

// error text of calls without a context (create), one per host thread
static thread_local char g_create_err[512] = "";


int set_err(lbm_ctx* c, int code, const char* fmt, ...) {
  char* dst = c ? c->err : g_create_err;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(dst, 512, fmt, ap);
  va_end(ap);
  // a failed runtime call also leaves HIP's per-thread last error set; it is
  // reported here, so discard it: a later launch check must not report it again
  if (code == LBM_EHIP || code == LBM_ENOMEM) (void)hipGetLastError();
  return code;
}



extern "C" void lbm_config_default(lbm_config* cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->storage = LBM_F32;
  cfg->omega_mode = LBM_OMEGA_PAPER;
  cfg->nu = 1.0 / 6.0;
  cfg->omega_bulk = 1.0;
  cfg->omega_higher = 1.0;
  cfg->les_aplus = 26.0;
}

// Eq. (transportcoeff3DFPCLBM): nu = c_s^2 (1/omega - 1/2), c_s^2 = 1/3.
extern "C" int lbm_omega_table(const lbm_config* cfg, double out[LBM_Q]) {
  if (!cfg || !out) return LBM_EINVAL;
  double w[LBM_Q];
  if (cfg->omega_mode == LBM_OMEGA_EXPLICIT) {
    for (int j = 0; j < LBM_Q; ++j) w[j] = cfg->omega[j];
  } else if (cfg->omega_mode == LBM_OMEGA_PAPER || cfg->omega_mode == LBM_OMEGA_ORDER_SCALED) {
    if (!(cfg->nu > 0.0) || !std::isfinite(cfg->nu)) return LBM_EINVAL;
    const double w2 = 1.0 / (3.0 * cfg->nu + 0.5);
    for (int j = 0; j < LBM_Q; ++j) w[j] = cfg->omega_higher;
    w[0] = w[1] = w[2] = w[3] = 1.0;
    w[4] = w[5] = w[6] = w[8] = w[9] = w2;
    w[7] = cfg->omega_bulk;
    if (cfg->omega_mode == LBM_OMEGA_ORDER_SCALED) {
      // order of the moments relaxed with omega_10..omega_26
      static const int order[LBM_Q] = {0, 1, 1, 1, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3,
                                       4, 4, 4, 4, 4, 4, 5, 5, 5, 6};
      for (int j = 10; j < LBM_Q; ++j) w[j] = 1.0 / ((2.0 / order[j]) * (1.0 / w2 - 0.5) + 0.5);
    }
  } else {
    return LBM_EINVAL;
  }
  for (int j = 0; j < LBM_Q; ++j)
    if (!(w[j] > 0.0 && w[j] < 2.0)) return LBM_EINVAL;
  for (int j = 0; j < LBM_Q; ++j) out[j] = w[j];
  return LBM_OK;
}

static int noalloc_setup(lbm_ctx* c, int dev);

extern "C" int lbm_create(const lbm_config* cfg, lbm_ctx** out) {
  if (!out) return set_err(nullptr, LBM_EINVAL, "lbm_create: out is NULL");
  *out = nullptr;
  if (!cfg) return set_err(nullptr, LBM_EINVAL, "lbm_create: cfg is NULL");
  if (cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1)
    return set_err(nullptr, LBM_EINVAL, "lbm_create: grid %d x %d x %d must be positive", cfg->nx, cfg->ny, cfg->nz);
  const int64_t n = (int64_t)cfg->nx * cfg->ny * cfg->nz;
  if (n >= (int64_t)1 << 31) return set_err(nullptr, LBM_EINVAL, "lbm_create: %lld nodes exceed 2^31 - 1", (long long)n);
  const size_t es = elem_size(cfg->storage);
  if (!es) return set_err(nullptr, LBM_EINVAL, "lbm_create: unknown storage %d", cfg->storage);
  const Geom geo = make_geom(cfg);
  if ((uint64_t)geo.rowlen * es >= ((uint64_t)1 << 32))
    return set_err(nullptr, LBM_EINVAL, "lbm_create: one row of the state must stay below 4 GiB");
  if (cfg->walls_y != 0 && cfg->walls_y != 1) return set_err(nullptr, LBM_EINVAL, "lbm_create: walls_y must be 0 or 1");
  if ((cfg->walls_x != 0 && cfg->walls_x != 1) || (cfg->walls_z != 0 && cfg->walls_z != 1))
    return set_err(nullptr, LBM_EINVAL, "lbm_create: walls_x and walls_z must be 0 or 1");
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(cfg->lid_velocity[d])) return set_err(nullptr, LBM_EINVAL, "lbm_create: non-finite lid velocity");
  if ((cfg->lid_velocity[0] != 0.0 || cfg->lid_velocity[1] != 0.0 || cfg->lid_velocity[2] != 0.0) && !cfg->walls_y)
    return set_err(nullptr, LBM_EINVAL, "lbm_create: a moving lid needs walls_y = 1");
  if (cfg->sym_top != 0 && cfg->sym_top != 1) return set_err(nullptr, LBM_EINVAL, "lbm_create: sym_top must be 0 or 1");
  if (cfg->sym_top && (!cfg->walls_y || cfg->lid_velocity[0] != 0.0 || cfg->lid_velocity[1] != 0.0 || cfg->lid_velocity[2] != 0.0))
    return set_err(nullptr, LBM_EINVAL, "lbm_create: a symmetry plane needs walls_y = 1 (the wall below) and no lid");
  if (!(cfg->les_cs >= 0.0) || !std::isfinite(cfg->les_cs) || !(cfg->les_wall_units >= 0.0) ||
      !std::isfinite(cfg->les_wall_units) || (cfg->les_cs > 0.0 && !(cfg->les_aplus > 0.0)))
    return set_err(nullptr, LBM_EINVAL, "lbm_create: LES needs les_cs >= 0, les_wall_units >= 0, les_aplus > 0");
  if (cfg->attractor != LBM_ATTRACTOR_FPC && cfg->attractor != LBM_ATTRACTOR_MAXWELL)
    return set_err(nullptr, LBM_EINVAL, "lbm_create: unknown attractor %d", cfg->attractor);
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(cfg->force[d])) return set_err(nullptr, LBM_EINVAL, "lbm_create: non-finite force");
  double w[LBM_Q];
  if (lbm_omega_table(cfg, w) != LBM_OK)
    return set_err(nullptr, LBM_EINVAL, "lbm_create: relaxation rates must lie in (0,2) (check nu, omega_bulk, omega_higher, omega[])");

  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return set_err(nullptr, LBM_ENOMEM, "lbm_create: host allocation failed");
  c->cfg = *cfg;
  std::memcpy(c->omega, w, sizeof w);
  c->n = n;
  c->g = geo;
  c->values = geo.rowlen * cfg->ny * cfg->nz;
  c->elem = es;
  hipError_t e = hipGetDevice(&c->device);
  if (e == hipSuccess) {
    if (cfg->hip_stream) {
      c->stream = (hipStream_t)cfg->hip_stream;
    } else {
      e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
      c->own_stream = (e == hipSuccess);
    }
  }
  for (int b = 0; b < 2 && e == hipSuccess; ++b) e = hipMalloc(&c->buf[b], (size_t)c->values * es);
  // The padding lanes of the x segments (nx not a multiple of 64) are never
  // written by the kernels: zero them once so that the raw state is defined.
  // The clear goes on the library's stream and completes before create
  // returns: a plain hipMemset would run on the null stream, unordered with
  // the (non-blocking) library stream, and could land after a following init.
  for (int b = 0; b < 2 && e == hipSuccess; ++b) e = hipMemsetAsync(c->buf[b], 0, (size_t)c->values * es, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = hipMalloc((void**)&c->part, sizeof(double) * (DIAG_BLOCKS * (NP + 1) + NP));
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->host_out, sizeof(double) * NP, hipHostMallocDefault);
  if (e != hipSuccess) {
    int code = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? LBM_ENOMEM : LBM_EHIP;
    set_err(nullptr, code, "lbm_create: %s", hipGetErrorString(e));
    lbm_destroy(c);
    return code;
  }
  // once per device: the address of the staging array of the no-allocation calls
  const int rc = noalloc_setup(nullptr, c->device);
  if (rc != LBM_OK) {
    lbm_destroy(c);
    return rc;
  }
  *out = c;
  return LBM_OK;
}

extern "C" void lbm_destroy(lbm_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (int b = 0; b < 2; ++b)
    if (c->buf[b]) (void)hipFree(c->buf[b]);
  if (c->scratch) (void)hipFree(c->scratch);
  if (c->part) (void)hipFree(c->part);
  if (c->host_out) (void)hipHostFree(c->host_out);
  if (c->closure) (void)hipFree(c->closure);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

extern "C" const char* lbm_last_error(const lbm_ctx* c) { return c ? c->err : g_create_err; }
extern "C" void* lbm_stream(const lbm_ctx* c) { return c ? (void*)c->stream : nullptr; }
extern "C" int64_t lbm_step_count(const lbm_ctx* c) { return c ? c->steps : -1; }
extern "C" int lbm_set_step_count(lbm_ctx* c, int64_t steps) {
  if (!c || steps < 0) return LBM_EINVAL;
  c->steps = steps;
  return LBM_OK;
}
extern "C" int64_t lbm_state_bytes(const lbm_ctx* c) { return c ? c->values * (int64_t)c->elem : -1; }



int alloc_scratch(lbm_ctx* c) {
  if (!c->scratch) HIPCHK(c, hipMalloc((void**)&c->scratch, sizeof(double) * 4 * c->n));
  return LBM_OK;
}

extern "C" int lbm_init(lbm_ctx* c, const double* rho, const double* u) {
  if (!c) return LBM_EINVAL;
  HIPCHK(c, hipSetDevice(c->device));
  int rc = alloc_scratch(c);
  if (rc) return rc;
  const int64_t n = c->n;
  double* drho = nullptr;
  double* du = nullptr;
  if (rho) {
    drho = c->scratch;
    HIPCHK(c, hipMemcpyAsync(drho, rho, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
  }
  if (u) {
    du = c->scratch + n;
    HIPCHK(c, hipMemcpyAsync(du, u, sizeof(double) * 3 * n, hipMemcpyHostToDevice, c->stream));
  }
  c->cur = 0;
  DISPATCH_ST(c->cfg.storage,
              k_init<ST><<<nblocks(n, 256), 256, 0, c->stream>>>(drho, du, (typename Stor<ST>::S*)c->buf[0], n, geom(c)));
  LAUNCHCHK(c);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->initialised = true;
  c->steps = 0;
  return LBM_OK;
}

// The rates of the paper's runs: every rate of orders 3-6 exactly 1
// (unit_rates_3_to_6), and the bulk rate omega_7 as well (unit_higher_rates).
// With no force and the bulk rate 1 the step kernel takes the collision that
// needs only the second-order moments (relax_unit_higher); with a force (or
// another bulk rate) the one that drops the pre-collision values of orders 3-6
// from their own relaxation (relax<..., UH = true>).
bool unit_rates_3_to_6(const lbm_ctx* c) {
  for (int j = 10; j < LBM_Q; ++j)
    if (c->omega[j] != 1.0) return false;
  return true;
}
static bool unit_higher_rates(const lbm_ctx* c) { return c->omega[7] == 1.0 && unit_rates_3_to_6(c); }

template <int ST>
static int launch_steps(lbm_ctx* c, int64_t nsteps) {
  using T = typename Stor<ST>::R;
  using S = typename Stor<ST>::S;
  StepArgs<T> A;
  A.g = geom(c);
  for (int j = 0; j < LBM_Q; ++j) {
    A.r.w[j] = (T)c->omega[j];
    A.r.c[j] = (T)(1.0 - c->omega[j]);
    A.r.h[j] = (T)(1.0 - 0.5 * c->omega[j]);
  }
  for (int d = 0; d < 3; ++d) A.F[d] = (T)c->cfg.force[d];
  A.box = box_args<T>(c);
  const bool force = c->cfg.force[0] != 0.0 || c->cfg.force[1] != 0.0 || c->cfg.force[2] != 0.0;
  dim3 block, grid;
  step_launch_shape(c->cfg.nx, c->cfg.ny, c->cfg.nz, block, grid);
  using KFn = void (*)(const S*, S*, StepArgs<T>);
  static const KFn table[2][3][2] = {
      {{k_stream_collide<ST, 0, false, false>, k_stream_collide<ST, 0, true, false>},
       {k_stream_collide<ST, 1, false, false>, k_stream_collide<ST, 1, true, false>},
       {k_stream_collide<ST, 2, false, false>, k_stream_collide<ST, 2, true, false>}},
      {{k_stream_collide<ST, 0, false, true>, k_stream_collide<ST, 0, true, true>},
       {k_stream_collide<ST, 1, false, true>, k_stream_collide<ST, 1, true, true>},
       {k_stream_collide<ST, 2, false, true>, k_stream_collide<ST, 2, true, true>}}};
  static const KFn second_only[3] = {k_stream_collide<ST, 0, false, false, COLL_SECOND_ONLY>,
                                     k_stream_collide<ST, 1, false, false, COLL_SECOND_ONLY>,
                                     k_stream_collide<ST, 2, false, false, COLL_SECOND_ONLY>};
  static const KFn unit_forced[3] = {k_stream_collide<ST, 0, true, false, COLL_UNIT_HIGHER>,
                                     k_stream_collide<ST, 1, true, false, COLL_UNIT_HIGHER>,
                                     k_stream_collide<ST, 2, true, false, COLL_UNIT_HIGHER>};
  const bool maxwell = c->cfg.attractor == LBM_ATTRACTOR_MAXWELL;
  KFn kern = table[maxwell][bc_kind(c)][force];
  if (!maxwell && !force && unit_higher_rates(c)) kern = second_only[bc_kind(c)];
  if (!maxwell && force && unit_rates_3_to_6(c)) kern = unit_forced[bc_kind(c)];
  for (int64_t s = 0; s < nsteps; ++s) {
    const S* src = (const S*)c->buf[c->cur];
    S* dst = (S*)c->buf[c->cur ^ 1];
    A.step = (uint32_t)c->steps;
    kern<<<grid, block, 0, c->stream>>>(src, dst, A);
    LAUNCHCHK(c);
    c->cur ^= 1;
    c->steps++;
  }
  return LBM_OK;
}

extern "C" int lbm_step(lbm_ctx* c, int64_t n) {
  if (!c || n < 0) return LBM_EINVAL;
  if (!c->initialised) return set_err(c, LBM_ESTATE, "lbm_step: state not initialised (call lbm_init or lbm_set_f)");
  HIPCHK(c, hipSetDevice(c->device));
  if (c->closure) return launch_closure_steps(c, n);
  int rc = LBM_OK;
  DISPATCH_ST(c->cfg.storage, rc = launch_steps<ST>(c, n));
  return rc;
}

extern "C" int lbm_synchronize(lbm_ctx* c) {
  if (!c) return LBM_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

extern "C" int lbm_moments_device(lbm_ctx* c, void* rho_dev, void* u_dev, int32_t f64) {
  if (!c) return LBM_EINVAL;
  if (!c->initialised) return set_err(c, LBM_ESTATE, "lbm_moments: state not initialised");
  HIPCHK(c, hipSetDevice(c->device));
  const double* F = c->cfg.force;
  const int64_t n = c->n;
  if (f64) {
    DISPATCH_ST(c->cfg.storage,
                k_moments<ST, double><<<nblocks(n, 256), 256, 0, c->stream>>>(
                    (const typename Stor<ST>::S*)c->buf[c->cur], (double*)rho_dev, (double*)u_dev, n, geom(c), F[0], F[1], F[2]));
  } else {
    DISPATCH_ST(c->cfg.storage,
                k_moments<ST, float><<<nblocks(n, 256), 256, 0, c->stream>>>(
                    (const typename Stor<ST>::S*)c->buf[c->cur], (float*)rho_dev, (float*)u_dev, n, geom(c), F[0], F[1], F[2]));
  }
  LAUNCHCHK(c);
  return LBM_OK;
}

extern "C" int lbm_moments(lbm_ctx* c, double* rho, double* u) {
  if (!c) return LBM_EINVAL;
  if (!c->initialised) return set_err(c, LBM_ESTATE, "lbm_moments: state not initialised");
  HIPCHK(c, hipSetDevice(c->device));
  int rc = alloc_scratch(c);
  if (rc) return rc;
  rc = lbm_moments_device(c, c->scratch, c->scratch + c->n, 1);
  if (rc) return rc;
  if (rho) HIPCHK(c, hipMemcpyAsync(rho, c->scratch, sizeof(double) * c->n, hipMemcpyDeviceToHost, c->stream));
  if (u) HIPCHK(c, hipMemcpyAsync(u, c->scratch + c->n, sizeof(double) * 3 * c->n, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

extern "C" int lbm_get_f(lbm_ctx* c, double* f) {
  if (!c || !f) return LBM_EINVAL;
  if (!c->initialised) return set_err(c, LBM_ESTATE, "lbm_get_f: state not initialised");
  HIPCHK(c, hipSetDevice(c->device));
  double* tmp = nullptr;
  HIPCHK(c, hipMalloc((void**)&tmp, sizeof(double) * LBM_Q * c->n));
  DISPATCH_ST(c->cfg.storage,
              k_get_f<ST><<<nblocks(c->n, 256), 256, 0, c->stream>>>((const typename Stor<ST>::S*)c->buf[c->cur], tmp, c->n, geom(c)));
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(f, tmp, sizeof(double) * LBM_Q * c->n, hipMemcpyDeviceToHost, c->stream);
  hipError_t e3 = hipStreamSynchronize(c->stream);
  hipError_t e2 = hipFree(tmp);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = e3;
  if (e != hipSuccess) return set_err(c, LBM_EHIP, "lbm_get_f: %s", hipGetErrorString(e));
  return LBM_OK;
}

extern "C" int lbm_get_f_nodes(lbm_ctx* c, const int64_t* nodes, int64_t count, double* f) {
  if (!c || count < 0 || (count > 0 && (!nodes || !f))) return set_err(c, LBM_EINVAL, "lbm_get_f_nodes: bad arguments");
  if (!c->initialised) return set_err(c, LBM_ESTATE, "lbm_get_f_nodes: state not initialised");
  for (int64_t k = 0; k < count; ++k)
    if (nodes[k] < 0 || nodes[k] >= c->n)
      return set_err(c, LBM_EINVAL, "lbm_get_f_nodes: node %lld outside [0, %lld)", (long long)nodes[k], (long long)c->n);
  if (count == 0) return LBM_OK;
  HIPCHK(c, hipSetDevice(c->device));
  char* tmp = nullptr;
  const size_t nb = sizeof(int64_t) * count, fb = sizeof(double) * LBM_Q * count;
  HIPCHK(c, hipMalloc((void**)&tmp, nb + fb));
  int64_t* dn = (int64_t*)tmp;
  double* df = (double*)(tmp + nb);
  hipError_t e = hipMemcpyAsync(dn, nodes, nb, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) {
    DISPATCH_ST(c->cfg.storage,
                k_get_f_nodes<ST><<<nblocks(count, 256), 256, 0, c->stream>>>((const typename Stor<ST>::S*)c->buf[c->cur], dn,
                                                                              count, df, geom(c)));
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(f, df, fb, hipMemcpyDeviceToHost, c->stream);
  hipError_t e3 = hipStreamSynchronize(c->stream);
  hipError_t e2 = hipFree(tmp);
  if (e == hipSuccess) e = e3;
  if (e == hipSuccess) e = e2;
  if (e != hipSuccess) return set_err(c, LBM_EHIP, "lbm_get_f_nodes: %s", hipGetErrorString(e));
  return LBM_OK;
}

// ---------------------------------------------------------------------------
// lbm_get_f_nodes without allocation: the node list and the populations are
// staged in a file-scope device array instead of a per-call hipMalloc.  Each
// GPU the library runs on holds its own copy of the array until the process
// ends; host code never uses the array's name as an address (on the host it
// is only a stand-in): lbm_create looks up the device address once per device
// with hipGetSymbolAddress and keeps it in g_noalloc_ptr.
constexpr int64_t NOALLOC_BYTES = LBM_NOALLOC_MAX_NODES * (int64_t)sizeof(int64_t) +
                                  LBM_NOALLOC_MAX_NODES * (int64_t)LBM_Q * (int64_t)sizeof(double);
static __device__ __align__(256) char scratch[NOALLOC_BYTES];
constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_noalloc_mutex;
static void* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// with device `dev` current: the device address of its scratch array
static int noalloc_setup(lbm_ctx* c, int dev) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return set_err(c, LBM_EINVAL, "device %d beyond the library's table", dev);
  std::lock_guard<std::mutex> lock(g_noalloc_mutex);
  if (g_noalloc_ptr[dev]) return LBM_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return set_err(c, LBM_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
  g_noalloc_ptr[dev] = ptr;
  return LBM_OK;
}

extern "C" int lbm_get_f_nodes_noalloc(lbm_ctx* c, const int64_t* nodes, int64_t count, double* f) {
  if (!c || count < 0 || (count > 0 && (!nodes || !f)))
    return set_err(c, LBM_EINVAL, "lbm_get_f_nodes_noalloc: bad arguments");
  if (count > LBM_NOALLOC_MAX_NODES)
    return set_err(c, LBM_EINVAL, "lbm_get_f_nodes_noalloc: %lld nodes exceed the maximum of %d per call",
                   (long long)count, LBM_NOALLOC_MAX_NODES);
  if (!c->initialised) return set_err(c, LBM_ESTATE, "lbm_get_f_nodes_noalloc: state not initialised");
  for (int64_t k = 0; k < count; ++k)
    if (nodes[k] < 0 || nodes[k] >= c->n)
      return set_err(c, LBM_EINVAL, "lbm_get_f_nodes_noalloc: node %lld outside [0, %lld)", (long long)nodes[k],
                     (long long)c->n);
  if (count == 0) return LBM_OK;
  HIPCHK(c, hipSetDevice(c->device));
  char* base = (char*)g_noalloc_ptr[c->device];  // set by lbm_create on this device
  if (!base) return set_err(c, LBM_ESTATE, "lbm_get_f_nodes_noalloc: scratch not set up on device %d", c->device);
  int64_t* dn = (int64_t*)base;
  double* df = (double*)(base + LBM_NOALLOC_MAX_NODES * (int64_t)sizeof(int64_t));
  const size_t nb = sizeof(int64_t) * count, fb = sizeof(double) * LBM_Q * count;
  HIPCHK(c, hipMemcpyAsync(dn, nodes, nb, hipMemcpyHostToDevice, c->stream));
  DISPATCH_ST(c->cfg.storage,
              k_get_f_nodes<ST><<<nblocks(count, 256), 256, 0, c->stream>>>((const typename Stor<ST>::S*)c->buf[c->cur], dn,
                                                                            count, df, geom(c)));
  LAUNCHCHK(c);
  HIPCHK(c, hipMemcpyAsync(f, df, fb, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

extern "C" int lbm_set_f(lbm_ctx* c, const double* f) {
  if (!c || !f) return LBM_EINVAL;
  HIPCHK(c, hipSetDevice(c->device));
  double* tmp = nullptr;
  HIPCHK(c, hipMalloc((void**)&tmp, sizeof(double) * LBM_Q * c->n));
  hipError_t e = hipMemcpyAsync(tmp, f, sizeof(double) * LBM_Q * c->n, hipMemcpyHostToDevice, c->stream);
  c->cur = 0;
  if (e == hipSuccess) {
    DISPATCH_ST(c->cfg.storage,
                k_set_f<ST><<<nblocks(c->n, 256), 256, 0, c->stream>>>(tmp, (typename Stor<ST>::S*)c->buf[0], c->n, geom(c)));
    e = hipGetLastError();
  }
  hipError_t e3 = hipStreamSynchronize(c->stream);
  hipError_t e2 = hipFree(tmp);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = e3;
  if (e != hipSuccess) return set_err(c, LBM_EHIP, "lbm_set_f: %s", hipGetErrorString(e));
  c->initialised = true;
  c->steps = 0;
  return LBM_OK;
}

extern "C" int lbm_get_raw(lbm_ctx* c, void* host, int64_t nbytes) {
  if (!c || !host || nbytes != lbm_state_bytes(c)) return LBM_EINVAL;
  if (!c->initialised) return set_err(c, LBM_ESTATE, "lbm_get_raw: state not initialised");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipMemcpyAsync(host, c->buf[c->cur], (size_t)nbytes, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

extern "C" int lbm_set_raw(lbm_ctx* c, const void* host, int64_t nbytes) {
  if (!c || !host || nbytes != lbm_state_bytes(c)) return LBM_EINVAL;
  HIPCHK(c, hipSetDevice(c->device));
  c->cur = 0;
  HIPCHK(c, hipMemcpyAsync(c->buf[0], host, (size_t)nbytes, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->initialised = true;
  c->steps = 0;
  return LBM_OK;
}

extern "C" int lbm_diagnostics(lbm_ctx* c, lbm_diag* out) {
  if (!c || !out) return LBM_EINVAL;
  if (!c->initialised) return set_err(c, LBM_ESTATE, "lbm_diagnostics: state not initialised");
  HIPCHK(c, hipSetDevice(c->device));
  int rc = alloc_scratch(c);
  if (rc) return rc;
  const Geom g = geom(c);
  const double* F = c->cfg.force;
  double* part = c->part;
  double* part_ens = c->part + DIAG_BLOCKS * NP;
  double* dout = part_ens + DIAG_BLOCKS;
  DISPATCH_ST(c->cfg.storage,
              k_diag_nodes<ST><<<DIAG_BLOCKS, DIAG_THREADS, 0, c->stream>>>(
                  (const typename Stor<ST>::S*)c->buf[c->cur], c->scratch, part, g, wall_mask(c), F[0], F[1], F[2]));
  LAUNCHCHK(c);
  const double* lid = c->cfg.lid_velocity;
  k_diag_enstrophy<<<DIAG_BLOCKS, DIAG_THREADS, 0, c->stream>>>(c->scratch, part_ens, g, wall_mask(c), lid[0], lid[1],
                                                                lid[2]);
  LAUNCHCHK(c);
  k_diag_final<<<1, DIAG_THREADS, 0, c->stream>>>(part, part_ens, dout);
  LAUNCHCHK(c);
  HIPCHK(c, hipMemcpyAsync(c->host_out, dout, sizeof(double) * NP, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double* h = c->host_out;
  out->mass = h[P_MASS];
  out->momentum[0] = h[P_MX];
  out->momentum[1] = h[P_MY];
  out->momentum[2] = h[P_MZ];
  out->kinetic_energy = h[P_KE];
  out->enstrophy = h[P_ENS];
  out->wall_force[0] = h[P_WX];
  out->wall_force[1] = h[P_WY];
  out->wall_force[2] = h[P_WZ];
  out->max_speed = h[P_MAXU];
  out->min_rho = h[P_MINRHO];
  out->n_nonfinite = (int64_t)h[P_NONFIN];
  out->step = c->steps;
  if (out->n_nonfinite > 0 || !(out->min_rho > 0.0) || !std::isfinite(out->mass))
    return set_err(c, LBM_EUNSTABLE, "lbm_diagnostics: %lld non-finite nodes, min rho %g", (long long)out->n_nonfinite, out->min_rho);
  return LBM_OK;
}
