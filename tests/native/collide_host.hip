// Host build of the kernels' per-node arithmetic (paper_2410_09739_amd/csrc/fpc_collide.hpp)
// for CPU-side tests against the oracle.  It runs the same __host__ __device__
// sweeps and collision the GPU runs, on one node given as 27 populations.
#include <cstdint>
#include <vector>

#include "../../paper_2410_09739_amd/csrc/fpc_collide.hpp"

using namespace fpc;

template <typename T, bool MAXWELL>
static void run(const double* f, const double* omega, const double* F, double* out) {
  T v[3][3][3];
  for (int a = 0; a < Q; ++a) v[EZ[a] + 1][EY[a] + 1][EX[a] + 1] = (T)(f[a] - weight(a));
  Rates<T> R;
  for (int j = 0; j < Q; ++j) {
    R.w[j] = (T)omega[j];
    R.c[j] = (T)(1.0 - omega[j]);
    R.h[j] = (T)(1.0 - 0.5 * omega[j]);
  }
  const T ws[6] = {R.w[4], R.w[5], R.w[6], R.w[7], R.w[8], R.w[9]};
  const T cs[6] = {R.c[4], R.c[5], R.c[6], R.c[7], R.c[8], R.c[9]};
  T rho, ux, uy, uz;
  const bool force = F[0] != 0.0 || F[1] != 0.0 || F[2] != 0.0;
  if (force)
    collide<T, true, MAXWELL>(v, R, ws, cs, (T)F[0], (T)F[1], (T)F[2], rho, ux, uy, uz);
  else
    collide<T, false, MAXWELL>(v, R, ws, cs, T(0), T(0), T(0), rho, ux, uy, uz);
  for (int a = 0; a < Q; ++a) out[a] = weight(a) + (double)(v[EZ[a] + 1][EY[a] + 1][EX[a] + 1] * (T)inv_factor(a));
}

extern "C" void host_collide_f64(const double* f, const double* omega, const double* F, double* out) {
  run<double, false>(f, omega, F, out);
}
extern "C" void host_collide_f32(const double* f, const double* omega, const double* F, double* out) {
  run<float, false>(f, omega, F, out);
}
// the Maxwellian-attractor comparison model
extern "C" void host_collide_maxwell_f64(const double* f, const double* omega, const double* F, double* out) {
  run<double, true>(f, omega, F, out);
}
extern "C" void host_collide_maxwell_f32(const double* f, const double* omega, const double* F, double* out) {
  run<float, true>(f, omega, F, out);
}
// The same collision in storage units (the FP16/BF16 kernels' arithmetic):
// the cube comes in as deviations times dev_scale(alpha) and goes out times
// UNIT; out holds the deviations times 2^inv_shift (scales removed), so that a
// test can compare them bitwise with host_collide_dev_f32.
template <bool SU, bool MAXWELL>
static void run_dev(const float* dev, const double* omega, const double* F, float* out) {
  float v[3][3][3];
  for (int a = 0; a < Q; ++a) v[EZ[a] + 1][EY[a] + 1][EX[a] + 1] = SU ? dev[a] * dev_scale(a) : dev[a];
  Rates<float> R;
  for (int j = 0; j < Q; ++j) {
    R.w[j] = (float)omega[j];
    R.c[j] = (float)(1.0 - omega[j]);
    R.h[j] = (float)(1.0 - 0.5 * omega[j]);
  }
  const float ws[6] = {R.w[4], R.w[5], R.w[6], R.w[7], R.w[8], R.w[9]};
  const float cs[6] = {R.c[4], R.c[5], R.c[6], R.c[7], R.c[8], R.c[9]};
  float rho, ux, uy, uz;
  collide<float, true, MAXWELL, SU>(v, R, ws, cs, (float)F[0], (float)F[1], (float)F[2], rho, ux, uy, uz);
  for (int a = 0; a < Q; ++a) out[a] = v[EZ[a] + 1][EY[a] + 1][EX[a] + 1] * (float)(1.0 / Units<SU>::U);
}
extern "C" void host_collide_dev_f32(const float* dev, const double* omega, const double* F, int maxwell, float* out) {
  if (maxwell) run_dev<false, true>(dev, omega, F, out);
  else run_dev<false, false>(dev, omega, F, out);
}
extern "C" void host_collide_units_f32(const float* dev, const double* omega, const double* F, int maxwell,
                                       float* out) {
  if (maxwell) run_dev<true, true>(dev, omega, F, out);
  else run_dev<true, false>(dev, omega, F, out);
}

// The collision the step kernels take for the paper's rates (bulk and orders
// 3-6 at 1) without a force: second-order moments only (relax_unit_higher).
template <typename T>
static void run_unit(const double* f, const double* omega, double* out) {
  T v[3][3][3];
  for (int a = 0; a < Q; ++a) v[EZ[a] + 1][EY[a] + 1][EX[a] + 1] = (T)(f[a] - weight(a));
  const T cs[6] = {(T)(1.0 - omega[4]), (T)(1.0 - omega[5]), (T)(1.0 - omega[6]),
                   (T)(1.0 - omega[7]), (T)(1.0 - omega[8]), (T)(1.0 - omega[9])};
  T rho, ux, uy, uz;
  collide_unit_higher<T>(v, cs, rho, ux, uy, uz);
  for (int a = 0; a < Q; ++a) out[a] = weight(a) + (double)(v[EZ[a] + 1][EY[a] + 1][EX[a] + 1] * (T)inv_factor(a));
}
extern "C" void host_collide_unit_f64(const double* f, const double* omega, double* out) {
  run_unit<double>(f, omega, out);
}
extern "C" void host_collide_unit_f32(const double* f, const double* omega, double* out) {
  run_unit<float>(f, omega, out);
}
// the same in storage units and on plain deviations (FP32), for a bitwise comparison
template <bool SU>
static void run_unit_dev(const float* dev, const double* omega, float* out) {
  float v[3][3][3];
  for (int a = 0; a < Q; ++a) v[EZ[a] + 1][EY[a] + 1][EX[a] + 1] = SU ? dev[a] * dev_scale(a) : dev[a];
  const float cs[6] = {(float)(1.0 - omega[4]), (float)(1.0 - omega[5]), (float)(1.0 - omega[6]),
                       (float)(1.0 - omega[7]), (float)(1.0 - omega[8]), (float)(1.0 - omega[9])};
  float rho, ux, uy, uz;
  collide_unit_higher<float, SU>(v, cs, rho, ux, uy, uz);
  for (int a = 0; a < Q; ++a) out[a] = v[EZ[a] + 1][EY[a] + 1][EX[a] + 1] * (float)(1.0 / Units<SU>::U);
}
extern "C" void host_collide_unit_dev_f32(const float* dev, const double* omega, float* out) {
  run_unit_dev<false>(dev, omega, out);
}
extern "C" void host_collide_unit_units_f32(const float* dev, const double* omega, float* out) {
  run_unit_dev<true>(dev, omega, out);
}

// The collision the step kernels take when every rate of orders 3-6 is 1 and
// there is a body force (or a bulk rate other than 1): relax<..., UH = true>,
// which drops the pre-collision values of orders 3-6 from their relaxation.
template <typename T>
static void run_uh(const double* f, const double* omega, const double* F, double* out) {
  T v[3][3][3];
  for (int a = 0; a < Q; ++a) v[EZ[a] + 1][EY[a] + 1][EX[a] + 1] = (T)(f[a] - weight(a));
  Rates<T> R;
  for (int j = 0; j < Q; ++j) {
    R.w[j] = (T)omega[j];
    R.c[j] = (T)(1.0 - omega[j]);
    R.h[j] = (T)(1.0 - 0.5 * omega[j]);
  }
  const T ws[6] = {R.w[4], R.w[5], R.w[6], R.w[7], R.w[8], R.w[9]};
  const T cs[6] = {R.c[4], R.c[5], R.c[6], R.c[7], R.c[8], R.c[9]};
  T rho, ux, uy, uz;
  if (F[0] != 0.0 || F[1] != 0.0 || F[2] != 0.0)
    collide<T, true, false, false, true>(v, R, ws, cs, (T)F[0], (T)F[1], (T)F[2], rho, ux, uy, uz);
  else
    collide<T, false, false, false, true>(v, R, ws, cs, T(0), T(0), T(0), rho, ux, uy, uz);
  for (int a = 0; a < Q; ++a) out[a] = weight(a) + (double)(v[EZ[a] + 1][EY[a] + 1][EX[a] + 1] * (T)inv_factor(a));
}
extern "C" void host_collide_uh_f64(const double* f, const double* omega, const double* F, double* out) {
  run_uh<double>(f, omega, F, out);
}
extern "C" void host_collide_uh_f32(const double* f, const double* omega, const double* F, double* out) {
  run_uh<float>(f, omega, F, out);
}
// the same in storage units and on plain deviations (FP32, with a force), for a bitwise comparison
template <bool SU>
static void run_uh_dev(const float* dev, const double* omega, const double* F, float* out) {
  float v[3][3][3];
  for (int a = 0; a < Q; ++a) v[EZ[a] + 1][EY[a] + 1][EX[a] + 1] = SU ? dev[a] * dev_scale(a) : dev[a];
  Rates<float> R;
  for (int j = 0; j < Q; ++j) {
    R.w[j] = (float)omega[j];
    R.c[j] = (float)(1.0 - omega[j]);
    R.h[j] = (float)(1.0 - 0.5 * omega[j]);
  }
  const float ws[6] = {R.w[4], R.w[5], R.w[6], R.w[7], R.w[8], R.w[9]};
  const float cs[6] = {R.c[4], R.c[5], R.c[6], R.c[7], R.c[8], R.c[9]};
  float rho, ux, uy, uz;
  collide<float, true, false, SU, true>(v, R, ws, cs, (float)F[0], (float)F[1], (float)F[2], rho, ux, uy, uz);
  for (int a = 0; a < Q; ++a) out[a] = v[EZ[a] + 1][EY[a] + 1][EX[a] + 1] * (float)(1.0 / Units<SU>::U);
}
extern "C" void host_collide_uh_dev_f32(const float* dev, const double* omega, const double* F, float* out) {
  run_uh_dev<false>(dev, omega, F, out);
}
extern "C" void host_collide_uh_units_f32(const float* dev, const double* omega, const double* F, float* out) {
  run_uh_dev<true>(dev, omega, F, out);
}

// f^eq(rho, u) through the kernels' inverse sweeps (what lbm_init stores)
extern "C" void host_feq_f64(double rho, const double* u, double* out) {
  double v[3][3][3];
  for (int c = 0; c < 3; ++c)
    for (int b = 0; b < 3; ++b)
      for (int a = 0; a < 3; ++a) v[c][b][a] = (rho - 1.0) * C1[a] * C1[b] * C1[c];
  inverse_all(v, u[0], u[1], u[2]);
  for (int a = 0; a < Q; ++a) out[a] = weight(a) + v[EZ[a] + 1][EY[a] + 1][EX[a] + 1] * inv_factor(a);
}

// A periodic nx x ny x nz lattice stepped with the kernels' arithmetic (pull
// streaming, then the collision) in T, from the given populations f[27][n]
// (x fastest); ke[s] = 1/2 sum rho |u|^2 after s steps, s = 0..steps, summed in
// FP64.  general = 0: the unit-rate collision (the paper's rates, no force);
// 1: the general one with the same rates.
template <typename T>
static void run_lattice(int nx, int ny, int nz, const double* f, const double* omega, int steps, int general,
                        double* ke) {
  const size_t n = (size_t)nx * ny * nz;
  std::vector<T> a(Q * n), b(Q * n);
  for (int q = 0; q < Q; ++q)
    for (size_t i = 0; i < n; ++i) a[q * n + i] = (T)(f[q * n + i] - weight(q));
  Rates<T> R;
  for (int j = 0; j < Q; ++j) {
    R.w[j] = (T)omega[j];
    R.c[j] = (T)(1.0 - omega[j]);
    R.h[j] = (T)(1.0 - 0.5 * omega[j]);
  }
  const T ws[6] = {R.w[4], R.w[5], R.w[6], R.w[7], R.w[8], R.w[9]};
  const T cs[6] = {R.c[4], R.c[5], R.c[6], R.c[7], R.c[8], R.c[9]};
  for (int s = 0;; ++s) {
    double e = 0;
    for (size_t i = 0; i < n; ++i) {
      double r = 1, jx = 0, jy = 0, jz = 0;
      for (int q = 0; q < Q; ++q) {
        const double d = (double)a[q * n + i];
        r += d;
        jx += d * EX[q];
        jy += d * EY[q];
        jz += d * EZ[q];
      }
      e += 0.5 * (jx * jx + jy * jy + jz * jz) / r;
    }
    ke[s] = e;
    if (s == steps) break;
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          T v[3][3][3];
          for (int q = 0; q < Q; ++q) {
            const int xs = (x - EX[q] + nx) % nx, ys = (y - EY[q] + ny) % ny, zs = (z - EZ[q] + nz) % nz;
            v[EZ[q] + 1][EY[q] + 1][EX[q] + 1] = a[q * n + ((size_t)zs * ny + ys) * nx + xs];
          }
          T rho, ux, uy, uz;
          if (general) collide<T, false, false>(v, R, ws, cs, T(0), T(0), T(0), rho, ux, uy, uz);
          else collide_unit_higher<T>(v, cs, rho, ux, uy, uz);
          const size_t i = ((size_t)z * ny + y) * nx + x;
          for (int q = 0; q < Q; ++q) b[q * n + i] = v[EZ[q] + 1][EY[q] + 1][EX[q] + 1] * (T)inv_factor(q);
        }
    a.swap(b);
  }
}
extern "C" void host_lattice_ke_f64(int nx, int ny, int nz, const double* f, const double* omega, int steps,
                                    int general, double* ke) {
  run_lattice<double>(nx, ny, nz, f, omega, steps, general, ke);
}
extern "C" void host_lattice_ke_f32(int nx, int ny, int nz, const double* f, const double* omega, int steps,
                                    int general, double* ke) {
  run_lattice<float>(nx, ny, nz, f, omega, steps, general, ke);
}

// The step kernels' launch mapping (lbm_internal.hpp: step_launch_shape,
// make_geom, segment_of) enumerated on the host for an nx x ny x nz lattice:
// count[i] = how many lanes map to node i (x fastest), *bad = the number of
// wavefronts whose lanes disagree on (y, z) or hold x outside one 64-node
// segment.  Returns the number of blocks.
#include "../../paper_2410_09739_amd/csrc/lattice.hpp"
extern "C" long long host_launch_cover(int nx, int ny, int nz, int storage, int* count, long long* bad) {
  lbm_config cfg{};
  cfg.storage = (lbm_storage)storage;
  cfg.nx = nx;
  cfg.ny = ny;
  cfg.nz = nz;
  const Geom g = make_geom(&cfg);
  dim3 block, grid;
  step_launch_shape(nx, ny, nz, block, grid);
  *bad = 0;
  for (uint32_t bz = 0; bz < grid.z; ++bz)
    for (uint32_t by = 0; by < grid.y; ++by)
      for (uint32_t bx = 0; bx < grid.x; ++bx)
        for (uint32_t w = 0; w < block.x / 64; ++w) {
          int y0 = -1, z0 = -1, seg = -1;
          for (uint32_t lane = 0; lane < 64; ++lane) {
            int x, y, z;
            if (!segment_of(g, bx, by, bz, grid.x, grid.y, block.x, w, lane, x, y, z)) continue;
            if (lane == 0) {
              y0 = y;
              z0 = z;
              seg = x / 64;
            }
            if (y != y0 || z != z0 || x / 64 != seg || x % 64 != (int)lane) ++*bad;
            if (x >= nx) continue;  // padding lanes of a ragged row return at once
            if (y < 0 || y >= ny || z < 0 || z >= nz || x < 0) {
              ++*bad;
              continue;
            }
            ++count[((size_t)z * ny + y) * nx + x];
          }
        }
  return (long long)grid.x * grid.y * grid.z;
}
