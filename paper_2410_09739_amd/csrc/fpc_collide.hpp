// fpc_collide.hpp -- per-node FPC-LBM collision in registers (device code).
//
// The state of one node is a 3x3x3 register cube v[iz][iy][ix] indexed by the
// velocity (ix = e_x + 1, ...).  It holds deviations delta = f - w_alpha from
// the lattice weights, never f itself, so that FP32 arithmetic keeps the small
// non-equilibrium and force contributions (the weights would otherwise take
// most of the mantissa).
//
// Raw and central moments of the paper (Appendix D Steps 1 and 2: m = P f,
// kappa = F(u) m) are both tensor products over the three axes, because the
// D3Q27 moment set is {0,1,2}^3.  So kappa = F(u) P f is computed as three
// sweeps of a 3-point transform, one per axis, that map the values at
// e = -1, 0, +1 straight to the central moments of order 0, 1, 2 about u_d.
// Each sweep also carries the rest state's contribution as a compile-time
// constant W, so that the cube ends up holding kappa' = kappa - E with
// E_abc = C1[a] C1[b] C1[c] the rest-state central moments (C1 = 1, 0, c_s^2).
// Steps 4 and 5 (m~ = F^-1 kappa~, f~ = P^-1 m~) are the inverse sweeps; they
// return each deviation times an exact power of two (inv_shift), which the
// caller removes when it stores the value.
//
// The collision (Step 3) relaxes the primed moments in the paper's order:
// orders 0-2 (grouped 2s1/2d1/2d2), decomposition, order 3 (3s*/3m*, 111),
// decomposition, order 4 with attractors from post-collision order 2
// (4s1/4d1/4d2, 211/121/112), decomposition, order 5 from post-collision
// orders 2 and 3, order 6 from post-collision orders 2 and 4.  Attractors are
// those of Sec. 3.5 (Eq. Mvcmattractor3D with the diffusion tensor of
// Eq. diffusion-tensor-parameter-3D), rewritten exactly for primed moments;
// sources follow Eq. (cmupdatesourceD3Q27) with the pre-collision moments,
// kappa_000 = rho and first-order moments taken as zero.  kappa^Mv_122 uses the
// product kappa~_110 kappa~_012 that the general attractor formula gives.
//
// Storage units (SU = true, the FP16/BF16 deviation forms): the cube holds
// each deviation times its storage scale dev_scale(alpha) = 2^(12 + 2|e|^2),
// i.e. the stored numbers themselves, so that loading a value needs no
// multiply.  The two outer points of every 3-point line share a scale and the
// middle one has a quarter of it, so each sweep takes its middle value times 4
// and its outputs carry the outer points' scale; after the three forward
// sweeps every moment carries the one factor UNIT = 2^18 (Units<SU>::U).  The collision then
// runs on moments times UNIT: constants of the rest state and the force are
// taken times UNIT and 1/rho (where it multiplies a product of two moments)
// times 1/UNIT.  Every such factor is an exact power of two, so the results
// are bitwise those of the same arithmetic on plain deviations (no FP32
// underflow or overflow is reached at these scales).
//
// MAXWELL = true is the comparison model with Maxwellian equilibria (the
// MCM-LBM of Sec. 4): orders >= 4 relax to the discrete Maxwellian's central
// moments rho c_a c_b c_c (c = 1, 0, c_s^2) instead of the Markovian
// attractors; orders <= 3, rates, grouping and sources are unchanged.
#pragma once

#include <hip/hip_runtime.h>

#include "d3q27.hpp"

namespace fpc {

// 1/x: FP64 and host builds divide.  FP32 on the GPU takes the hardware
// reciprocal (v_rcp_f32) and one Newton step, r' = r + r (1 - x r) with the
// residual from a fused multiply-add, instead of the ten-instruction IEEE
// division.  The hardware value is within 1 ulp but not always the nearest
// (measured: about one value in nine one ulp off for x near 1, most of them
// above, so it is biased); after the step it is the correctly rounded 1/x
// (measured on 4M values in each of [0.5, 2] and [0.999, 1.001]).
template <typename T>
__host__ __device__ __forceinline__ T recip(T x) {
  return T(1) / x;
}
template <>
__host__ __device__ __forceinline__ float recip<float>(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const float r = __builtin_amdgcn_rcpf(x);
  return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
#else
  return 1.0f / x;
#endif
}

template <typename T>
struct Rates {
  T w[Q];   // omega_0 .. omega_26 (Appendix D numbering)
  T c[Q];   // 1 - omega_j
  T h[Q];   // 1 - omega_j / 2
};

// Factors of the storage units (see the header).  line(k): factor carried by
// the outputs of a forward sweep whose outer points have k + 1 non-zero
// velocity components; U: factor carried by the moments after all three.
template <bool SU>
struct Units {
  static constexpr int M = SU ? 4 : 1;  // middle point of a line, in its outer points' units
  static constexpr double line(int k) { return SU ? double(1u << (DEV_LOG2_0 + 2 * (k + 1))) : 1.0; }
  static constexpr double U = line(2);
};

// 1 / rho for rho = 1 + x, x = rho' (the density deviation; rhop carries UNIT
// in storage units), without rounding 1 + x first.  The momentum the
// collision rebuilds is (1 + x) u with u = j / rho; taken as j / fl(1 + x), it
// is off by the rounding of 1 + x (up to 6e-8 in FP32), and these offsets do
// not average out: on the Taylor-Green vortex they added about 4e-9 of the
// kinetic energy per step.  One Newton step on the exact 1 + x,
// r' = r + r e with e = (1 - r) - x r (1 - r is exact for r in [1/2, 2]),
// from the hardware reciprocal of fl(1 + x) gives 1 / (1 + x) to within about
// half an ulp.
template <typename T, bool SU = false>
__host__ __device__ __forceinline__ T recip_rho(T rhop) {
  const T x = rhop * T(1.0 / Units<SU>::U);
#if defined(__HIP_DEVICE_COMPILE__)
  const T r = sizeof(T) == sizeof(float) ? T(__builtin_amdgcn_rcpf(float(T(1) + x))) : T(1) / (T(1) + x);
#else
  const T r = T(1) / (T(1) + x);
#endif
  const T e = fma(-x, r, T(1) - r);
  return fma(r, e, r);
}


// ---------------------------------------------------------------------------
// 3-point sweeps.  Forward: values (dm, d0, dp) at e = -1, 0, +1, deviations
// from W * (1/6, 2/3, 1/6)  ->  central moments (r0, r1, r2) about u, minus
// W * (1, 0, 1/3).
// M: the middle value's factor (4 in storage units, see Units).
template <typename T, int WNUM_IS_ZERO, int M = 1>
__host__ __device__ __forceinline__ void fwd3(T& a0, T& a1, T& a2, T u, T W) {
  const T sp = a2 + a0;
  const T s0 = sp + T(M) * a1;
  const T d1 = a2 - a0;
  const T S = WNUM_IS_ZERO ? s0 : s0 + W;
  a0 = s0;
  a1 = d1 - u * S;
  a2 = sp - T(2) * u * d1 + u * u * S;
}

// Inverse: (r0, r1, r2) as produced by fwd3 -> deviations at e = -1, 0, +1,
// with the two outer values returned doubled: with the raw moments
// m1 = R0 u + r1 and m2 = R0 u^2 + 2 u r1 + r2 (R0 = r0 + W) of the line,
// the values are d(0) = r0 - m2 and d(+-1) = (m2 +- m1) / 2; the halving is
// left to the caller (an exact power of two folded into the store).
template <typename T, int WNUM_IS_ZERO>
__host__ __device__ __forceinline__ void inv3(T& a0, T& a1, T& a2, T u, T u2, T two_u, T W) {
  const T r0 = a0, r1 = a1, r2 = a2;
  const T R0 = WNUM_IS_ZERO ? r0 : r0 + W;
  const T m1 = R0 * u + r1;
  const T m2 = R0 * u2 + (two_u * r1 + r2);
  a1 = r0 - m2;
  a2 = m2 + m1;
  a0 = m2 - m1;
}

// log2 of the factor inverse_all leaves on the value of direction alpha:
// one doubling per non-zero velocity component.
constexpr int inv_shift(int a) { return (EX[a] != 0) + (EY[a] != 0) + (EZ[a] != 0); }
constexpr double inv_factor(int a) { return 1.0 / double(1 << inv_shift(a)); }

// Forward sweeps over the cube (x, then y, then z).  On return v[c][b][a] holds
// kappa'_abc.  The x sweep is split so that rho and j come out of its line sums.
template <typename T, bool SU = false>
__host__ __device__ __forceinline__ void forward_x(T (&v)[3][3][3], T ux) {
  using Un = Units<SU>;
#pragma unroll
  for (int iz = 0; iz < 3; ++iz)
#pragma unroll
    for (int iy = 0; iy < 3; ++iy)
      fwd3<T, 0, Un::M>(v[iz][iy][0], v[iz][iy][1], v[iz][iy][2], ux,
                        T(W1[iy] * W1[iz] * Un::line((iy != 1) + (iz != 1))));
}

template <typename T, bool SU = false>
__host__ __device__ __forceinline__ void forward_yz(T (&v)[3][3][3], T uy, T uz) {
  using Un = Units<SU>;
#pragma unroll
  for (int iz = 0; iz < 3; ++iz) {
    const double l = Un::line(1 + (iz != 1));
    fwd3<T, 0, Un::M>(v[iz][0][0], v[iz][1][0], v[iz][2][0], uy, T(C1[0] * W1[iz] * l));
    fwd3<T, 1, Un::M>(v[iz][0][1], v[iz][1][1], v[iz][2][1], uy, T(0));
    fwd3<T, 0, Un::M>(v[iz][0][2], v[iz][1][2], v[iz][2][2], uy, T(C1[2] * W1[iz] * l));
  }
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (a == 1 || b == 1)
        fwd3<T, 1, Un::M>(v[0][b][a], v[1][b][a], v[2][b][a], uz, T(0));
      else
        fwd3<T, 0, Un::M>(v[0][b][a], v[1][b][a], v[2][b][a], uz, T(C1[a] * C1[b] * Un::U));
    }
}

// Rest-state constants of the inverse-sweep lines that rebuild the momentum:
// the y lines of x-order 0 (rest weight W1[iz], times 2 for an outer z line,
// which the z sweep doubled) and every x line (W1[iy] W1[iz], times the
// doublings of both earlier sweeps).  In exact arithmetic the rest weights of
// the lines of one sweep sum to 1, so the momentum is rebuilt as rho u.  The
// nearest FP32 values do not: the y lines give 1 + 2^-25 and the x lines
// 1 + 2^-27, so every collision would scale u_y and u_x by that factor, a
// steady gain of kinetic energy of about 4e-8 of it per step on the
// Taylor-Green vortex.  For FP32 one constant of each sweep is taken one unit
// in the last place below the nearest value (the outer y lines, 1/3 -> 11184810
// 2^-25; the corner x lines, 1/9 -> 14913080 2^-27), which makes each sum
// exactly 1.  FP64 keeps the nearest values (its excess is 2^-54 per step).
template <typename T>
constexpr double rest_y(int iz) {
  return iz == 1 ? W1[1] : (sizeof(T) == sizeof(float) ? 11184810.0 / 33554432.0 : 2.0 * W1[0]);
}
template <typename T>
constexpr double rest_x(int iy, int iz) {
  const int outer = (iy != 1) + (iz != 1);
  if (outer == 2 && sizeof(T) == sizeof(float)) return 14913080.0 / 134217728.0;
  return W1[iy] * W1[iz] * double(1 << outer);
}

// Inverse sweeps (z, then y, then x).  Each sweep doubles the values it writes
// at e = +-1, so the line constants W of a later sweep are scaled by the
// doublings its inputs already carry; on return the cube holds
// delta_alpha * 2^inv_shift(alpha).
template <typename T, bool SU = false>
__host__ __device__ __forceinline__ void inverse_all(T (&v)[3][3][3], T ux, T uy, T uz) {
  constexpr double U = Units<SU>::U;  // the line constants in the moments' units
  const T uz2 = uz * uz, uy2 = uy * uy, ux2 = ux * ux;
  const T tz = uz + uz, ty = uy + uy, tx = ux + ux;
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (a == 1 || b == 1)
        inv3<T, 1>(v[0][b][a], v[1][b][a], v[2][b][a], uz, uz2, tz, T(0));
      else
        inv3<T, 0>(v[0][b][a], v[1][b][a], v[2][b][a], uz, uz2, tz, T(C1[a] * C1[b] * U));
    }
#pragma unroll
  for (int iz = 0; iz < 3; ++iz) {
    const double sz = iz == 1 ? 1.0 : 2.0;
    inv3<T, 0>(v[iz][0][0], v[iz][1][0], v[iz][2][0], uy, uy2, ty, T(rest_y<T>(iz) * U));
    inv3<T, 1>(v[iz][0][1], v[iz][1][1], v[iz][2][1], uy, uy2, ty, T(0));
    inv3<T, 0>(v[iz][0][2], v[iz][1][2], v[iz][2][2], uy, uy2, ty, T(C1[2] * W1[iz] * sz * U));
  }
#pragma unroll
  for (int iz = 0; iz < 3; ++iz)
#pragma unroll
    for (int iy = 0; iy < 3; ++iy) {
      inv3<T, 0>(v[iz][iy][0], v[iz][iy][1], v[iz][iy][2], ux, ux2, tx, T(rest_x<T>(iy, iz) * U));
    }
}

// Macroscopic fields from the deviation cube: rho' = sum delta, j = sum delta e
// (in storage units: times UNIT).  The sums are the line sums and differences
// of the forward sweeps, in the same order, so the compiler computes them once
// for both; every 3-point combination weights its middle term by M.
template <typename T, bool SU = false>
__host__ __device__ __forceinline__ void density_momentum(const T (&v)[3][3][3], T& rhop, T& jx, T& jy, T& jz) {
  constexpr int M = Units<SU>::M;
  T s[3][3], d[3][3], p[3], q[3], r[3];
#pragma unroll
  for (int iz = 0; iz < 3; ++iz)
#pragma unroll
    for (int iy = 0; iy < 3; ++iy) {
      s[iz][iy] = (v[iz][iy][2] + v[iz][iy][0]) + T(M) * v[iz][iy][1];
      d[iz][iy] = v[iz][iy][2] - v[iz][iy][0];
    }
#pragma unroll
  for (int iz = 0; iz < 3; ++iz) {
    p[iz] = (s[iz][2] + s[iz][0]) + T(M) * s[iz][1];
    q[iz] = (d[iz][2] + d[iz][0]) + T(M) * d[iz][1];
    r[iz] = s[iz][2] - s[iz][0];
  }
  jx = (q[2] + q[0]) + T(M) * q[1];
  jy = (r[2] + r[0]) + T(M) * r[1];
  jz = p[2] - p[0];
  rhop = (p[2] + p[0]) + T(M) * p[1];
}

// ---------------------------------------------------------------------------
// Pre-collision part of one node: Step 7 fields (rho = 1 + rho', rho u =
// sum f e + F/2) and the forward sweeps; on return v holds kappa' (and rhop
// rho', both times UNIT in storage units; rho and u are plain).
template <typename T, bool FORCE, bool SU = false>
__host__ __device__ __forceinline__ void pre_collision(T (&v)[3][3][3], T Fx, T Fy, T Fz, T& rhop, T& rho,
                                                       T& ux, T& uy, T& uz) {
  constexpr double U = Units<SU>::U;
  T jx, jy, jz;
  density_momentum<T, SU>(v, rhop, jx, jy, jz);
  rho = T(1) + rhop * T(1.0 / U);
  const T iru = recip_rho<T, SU>(rhop) * T(1.0 / U);
  if (FORCE) {
    jx += T(0.5 * U) * Fx;
    jy += T(0.5 * U) * Fy;
    jz += T(0.5 * U) * Fz;
  }
  ux = jx * iru;
  uy = jy * iru;
  uz = jz * iru;
  forward_x<T, SU>(v, ux);
  forward_yz<T, SU>(v, uy, uz);
}

// Step 3 on the primed moments in v (as left by pre_collision), then the
// inverse sweeps.  ws[6], cs[6]: the second-order rates omega_4..omega_9 to use
// at this node (the rates table, or a per-node closure) and 1 - ws.
// In storage units (SU) v and rhop carry UNIT, rho and u are plain: the rest
// state's constants are taken times UNIT (thirdU, ninthU) and a product of two
// moments is scaled by iru = 1 / (rho UNIT).
// UH (unit higher): every rate of orders 3-6 (omega_10..omega_26) is 1, as in
// all runs of the paper (Sec. 4); R.w/c/h[10..26] are then not read.  A group
// relaxed at rate 1 lands on its attractor plus half its source,
// kappa~ = kappa + 1 (kappa^Mv - kappa) + (1 - 1/2) sigma, whatever its
// pre-collision value, and since all members of a decomposition family share
// the rate, each member does so on its own (t_abc = kappa^Mv_abc + sigma_abc/2).
// The pre-collision moments of orders 3-5 still enter through the sources.
// The second order (bulk rate included) stays general.  Equal to UH = false
// with those rates up to rounding.
template <typename T, bool FORCE, bool MAXWELL = false, bool SU = false, bool UH = false>
__host__ __device__ __forceinline__ void relax(T (&v)[3][3][3], const Rates<T>& R, const T (&ws)[6],
                                               const T (&cs)[6], T Fx, T Fy, T Fz, T rhop, T rho, T ux,
                                               T uy, T uz) {
  static_assert(!(UH && MAXWELL), "the unit-rate form takes the Markovian attractors");
  constexpr double U = Units<SU>::U;
  const T third = T(1.0 / 3.0), ninth = T(1.0 / 9.0);
  const T thirdU = T(U / 3.0), ninthU = T(U / 9.0);
  const T ir = recip_rho<T, SU>(rhop);
  const T iru = ir * T(1.0 / U);

  // pre-collision primed central moments (v[c][b][a] = kappa'_abc)
  const T k100 = v[0][0][1], k010 = v[0][1][0], k001 = v[1][0][0];
  const T k110 = v[0][1][1], k101 = v[1][0][1], k011 = v[1][1][0];
  const T k200 = v[0][0][2], k020 = v[0][2][0], k002 = v[2][0][0];
  const T k120 = v[0][2][1], k102 = v[2][0][1], k210 = v[0][1][2];
  const T k012 = v[2][1][0], k201 = v[1][0][2], k021 = v[1][2][0];
  const T k111 = v[1][1][1];
  const T k220 = v[0][2][2], k202 = v[2][0][2], k022 = v[2][2][0];
  const T k211 = v[1][1][2], k121 = v[1][2][1], k112 = v[2][1][1];
  const T k122 = v[2][2][1], k212 = v[2][1][2], k221 = v[1][2][2];
  const T k222 = v[2][2][2];

  // sources sigma_abc = a gx K_(a-1)bc + b gy K_a(b-1)c + c gz K_ab(c-1), full K = E + kappa'
  T s100 = 0, s010 = 0, s001 = 0;
  T s120 = 0, s102 = 0, s210 = 0, s012 = 0, s201 = 0, s021 = 0, s111 = 0;
  T s220 = 0, s202 = 0, s022 = 0, s211 = 0, s121 = 0, s112 = 0;
  T s122 = 0, s212 = 0, s221 = 0, s222 = 0;
  if (FORCE) {
    // UH: orders 3-6 take half their source, so the sources of those orders are
    // formed at once with g / 2 (an exact power-of-two factor); s100..s001 stay whole.
    const T irs = UH ? T(0.5) * ir : ir;
    const T gx = Fx * irs, gy = Fy * irs, gz = Fz * irs;
    const T K200 = thirdU + k200, K020 = thirdU + k020, K002 = thirdU + k002;
    const T K220 = ninthU + k220, K202 = ninthU + k202, K022 = ninthU + k022;
    s100 = T(U) * Fx;
    s010 = T(U) * Fy;
    s001 = T(U) * Fz;
    s120 = gx * K020 + T(2) * gy * k110;
    s102 = gx * K002 + T(2) * gz * k101;
    s210 = T(2) * gx * k110 + gy * K200;
    s012 = gy * K002 + T(2) * gz * k011;
    s201 = T(2) * gx * k101 + gz * K200;
    s021 = T(2) * gy * k011 + gz * K020;
    s111 = gx * k011 + gy * k101 + gz * k110;
    s220 = T(2) * (gx * k120 + gy * k210);
    s202 = T(2) * (gx * k102 + gz * k201);
    s022 = T(2) * (gy * k012 + gz * k021);
    s211 = T(2) * gx * k111 + gy * k201 + gz * k210;
    s121 = gx * k021 + T(2) * gy * k111 + gz * k120;
    s112 = gx * k012 + gy * k102 + T(2) * gz * k111;
    s122 = gx * K022 + T(2) * (gy * k112 + gz * k121);
    s212 = gy * K202 + T(2) * (gx * k112 + gz * k211);
    s221 = gz * K220 + T(2) * (gx * k121 + gy * k211);
    s222 = T(2) * (gx * k122 + gy * k212 + gz * k221);
  }

  // ---- orders 0-2.  kappa~_000 = rho' (conserved); first order: attractor 0.
  // First order: kappa = -F/2 before collision (u carries the F/2 shift), so
  // kappa + omega (0 - kappa) + (1 - omega/2) F = F/2 for every omega_1..3.
  const T t100 = T(0.5) * s100, t010 = T(0.5) * s010, t001 = T(0.5) * s001;
  (void)k100; (void)k010; (void)k001;
  const T t110 = cs[0] * k110;  // sigma_110 = 0
  const T t101 = cs[1] * k101;
  const T t011 = cs[2] * k011;
  const T c2s1 = k200 + k020 + k002;      // primed: attractor rho c_s^2 * 3 -> rho'
  const T c2d1 = k200 - k020, c2d2 = k200 - k002;
  const T t2s1 = c2s1 + ws[3] * (rhop - c2s1);  // sigma_200 = sigma_020 = sigma_002 = 0
  const T t2d1 = cs[4] * c2d1;
  const T t2d2 = cs[5] * c2d2;
  const T t200 = third * (t2s1 + t2d1 + t2d2);
  const T t020 = third * (t2s1 - T(2) * t2d1 + t2d2);
  const T t002 = third * (t2s1 + t2d1 - T(2) * t2d2);

  T t120, t102, t210, t012, t201, t021, t111, t220, t202, t022, t211, t121, t112, t122, t212, t221, t222;
  if constexpr (UH) {
    // ---- orders 3-6 at rate 1: attractor + sigma / 2 (the s here are already halved)
    (void)R;
    t120 = s120; t102 = s102; t210 = s210; t012 = s012; t201 = s201; t021 = s021; t111 = s111;
    // order 4 from post-collision order 2
    const T A2 = thirdU + t200, B2 = thirdU + t020, C2 = thirdU + t002;
    t220 = ((t200 + t020) * thirdU + t200 * t020 + T(2) * t110 * t110 - ninthU * rhop) * iru + s220;
    t202 = ((t200 + t002) * thirdU + t200 * t002 + T(2) * t101 * t101 - ninthU * rhop) * iru + s202;
    t022 = ((t020 + t002) * thirdU + t020 * t002 + T(2) * t011 * t011 - ninthU * rhop) * iru + s022;
    t211 = (A2 * t011 + T(2) * t110 * t101) * iru + s211;
    t121 = (B2 * t101 + T(2) * t110 * t011) * iru + s121;
    t112 = (C2 * t110 + T(2) * t011 * t101) * iru + s112;
    // order 5 from post-collision orders 2 and 3
    const T f5 = T(0.4) * iru;  // 2 / (5 rho)
    t122 = f5 * (B2 * t102 + C2 * t120 + T(4) * t011 * t111 + T(2) * (t101 * t021 + t110 * t012)) + s122;
    t212 = f5 * (A2 * t012 + C2 * t210 + T(4) * t101 * t111 + T(2) * (t110 * t102 + t011 * t201)) + s212;
    t221 = f5 * (A2 * t021 + B2 * t201 + T(4) * t110 * t111 + T(2) * (t011 * t210 + t101 * t120)) + s221;
    // order 6 from post-collision orders 2 and 4
    t222 = ((t200 + t020 + t002) * ninthU + (t022 + t202 + t220) * thirdU + t200 * t022 + t020 * t202 +
            t002 * t220 + T(4) * (t110 * t112 + t101 * t121 + t011 * t211)) *
               (third * iru) -
           rhop * (T(1.0 / 27.0) * ir) + s222;
    (void)k120; (void)k102; (void)k210; (void)k012; (void)k201; (void)k021; (void)k111;
    (void)k220; (void)k202; (void)k022; (void)k211; (void)k121; (void)k112;
    (void)k122; (void)k212; (void)k221; (void)k222;
  } else {
    // ---- order 3: attractors 0.
    const T t3s1 = R.c[10] * (k120 + k102) + R.h[10] * (s120 + s102);
    const T t3m1 = R.c[11] * (k120 - k102) + R.h[11] * (s120 - s102);
    const T t3s2 = R.c[12] * (k210 + k012) + R.h[12] * (s210 + s012);
    const T t3m2 = R.c[13] * (k210 - k012) + R.h[13] * (s210 - s012);
    const T t3s3 = R.c[14] * (k201 + k021) + R.h[14] * (s201 + s021);
    const T t3m3 = R.c[15] * (k201 - k021) + R.h[15] * (s201 - s021);
    t111 = R.c[16] * k111 + R.h[16] * s111;
    t120 = T(0.5) * (t3s1 + t3m1); t102 = T(0.5) * (t3s1 - t3m1);
    t210 = T(0.5) * (t3s2 + t3m2); t012 = T(0.5) * (t3s2 - t3m2);
    t201 = T(0.5) * (t3s3 + t3m3); t021 = T(0.5) * (t3s3 - t3m3);

    // ---- order 4: attractors from post-collision order 2 (primed form of
    // (K200 K020 + 2 K110^2)/rho - 1/9 etc.).
    // (Maxwellian model: rho' c_s^4 and 0, the primed discrete Maxwellian.)
    const T m220 = MAXWELL ? ninth * rhop : ((t200 + t020) * thirdU + t200 * t020 + T(2) * t110 * t110 - ninthU * rhop) * iru;
    const T m202 = MAXWELL ? ninth * rhop : ((t200 + t002) * thirdU + t200 * t002 + T(2) * t101 * t101 - ninthU * rhop) * iru;
    const T m022 = MAXWELL ? ninth * rhop : ((t020 + t002) * thirdU + t020 * t002 + T(2) * t011 * t011 - ninthU * rhop) * iru;
    const T A2 = thirdU + t200, B2 = thirdU + t020, C2 = thirdU + t002;  // full post-collision order 2
    const T m211 = MAXWELL ? T(0) : (A2 * t011 + T(2) * t110 * t101) * iru;
    const T m121 = MAXWELL ? T(0) : (B2 * t101 + T(2) * t110 * t011) * iru;
    const T m112 = MAXWELL ? T(0) : (C2 * t110 + T(2) * t011 * t101) * iru;
    const T c4s1 = k220 + k202 + k022, c4d1 = k220 + k202 - k022, c4d2 = k220 - k202;
    const T t4s1 = c4s1 + R.w[17] * ((m220 + m202 + m022) - c4s1) + R.h[17] * (s220 + s202 + s022);
    const T t4d1 = c4d1 + R.w[18] * ((m220 + m202 - m022) - c4d1) + R.h[18] * (s220 + s202 - s022);
    const T t4d2 = c4d2 + R.w[19] * ((m220 - m202) - c4d2) + R.h[19] * (s220 - s202);
    t211 = k211 + R.w[20] * (m211 - k211) + R.h[20] * s211;
    t121 = k121 + R.w[21] * (m121 - k121) + R.h[21] * s121;
    t112 = k112 + R.w[22] * (m112 - k112) + R.h[22] * s112;
    t220 = T(0.25) * (t4s1 + t4d1 + T(2) * t4d2);
    t202 = T(0.25) * (t4s1 + t4d1 - T(2) * t4d2);
    t022 = T(0.5) * (t4s1 - t4d1);

    // ---- order 5: attractors from post-collision orders 2 and 3.
    const T f5 = T(0.4) * iru;  // 2 / (5 rho)
    const T m122 = MAXWELL ? T(0) : f5 * (B2 * t102 + C2 * t120 + T(4) * t011 * t111 + T(2) * (t101 * t021 + t110 * t012));
    const T m212 = MAXWELL ? T(0) : f5 * (A2 * t012 + C2 * t210 + T(4) * t101 * t111 + T(2) * (t110 * t102 + t011 * t201));
    const T m221 = MAXWELL ? T(0) : f5 * (A2 * t021 + B2 * t201 + T(4) * t110 * t111 + T(2) * (t011 * t210 + t101 * t120));
    t122 = k122 + R.w[23] * (m122 - k122) + R.h[23] * s122;
    t212 = k212 + R.w[24] * (m212 - k212) + R.h[24] * s212;
    t221 = k221 + R.w[25] * (m221 - k221) + R.h[25] * s221;

    // ---- order 6: attractor from post-collision orders 2 and 4 (primed form).
    const T m222 = MAXWELL ? rhop * T(1.0 / 27.0) : ((t200 + t020 + t002) * ninthU + (t022 + t202 + t220) * thirdU + t200 * t022 + t020 * t202 +
                    t002 * t220 + T(4) * (t110 * t112 + t101 * t121 + t011 * t211)) *
                       (third * iru) -
                   rhop * (T(1.0 / 27.0) * ir);
    t222 = k222 + R.w[26] * (m222 - k222) + R.h[26] * s222;
  }

  v[0][0][0] = rhop;
  v[0][0][1] = t100; v[0][1][0] = t010; v[1][0][0] = t001;
  v[0][1][1] = t110; v[1][0][1] = t101; v[1][1][0] = t011;
  v[0][0][2] = t200; v[0][2][0] = t020; v[2][0][0] = t002;
  v[0][2][1] = t120; v[2][0][1] = t102; v[0][1][2] = t210;
  v[2][1][0] = t012; v[1][0][2] = t201; v[1][2][0] = t021;
  v[1][1][1] = t111;
  v[0][2][2] = t220; v[2][0][2] = t202; v[2][2][0] = t022;
  v[1][1][2] = t211; v[1][2][1] = t121; v[2][1][1] = t112;
  v[2][2][1] = t122; v[2][1][2] = t212; v[1][2][2] = t221;
  v[2][2][2] = t222;

  inverse_all<T, SU>(v, ux, uy, uz);
}

// ---------------------------------------------------------------------------
// The collision with the rates of the paper's runs (Sec. 4: bulk rate omega_7
// and every rate of orders 3-6 equal to 1) and no body force.  A group relaxed
// at rate 1 lands on its attractor: order 3 on 0, the orders-4 and -5
// attractors are built from the post-collision orders 2 and 3, order 6 from
// orders 2 and 4 (Sec. 3.5), and the 2s1 combination on its equilibrium rho'.
// So the post-collision cube depends only on rho', u and the five
// second-order moments that relax at the shear rates (110, 101, 011, 2d1,
// 2d2): none of the pre-collision moments of order 3 or higher is needed.
// They are not computed.  The second-order central moments come from the raw
// ones about the origin, kappa_ab = M_ab - j_a u_b (j = rho u without a
// force), the raw moments from line sums of the cube.  The result equals the
// general relax() up to rounding; that one computes kappa + 1 (kappa^Mv - kappa).

// Raw moments of orders 0-2 of the deviation cube (times UNIT in storage
// units): m0 = rho', j = sum delta e, m2 = (200, 020, 002, 110, 101, 011).
// One pass per axis over line sums, as density_momentum, keeping the pair
// sums f(+1) + f(-1) that give the second order.
template <typename T, bool SU = false>
__host__ __device__ __forceinline__ void low_moments(const T (&v)[3][3][3], T& m0, T& jx, T& jy, T& jz, T (&m2)[6]) {
  constexpr int M = Units<SU>::M;
  // x: order 0, 1, 2 of every (y, z) line
  T s[3][3], d[3][3], p[3][3];
#pragma unroll
  for (int iz = 0; iz < 3; ++iz)
#pragma unroll
    for (int iy = 0; iy < 3; ++iy) {
      p[iz][iy] = v[iz][iy][2] + v[iz][iy][0];
      s[iz][iy] = p[iz][iy] + T(M) * v[iz][iy][1];
      d[iz][iy] = v[iz][iy][2] - v[iz][iy][0];
    }
  // y: (x order, y order) = (0,0), (0,1), (0,2), (1,0), (1,1), (2,0) per z plane
  T a00[3], a01[3], a02[3], a10[3], a11[3], a20[3];
#pragma unroll
  for (int iz = 0; iz < 3; ++iz) {
    a02[iz] = s[iz][2] + s[iz][0];
    a00[iz] = a02[iz] + T(M) * s[iz][1];
    a01[iz] = s[iz][2] - s[iz][0];
    a10[iz] = (d[iz][2] + d[iz][0]) + T(M) * d[iz][1];
    a11[iz] = d[iz][2] - d[iz][0];
    a20[iz] = (p[iz][2] + p[iz][0]) + T(M) * p[iz][1];
  }
  // z
  const T zz = a00[2] + a00[0];
  m0 = zz + T(M) * a00[1];
  jz = a00[2] - a00[0];
  jy = (a01[2] + a01[0]) + T(M) * a01[1];
  jx = (a10[2] + a10[0]) + T(M) * a10[1];
  m2[0] = (a20[2] + a20[0]) + T(M) * a20[1];  // 200
  m2[1] = (a02[2] + a02[0]) + T(M) * a02[1];  // 020
  m2[2] = zz;                                  // 002
  m2[3] = (a11[2] + a11[0]) + T(M) * a11[1];  // 110
  m2[4] = a10[2] - a10[0];                     // 101
  m2[5] = a01[2] - a01[0];                     // 011
}

// Step 7 fields and the primed second-order central moments without a force:
// k2 = (kappa'_200, kappa'_020, kappa'_002, kappa_110, kappa_101, kappa_011),
// kappa'_aa = kappa_aa - c_s^2 (the rest state's part; it is M'_aa - j_a u_a
// for the deviation moments M').  Storage units as pre_collision.
template <typename T, bool SU = false>
__host__ __device__ __forceinline__ void second_order_central(const T (&v)[3][3][3], T& rhop, T& rho, T& ux, T& uy,
                                                              T& uz, T (&k2)[6]) {
  constexpr double U = Units<SU>::U;
  T jx, jy, jz, m2[6];
  low_moments<T, SU>(v, rhop, jx, jy, jz, m2);
  rho = T(1) + rhop * T(1.0 / U);
  const T iru = recip_rho<T, SU>(rhop) * T(1.0 / U);
  ux = jx * iru;
  uy = jy * iru;
  uz = jz * iru;
  k2[0] = m2[0] - jx * ux;
  k2[1] = m2[1] - jy * uy;
  k2[2] = m2[2] - jz * uz;
  k2[3] = m2[3] - jx * uy;
  k2[4] = m2[4] - jx * uz;
  k2[5] = m2[5] - jy * uz;
}

// Step 3 with bulk and higher rates 1 and no force, from the moments of
// second_order_central, then the inverse sweeps: the cube is overwritten
// with the post-collision deviations (times 2^inv_shift, and UNIT in storage
// units), as collide() leaves it.  ws, cs: the shear-group rates
// omega_4..omega_9 at this node and 1 - ws (ws[3], the bulk rate, is 1).
template <typename T, bool SU = false>
__host__ __device__ __forceinline__ void relax_unit_higher(T (&v)[3][3][3], const T (&cs)[6], T rhop, T rho, T ux,
                                                           T uy, T uz, const T (&k2)[6]) {
  constexpr double U = Units<SU>::U;
  const T third = T(1.0 / 3.0);
  const T thirdU = T(U / 3.0), ninthU = T(U / 9.0);
  const T ir = recip_rho<T, SU>(rhop);
  const T iru = ir * T(1.0 / U);
  // order 2: 2s1 on its attractor rho' (rate 1), the shear groups at their rates
  const T t110 = cs[0] * k2[3];
  const T t101 = cs[1] * k2[4];
  const T t011 = cs[2] * k2[5];
  const T t2d1 = cs[4] * (k2[0] - k2[1]);
  const T t2d2 = cs[5] * (k2[0] - k2[2]);
  const T t200 = third * (rhop + t2d1 + t2d2);
  const T t020 = third * (rhop - T(2) * t2d1 + t2d2);
  const T t002 = third * (rhop + t2d1 - T(2) * t2d2);
  // order 3 -> 0; order 4 -> attractors from post-collision order 2
  const T t220 = ((t200 + t020) * thirdU + t200 * t020 + T(2) * t110 * t110 - ninthU * rhop) * iru;
  const T t202 = ((t200 + t002) * thirdU + t200 * t002 + T(2) * t101 * t101 - ninthU * rhop) * iru;
  const T t022 = ((t020 + t002) * thirdU + t020 * t002 + T(2) * t011 * t011 - ninthU * rhop) * iru;
  const T A2 = thirdU + t200, B2 = thirdU + t020, C2 = thirdU + t002;
  const T t211 = (A2 * t011 + T(2) * t110 * t101) * iru;
  const T t121 = (B2 * t101 + T(2) * t110 * t011) * iru;
  const T t112 = (C2 * t110 + T(2) * t011 * t101) * iru;
  // order 5 -> its attractor, which vanishes with order 3 at 0 (every term
  // holds a third-order moment); order 6 -> attractor from orders 2 and 4
  const T t222 = ((t200 + t020 + t002) * ninthU + (t022 + t202 + t220) * thirdU + t200 * t022 + t020 * t202 +
                  t002 * t220 + T(4) * (t110 * t112 + t101 * t121 + t011 * t211)) *
                     (third * iru) -
                 rhop * (T(1.0 / 27.0) * ir);
  v[0][0][0] = rhop;
  v[0][0][1] = T(0); v[0][1][0] = T(0); v[1][0][0] = T(0);
  v[0][1][1] = t110; v[1][0][1] = t101; v[1][1][0] = t011;
  v[0][0][2] = t200; v[0][2][0] = t020; v[2][0][0] = t002;
  v[0][2][1] = T(0); v[2][0][1] = T(0); v[0][1][2] = T(0);
  v[2][1][0] = T(0); v[1][0][2] = T(0); v[1][2][0] = T(0);
  v[1][1][1] = T(0);
  v[0][2][2] = t220; v[2][0][2] = t202; v[2][2][0] = t022;
  v[1][1][2] = t211; v[1][2][1] = t121; v[2][1][1] = t112;
  v[2][2][1] = T(0); v[2][1][2] = T(0); v[1][2][2] = T(0);
  v[2][2][2] = t222;
  inverse_all<T, SU>(v, ux, uy, uz);
}

// Whole collision of one node (Appendix D Steps 7, 1-5): deviation cube in,
// post-collision deviations (times 2^inv_shift) out; in storage units (SU) the
// cube comes in as stored numbers and goes out times UNIT.  UH: rates of
// orders 3-6 equal to 1 (see relax).
template <typename T, bool FORCE, bool MAXWELL = false, bool SU = false, bool UH = false>
__host__ __device__ __forceinline__ void collide(T (&v)[3][3][3], const Rates<T>& R, const T (&ws)[6],
                                                 const T (&cs)[6], T Fx, T Fy, T Fz, T& rho, T& ux, T& uy,
                                                 T& uz) {
  T rhop;
  pre_collision<T, FORCE, SU>(v, Fx, Fy, Fz, rhop, rho, ux, uy, uz);
  relax<T, FORCE, MAXWELL, SU, UH>(v, R, ws, cs, Fx, Fy, Fz, rhop, rho, ux, uy, uz);
}

// Whole collision with bulk and higher rates 1 and no force (see
// relax_unit_higher); same contract as collide().
template <typename T, bool SU = false>
__host__ __device__ __forceinline__ void collide_unit_higher(T (&v)[3][3][3], const T (&cs)[6], T& rho, T& ux, T& uy,
                                                             T& uz) {
  T rhop, k2[6];
  second_order_central<T, SU>(v, rhop, rho, ux, uy, uz, k2);
  relax_unit_higher<T, SU>(v, cs, rhop, rho, ux, uy, uz, k2);
}

}  // namespace fpc
