// stream_collide.hpp -- the fused stream + collide kernel of the plain method
// (one time step: Appendix D Steps 6, 7, 1-5 in the library's order, see
// lbm.hip).  Kept in a header of its own so that what a measurement of this
// kernel depends on is exactly this file and the ones it includes.
#pragma once

#include "lattice.hpp"

// Block of up to 4 wavefronts; each wavefront is one 64-node x segment of one
// row (y, z uniform; wave_segment).  BC: 0 periodic, 1 walls across y (the
// channel), 2 walls on any faces, a moving lid, the symmetry plane and LES
// (StepArgs::box).  FORCE: a body force is applied.  MAXWELL: the comparison
// model's attractors.  COLL picks the form of the collision:
//   COLL_GENERAL: any rates;
//   COLL_SECOND_ONLY: the rates of the paper's runs (bulk and orders 3-6 equal
//     to 1) with no force and the Markovian attractors; the collision then
//     needs only the second-order moments (relax_unit_higher);
//   COLL_UNIT_HIGHER: orders 3-6 at rate 1 with the Markovian attractors, any
//     second-order rates, with or without a force (relax<..., UH = true>):
//     the paper's rates under a body force.
enum : int { COLL_GENERAL = 0, COLL_SECOND_ONLY = 1, COLL_UNIT_HIGHER = 2 };

template <int ST, int BC, bool FORCE, bool MAXWELL, int COLL = COLL_GENERAL>
__global__ __launch_bounds__(256) void k_stream_collide(const typename Stor<ST>::S* __restrict__ src,
                                                        typename Stor<ST>::S* __restrict__ dst,
                                                        StepArgs<typename Stor<ST>::R> A) {
  constexpr bool UNIT_HIGHER = COLL == COLL_SECOND_ONLY;
  static_assert(!UNIT_HIGHER || (!FORCE && !MAXWELL), "the unit-rate collision has no force and FPC attractors");
  static_assert(COLL != COLL_UNIT_HIGHER || !MAXWELL, "the unit-rate form takes the Markovian attractors");
  using T = typename Stor<ST>::R;
  // FP16/BF16: arithmetic on the stored numbers (storage units), which drops
  // the multiply of every loaded value by its scale.  Not in the periodic
  // FP16 kernel of the general collision: its single gather path lets the
  // compiler fold the scale into the conversions (v_fma_mix_f32) already, and
  // storage units measured a few instructions more there.
  constexpr bool SU =
      Stor<ST>::units && (UNIT_HIGHER || !(BC == 0 && (ST == LBM_F16DEV || ST == LBM_F16DEV_RNE)));
  int x, y, z;
  if (!wave_segment(A.g, x, y, z) || x >= A.g.nx) return;
  T v[3][3][3];
  if (BC == 2) pull_box<ST, SU>(src, A.g, A.box, x, y, z, v);
  else pull<ST, BC == 1, SU>(src, A.g, x, y, z, v);
  T ws[6] = {A.r.w[4], A.r.w[5], A.r.w[6], A.r.w[7], A.r.w[8], A.r.w[9]};
  T cs[6] = {A.r.c[4], A.r.c[5], A.r.c[6], A.r.c[7], A.r.c[8], A.r.c[9]};
  T rhop, rho, ux, uy, uz;
  if constexpr (UNIT_HIGHER) {
    T k2[6];
    second_order_central<T, SU>(v, rhop, rho, ux, uy, uz, k2);
    if (BC == 2 && A.box.les_on) les_rates<SU>(k2, rho, A.box, A.r, y, A.g.ny, ws, cs);  // uniform branch
    relax_unit_higher<T, SU>(v, cs, rhop, rho, ux, uy, uz, k2);
  } else {
    pre_collision<T, FORCE, SU>(v, A.F[0], A.F[1], A.F[2], rhop, rho, ux, uy, uz);
    if (BC == 2 && A.box.les_on) {  // uniform branch
      const T k2[6] = {v[0][0][2], v[0][2][0], v[2][0][0], v[0][1][1], v[1][0][1], v[1][1][0]};
      les_rates<SU>(k2, rho, A.box, A.r, y, A.g.ny, ws, cs);
    }
    relax<T, FORCE, MAXWELL, SU, COLL == COLL_UNIT_HIGHER>(v, A.r, ws, cs, A.F[0], A.F[1], A.F[2], rhop, rho, ux, uy,
                                                          uz);
  }
  push<ST, SU>(dst, A.g, x, y, z, v, A.step);
}
