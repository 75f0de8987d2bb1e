// lattice.hpp -- device-side pieces of the step kernels: storage forms, the
// blocked layout of the state in HBM, the pull gather with its boundaries,
// the store, and the launch mapping of wavefronts to row segments.  Not part
// of the public interface (include/lbm.h).
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
  static constexpr bool units = false;  // stores plain deviations
  static __device__ __forceinline__ R dec(S s, int) { return s; }
  static __device__ __forceinline__ R raw(S s) { return s; }
  // f: exact power of two still carried by r (see inverse_all)
  static constexpr bool stochastic = false;
  static __device__ __forceinline__ S enc(R r, int, double f = 1.0, uint32_t = 0) { return r * f; }
  static __device__ __forceinline__ S enc_nearest(R r, int a, double f = 1.0) { return enc(r, a, f); }
};

template <>
struct Stor<LBM_F32> {
  using S = float;
  using R = float;
  static constexpr bool units = false;
  static __device__ __forceinline__ R dec(S s, int) { return s; }
  static __device__ __forceinline__ R raw(S s) { return s; }
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
  // the kernels' arithmetic runs in storage units (fpc_collide.hpp): raw()
  // is the stored number, dec() the deviation
  static constexpr bool units = true;
  static __device__ __forceinline__ R raw(S s) { return (float)s; }
  static __device__ __forceinline__ R dec(S s, int a) { return (float)s * (1.0f / dev_scale(a)); }
  static __device__ __forceinline__ S enc(R r, int a, double f = 1.0, uint32_t rnd = 0) {
    const float x = r * (float)(dev_scale(a) * f);
    if (SR) {
      // the conversion writes the low half and keeps the high one, which is
      // never stored: seed it with x's own bits (x is dead afterwards), so
      // no register has to be cleared first
      f16x2_t h = __builtin_bit_cast(f16x2_t, x);
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
  static constexpr bool units = true;
  static __device__ __forceinline__ R raw(S s) { return __uint_as_float((uint32_t)s << 16); }
  static __device__ __forceinline__ R dec(S s, int a) {
    return __uint_as_float((uint32_t)s << 16) * (1.0f / dev_scale(a));
  }
  static __device__ __forceinline__ S enc(R r, int a, double f = 1.0, uint32_t rnd = 0) {
    const float x = r * (float)(dev_scale(a) * f);
    if (SR) {
      bf16x2_t h = __builtin_bit_cast(bf16x2_t, x);  // high half never stored (see StorF16)
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

// Layout of a state buffer in HBM (every storage form): x is cut into
// segments of SEG = 64 nodes (one wavefront); for every (y, z) row the
// nxp = ceil(nx / 64) * 64 padded nodes form nxp / 64 segments, and a segment
// holds its 27 directions one after the other, 64 consecutive x values each:
//   index(a, x, y, z) = (z ny + y) 27 nxp + 27 * 64 floor(x / 64) + 64 slot(a) + (x mod 64).
// A wavefront that updates one segment reads and writes a few contiguous
// 27 x 64-value blocks (its own row and the y/z neighbour rows) instead of 54
// separate direction arrays.  Measured on the 256x128x128 channel against 27
// direction arrays: FP32 +11 %, FP64 +5 %, BF16 +7 %, FP16 +2 %.
constexpr int SEG = 64;

// Division of numerators below 2^31 by an invariant d >= 1 as a multiply and
// a shift (Granlund and Montgomery, 1994): with l = ceil(log2 d) and
// m = ceil(2^(31+l) / d) < 2^32, floor(n / d) = (n m) >> (31 + l).
struct Div31 {
  uint32_t m;
  uint32_t shift;  // 31 + l
  __host__ __device__ __forceinline__ uint32_t div(uint32_t n) const {
    return (uint32_t)(((uint64_t)n * m) >> shift);
  }
};
inline Div31 make_div31(uint32_t d) {
  uint32_t l = 0;
  while (((uint64_t)1 << l) < d) ++l;
  const uint64_t p = (uint64_t)1 << (31 + l);
  return Div31{(uint32_t)((p + d - 1) / d), 31 + l};
}

struct Geom {
  int nx, ny, nz;
  int nxs;         // x segments per row, ceil(nx / SEG)
  int nxp;         // nx rounded up to a multiple of SEG
  int64_t rowlen;  // values per (y, z) row: 27 nxp
  Div31 by_nxs, by_ny;  // wavefront -> (segment, row) of the step kernels
  int flat;             // 1: flat grid over all row segments; 0: blocks inside one row
  Div31 by_bpr;         // blocks per row (grid of blocks inside one row)
  uint32_t blk_per_xcd; // XCD-aware block order: blocks / 8, or 0 for the plain order
};

// Position of direction a's block inside a segment: the directions are kept
// in the order of their velocity cube, slot = 9 (e_z + 1) + 3 (e_y + 1) + (e_x + 1),
// so the three directions a wavefront pulls from one source row (equal e_y,
// e_z) lie next to each other.
__host__ __device__ constexpr int slot(int a) { return 9 * (EZ[a] + 1) + 3 * (EY[a] + 1) + (EX[a] + 1); }

// position of x inside a row, in values
__host__ __device__ __forceinline__ uint32_t x_part(int x) {
  const uint32_t u = (uint32_t)x;
  return (u / SEG) * (Q * SEG) + u % SEG;
}

__host__ __device__ __forceinline__ int64_t pop_index(const Geom& g, int a, int x, int y, int z) {
  return ((int64_t)z * g.ny + y) * g.rowlen + slot(a) * SEG + x_part(x);
}

// (x, y, z) of the linear node index i = x + nx (y + ny z)
__host__ __device__ __forceinline__ void node_xyz(const Geom& g, int64_t i, int& x, int& y, int& z) {
  const int ii = (int)i;  // N < 2^31
  x = ii % g.nx;
  const int r = ii / g.nx;
  y = r % g.ny;
  z = r / g.ny;
}

// walls on any face and a moving lid (the general boundary kernel)
template <typename T>
struct Box {
  int wx, wy, wz;  // halfway bounce-back walls across x / y / z
  int lid_on;      // the wall above y = ny - 1 moves with lid[]
  T lid6[3];       // 6 U = 2 U / c_s^2 (momentum correction per unit weight)
  int sym;         // the face above y = ny - 1 is a specular symmetry plane
  int les_on;      // Smagorinsky LES with van Driest damping
  T les_c;         // Smagorinsky constant C
  T les_s;         // u_tau / nu (0: no damping)
  T les_ia;        // 1 / A+
};

template <typename T>
struct StepArgs {
  Geom g;
  Rates<T> r;
  T F[3];
  uint32_t step;  // completed steps before this one (random words of SR storage)
  Box<T> box;
};

// ===========================================================================
// streaming (Appendix D Step 6), pull form, shared by every kernel that reads a
// time level: f_alpha(x) = f~_alpha(x - e_alpha), periodic wrap, and halfway
// bounce-back across the y walls (the node's own opposite population).
//
// The caller's wavefront covers one x segment of one row: y and z are uniform
// across it, so every row and direction base is a scalar 64-bit address and
// the only per-lane address terms are the three x offsets inside a row
// (32-bit; checked at creation).  Lanes with x >= nx must not call.
// SU: leave the stored numbers in v (storage units, fpc_collide.hpp) instead
// of the deviations.
template <int ST, bool WALLS, bool SU = false>
__device__ __forceinline__ void pull(const typename Stor<ST>::S* __restrict__ src, const Geom& g, int x, int y, int z,
                                     typename Stor<ST>::R (&v)[3][3][3]) {
  using T = typename Stor<ST>::R;
  using S = typename Stor<ST>::S;
  using SS = Stor<ST>;
  constexpr uint32_t SZ = sizeof(S);
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  // rows away from the walls (all but two per plane) take the wall-free gather,
  // whose loads keep the scalar-base form; the branch is wavefront-uniform
  if (WALLS && y > 0 && y < ny - 1) return pull<ST, false, SU>(src, g, x, y, z, v);
  const char* __restrict__ sb = (const char*)src;
  const int64_t rowb = g.rowlen * SZ;
  const int64_t planeb = rowb * ny;
  constexpr uint64_t dirb = SEG * SZ;  // one direction block of a segment
  // per-lane byte offsets inside a row of the source x for e_x = -1, 0, +1
  const uint32_t xo[3] = {x_part(x == nx - 1 ? 0 : x + 1) * SZ, x_part(x) * SZ, x_part(x == 0 ? nx - 1 : x - 1) * SZ};
  // uniform byte offsets: this row, and the steps to the source rows for
  // e_y, e_z = -1, 0, +1 (periodic wrap), additions only
  const int64_t r0 = ((int64_t)z * ny + y) * rowb;
  const int64_t dy[3] = {y == ny - 1 ? rowb - planeb : rowb, 0, y == 0 ? planeb - rowb : -rowb};
  const int64_t span = planeb * nz;
  const int64_t dz[3] = {z == nz - 1 ? planeb - span : planeb, 0, z == 0 ? span - planeb : -planeb};
  const char* dptr = sb + r0;  // this row of the direction in slot s
  // slot order: the three loads from one source row are issued together
#pragma unroll
  for (int s = 0; s < Q; ++s) {
    const int ex = s % 3 - 1, ey = (s / 3) % 3 - 1, ez = s / 9 - 1;
    const int a = alpha_of(ex, ey, ez);
    // halfway bounce-back: if x - e_alpha is a wall node, take the node's own
    // opposite population (same weight, so the deviation carries over)
    const bool bb = WALLS && ((ey == 1 && y == 0) || (ey == -1 && y == ny - 1));
    const int o = opposite(a);
    // bb is uniform: the base is chosen in scalar registers
    const char* base = bb ? sb + r0 + (uint64_t)slot(o) * dirb : dptr + (dy[ey + 1] + dz[ez + 1]);
    const uint32_t off = bb ? xo[1] : xo[ex + 1];
    dptr += dirb;
    // w_opp = w_alpha and the storage scales are equal
    const S sv = *(const S*)(base + off);
    v[ez + 1][ey + 1][ex + 1] = SU ? SS::raw(sv) : SS::dec(sv, a);
  }
}

// Gather with walls on any set of faces and an optional moving lid above
// y = ny - 1 (the cavity of Sec. 4).  A link whose source lies outside a
// walled face takes the node's own opposite population (halfway
// bounce-back); a link through the lid adds the moving-wall correction
// 2 w_a rho_w (e_a . U) / c_s^2 with rho_w = 1.  y and z walls are
// wavefront-uniform; x walls touch only the first and last lane of a row, so
// those lanes reload their own opposite population.  Wavefronts away from
// every wall take the wall-free gather.
template <int ST, bool SU = false>
__device__ __forceinline__ void pull_box(const typename Stor<ST>::S* __restrict__ src, const Geom& g,
                                         const Box<typename Stor<ST>::R>& b, int x, int y, int z,
                                         typename Stor<ST>::R (&v)[3][3][3]) {
  using T = typename Stor<ST>::R;
  using S = typename Stor<ST>::S;
  using SS = Stor<ST>;
  auto get = [](S sv, int a) -> T { return SU ? SS::raw(sv) : SS::dec(sv, a); };
  constexpr uint32_t SZ = sizeof(S);
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int x0 = __builtin_amdgcn_readfirstlane(x - (x % SEG));  // first x of the segment
  const bool yin = !b.wy || (y > 0 && y < ny - 1);
  const bool zin = !b.wz || (z > 0 && z < nz - 1);
  const bool xin = !b.wx || (x0 > 0 && x0 + SEG < nx);
  if (yin && zin && xin) return pull<ST, false, SU>(src, g, x, y, z, v);
  const char* __restrict__ sb = (const char*)src;
  const int64_t rowb = g.rowlen * SZ;
  const int64_t planeb = rowb * ny;
  constexpr uint64_t dirb = SEG * SZ;
  const uint32_t xo[3] = {x_part(x == nx - 1 ? 0 : x + 1) * SZ, x_part(x) * SZ, x_part(x == 0 ? nx - 1 : x - 1) * SZ};
  const int64_t r0 = ((int64_t)z * ny + y) * rowb;
  const int64_t dy[3] = {y == ny - 1 ? rowb - planeb : rowb, 0, y == 0 ? planeb - rowb : -rowb};
  const int64_t span = planeb * nz;
  const int64_t dz[3] = {z == nz - 1 ? planeb - span : planeb, 0, z == 0 ? span - planeb : -planeb};
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const int ex = EX[a], ey = EY[a], ez = EZ[a];
    const int o = opposite(a);
    const bool top = ey == -1 && y == ny - 1;
    const bool bby = b.wy && ((ey == 1 && y == 0) || (top && !b.sym));
    const bool bbz = b.wz && ((ez == 1 && z == 0) || (ez == -1 && z == nz - 1));
    const bool xwall = b.wx && ex != 0 && ((ex == 1 && x == 0) || (ex == -1 && x == nx - 1));  // per lane
    T val;
    if (b.sym && top && !bbz) {  // uniform: specular reflection at the symmetry plane
      // the population that left (x - e_x, ny - 1, z - e_z) with (e_x, +1, e_z)
      val = get(*(const S*)(sb + r0 + (uint64_t)slot(mirror_y(a)) * dirb + dz[ez + 1] + xo[ex + 1]), a);
      if (xwall) val = get(*(const S*)(sb + r0 + (uint64_t)slot(o) * dirb + xo[1]), a);
    } else if (bby || bbz) {  // uniform
      val = get(*(const S*)(sb + r0 + (uint64_t)slot(o) * dirb + xo[1]), a);
      // the correction in the units of val
      if (b.lid_on && b.wy && top)
        val += T(weight(a) * (SU ? dev_scale(a) : 1.0f)) * (ex * b.lid6[0] + ey * b.lid6[1] + ez * b.lid6[2]);
    } else {
      val = get(*(const S*)(sb + r0 + (uint64_t)slot(a) * dirb + (dy[ey + 1] + dz[ez + 1]) + xo[ex + 1]), a);
      if (xwall) val = get(*(const S*)(sb + r0 + (uint64_t)slot(o) * dirb + xo[1]), a);
    }
    v[ez + 1][ey + 1][ex + 1] = val;
  }
}

// Smagorinsky LES with van Driest damping (the Sec. 4 channel): the shear
// rates omega_4,5,6,8,9 of this node from its deviatoric pre-collision stress
// Pi (the primed second-order central moments; the rest state has no
// deviatoric part).  |S| = sqrt(2 S:S) with S = -Pi / (2 rho c_s^2 tau), so the
// relaxation time tau = tau_0 + 3 nu_t, nu_t = (C D)^2 |S|, is the positive root
// of tau^2 - tau_0 tau - 9 sqrt(2) (C D)^2 |Pi| / (2 rho) = 0.  D uses the
// distance to the nearest y wall half a link outside (uniform per wavefront).
// SU: v carries the factor UNIT of the storage units.
// k2: the node's second-order central moments (kappa'_200, kappa'_020,
// kappa'_002, kappa_110, kappa_101, kappa_011).
template <bool SU = false, typename T>
__device__ __forceinline__ void les_rates(const T (&k2)[6], T rho, const Box<T>& b, const Rates<T>& R, int y,
                                          int ny, T (&ws)[6], T (&cs)[6]) {
  const T k200 = k2[0], k020 = k2[1], k002 = k2[2];
  const T k110 = k2[3], k101 = k2[4], k011 = k2[5];
  const T tr = (k200 + k020 + k002) * T(1.0 / 3.0);
  const T dxx = k200 - tr, dyy = k020 - tr, dzz = k002 - tr;
  const T q = sqrt(dxx * dxx + dyy * dyy + dzz * dzz + T(2) * (k110 * k110 + k101 * k101 + k011 * k011));
  T yw = T(y) + T(0.5);
  if (!b.sym && T(ny) - T(0.5) - T(y) < yw) yw = T(ny) - T(0.5) - T(y);
  const T d = b.les_s > T(0) ? T(1) - exp(-yw * b.les_s * b.les_ia) : T(1);
  const T cd = b.les_c * d;
  const T tau0 = recip(R.w[4]);
  const T tau = T(0.5) * (tau0 + sqrt(tau0 * tau0 + T(18.0 * 1.4142135623730951 / Units<SU>::U) * cd * cd * q * recip(rho)));
  const T w = recip(tau);
  ws[0] = ws[1] = ws[2] = ws[4] = ws[5] = w;
  cs[0] = cs[1] = cs[2] = cs[4] = cs[5] = T(1) - w;
}

// store the post-collision cube (deviations times 2^inv_shift, and times
// UNIT in storage units) of node (x, y, z); same wavefront contract as
// pull().  The row base walks the 27 direction blocks of the segment in scalar
// registers; the per-lane part is the x offset only.
template <int ST, bool SU = false>
__device__ __forceinline__ void push(typename Stor<ST>::S* __restrict__ dst, const Geom& g, int x, int y, int z,
                                     const typename Stor<ST>::R (&v)[3][3][3], uint32_t step) {
  using S = typename Stor<ST>::S;
  constexpr uint32_t SZ = sizeof(S);
  constexpr uint64_t dirb = SEG * SZ;
  // random word input: the node's linear index
  const uint32_t node = ((uint32_t)z * (uint32_t)g.ny + (uint32_t)y) * (uint32_t)g.nx + (uint32_t)x;
  const uint32_t h = Stor<ST>::stochastic ? node_hash(node, step) : 0u;
  const uint32_t off = x_part(x) * SZ;
  char* base = (char*)dst + ((uint64_t)z * g.ny + y) * ((uint64_t)g.rowlen * SZ);
#pragma unroll
  for (int s = 0; s < Q; ++s) {  // slot order: one contiguous run of direction blocks
    const int a = alpha_of(s % 3 - 1, (s / 3) % 3 - 1, s / 9 - 1);
    // streaming store: the next step reads it back from HBM, not from cache
    __builtin_nontemporal_store(Stor<ST>::enc(v[s / 9][(s / 3) % 3][s % 3], a, inv_factor(a) / Units<SU>::U,
                                              h + (uint32_t)a * 0x9E3779B9u),
                                (S*)(base + off));
    base += dirb;
  }
}

// wavefront -> (x segment, row) for the step kernels; each wavefront keeps
// one segment of one row (y, z uniform, as pull() needs), and every block is
// full.  Rows that split into whole blocks (nxs <= 4 or a multiple of 4) use
// blocks of W = min(4, nxs) segments inside one row, B = nxs / W per row.
// Other rows (g.flat) take blocks of four consecutive row segments in
// row-major order, spanning rows.  false: a wavefront past the end of the
// flat grid.
//
// XCD-aware order.  The hardware hands consecutive blocks to the eight XCDs
// in turn, and each XCD has its own L2.  With g.blk_per_xcd > 0, block b runs
// logical block (b mod 8) P + b / 8 (P = blocks / 8; the last blocks / 8
// remainder keep b): XCD k takes the contiguous logical blocks
// [k P, (k + 1) P) in order, so each XCD streams through its own eighth of
// the lattice.  Two neighbouring segments of a row share the cache lines at
// their seam (a shifted load of the x-moving directions reads the neighbour's
// first or last value); in the plain order, with two blocks per row
// (nx = 512), the halves of a row sit on different XCDs and those lines are
// fetched by both L2s (measured: 4 % (FP32), 2 % (FP64) and 8 % (16-bit
// forms) more reads than the algorithmic bytes; with chunks, 0.3 %, 1.2 % and
// 0 %).  Time per step on the 512^3 vortex, chunks against the plain order
// (same box, interleaved runs; the spread between runs is about 2 %): FP64
// +4 %, FP32 +2 %, FP16/BF16 -1 % (their second fetch is served by the
// last-level cache); at 384^3 FP64 +3 %, FP32 -2 %, FP16 -3 %; at 256^3 (one
// block per row, no seam between blocks) FP32 -4 %.  Dealing whole rows to
// the XCDs in turns (runs of one row), and blocks of a whole row of up to 8
// segments, also removed the second fetch but were no faster than the plain
// order.  So the 4- and 8-byte forms take chunks where a row is split across
// blocks (more than four segments), the 16-bit forms keep the plain order.
constexpr int SEGS_PER_BLOCK = 4;
constexpr uint32_t XCDS = 8;
__host__ __device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t per) {
  return b < per * XCDS ? (b % XCDS) * per + b / XCDS : b;
}
// The mapping for block (bx, by, bz) of a grid (gx, gy, .) of blocks of
// blockdim threads, wavefront w and lane of it (host-callable for tests).
__host__ __device__ __forceinline__ bool segment_of(const Geom& g, uint32_t bx, uint32_t by, uint32_t bz, uint32_t gx,
                                                    uint32_t gy, uint32_t blockdim, uint32_t w, uint32_t lane, int& x,
                                                    int& y, int& z) {
  if (!g.flat) {  // grid (B, ny, nz), blocks of W = min(4, nxs) segments
    const uint32_t l = xcd_block(bx + gx * (by + gy * bz), g.blk_per_xcd);
    const uint32_t row = g.by_bpr.div(l);
    const uint32_t zz = g.by_ny.div(row);
    y = (int)(row - zz * (uint32_t)g.ny);
    z = (int)zz;
    x = (int)((l - row * gx) * blockdim + w * SEG + lane);
    return true;
  }
  const uint32_t s = xcd_block(bx, g.blk_per_xcd) * (uint32_t)SEGS_PER_BLOCK + w;  // below 2^31
  const uint32_t row = g.by_nxs.div(s);
  if (row >= (uint32_t)g.ny * (uint32_t)g.nz) return false;
  const uint32_t zz = g.by_ny.div(row);
  y = (int)(row - zz * (uint32_t)g.ny);
  z = (int)zz;
  x = (int)(s - row * (uint32_t)g.nxs) * SEG + (int)lane;
  return true;
}
__device__ __forceinline__ bool wave_segment(const Geom& g, int& x, int& y, int& z) {
  const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  return segment_of(g, blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x, gridDim.y, blockDim.x, w, threadIdx.x & 63, x, y,
                    z);
}
// Launch shape of the step kernels: 1D blocks of up to 4 wavefronts, each
// one 64-node x segment of one row (wave_segment); for nx = 256 a block is one
// row.
// Every block full either way: one block row per (y, z) when the row splits
// into whole blocks (nxs <= 4 or a multiple of 4), else the flat grid.
inline bool flat_grid(int nx, int ny, int nz) {
  const int nxs = (nx + SEG - 1) / SEG;
  return !(nxs <= SEGS_PER_BLOCK || nxs % SEGS_PER_BLOCK == 0) || ny > 65535 || nz > 65535;
}

inline void step_launch_shape(int nx, int ny, int nz, dim3& block, dim3& grid) {
  const int nxs = (nx + SEG - 1) / SEG;
  if (flat_grid(nx, ny, nz)) {
    const int64_t nseg = (int64_t)nxs * ny * nz;  // below 2^31 (lbm_create)
    block = dim3(SEG * SEGS_PER_BLOCK, 1, 1);
    grid = dim3((unsigned)((nseg + SEGS_PER_BLOCK - 1) / SEGS_PER_BLOCK), 1, 1);
  } else {
    const int w = nxs < SEGS_PER_BLOCK ? nxs : SEGS_PER_BLOCK;
    block = dim3(SEG * w, 1, 1);
    grid = dim3((nxs + w - 1) / w, ny, nz);
  }
}

// bytes per stored value of a storage form (0: unknown form)
inline size_t elem_size(int st) {
  switch (st) {
    case LBM_F64: return 8;
    case LBM_F32: return 4;
    case LBM_F16DEV:
    case LBM_BF16DEV:
    case LBM_F16DEV_RNE:
    case LBM_BF16DEV_RNE: return 2;
    default: return 0;
  }
}

// storage layout of a configuration (see the layout notes above)
inline Geom make_geom(const lbm_config* cfg) {
  Geom g{};
  g.nx = cfg->nx;
  g.ny = cfg->ny;
  g.nz = cfg->nz;
  g.nxs = (cfg->nx + SEG - 1) / SEG;
  g.nxp = g.nxs * SEG;
  // Rows whose byte length is a multiple of 1 KiB get 64 values of padding
  // (measured, same box: the 512^3 vortex +2.5 % (FP16/BF16) and +0.7 % (FP32),
  // FP64 unchanged; where the padding was tried on other rows, 256^3 and 384^3
  // in FP16, it cost 0.5-1.7 %, and those rows are not padded).
  const int64_t row = (int64_t)LBM_Q * g.nxp;
  g.rowlen = row + ((row * (int64_t)elem_size(cfg->storage)) % 1024 == 0 ? SEG : 0);
  g.by_nxs = make_div31((uint32_t)g.nxs);
  g.by_ny = make_div31((uint32_t)g.ny);
  g.flat = flat_grid(g.nx, g.ny, g.nz) ? 1 : 0;
  dim3 block, grid;
  step_launch_shape(g.nx, g.ny, g.nz, block, grid);
  g.by_bpr = make_div31(grid.x);
  const bool chunks = elem_size(cfg->storage) >= 4 && g.nxs > SEGS_PER_BLOCK;  // rows split across blocks
  g.blk_per_xcd = chunks ? (uint32_t)(((uint64_t)grid.x * grid.y * grid.z) / XCDS) : 0u;
  return g;
}

