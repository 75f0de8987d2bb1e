// d3q27.hpp -- compile-time description of the D3Q27 lattice used by the kernels.
//
// Velocity list in the order printed in Sec. 3.5 of the paper (alpha = 0..26) and
// the 27 central moments kappa_abc, a,b,c in {0,1,2}, in the order of the paper's
// moment vector.  Everything here is constexpr so that fully unrolled device loops
// fold every table lookup into register names.
#pragma once

namespace fpc {

constexpr int Q = 27;

constexpr int EX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
constexpr int EY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, 1, -1, -1, 1, 1, -1, -1};
constexpr int EZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1};

// alpha of the velocity (ex, ey, ez) -- inverse of the listing
constexpr int alpha_of(int ex, int ey, int ez) {
  for (int a = 0; a < Q; ++a)
    if (EX[a] == ex && EY[a] == ey && EZ[a] == ez) return a;
  return -1;
}
constexpr int opposite(int a) { return alpha_of(-EX[a], -EY[a], -EZ[a]); }
// the velocity mirrored in y (specular reflection at a y = const plane)
constexpr int mirror_y(int a) { return alpha_of(EX[a], -EY[a], EZ[a]); }

// Per-axis factors of the lattice weights: w_alpha = W1[ex+1] W1[ey+1] W1[ez+1]
// (1/6, 2/3, 1/6); with them w = 8/27, 2/27, 1/54, 1/216 by speed class.
// Per-axis factors of the rest-state central moments: kappa_abc = C1[a] C1[b] C1[c]
// with C1 = (1, 0, c_s^2), c_s^2 = 1/3.
constexpr double W1[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
constexpr double C1[3] = {1.0, 0.0, 1.0 / 3.0};

constexpr double weight(int a) { return W1[EX[a] + 1] * W1[EY[a] + 1] * W1[EZ[a] + 1]; }

// Exact power-of-two scale of the FP16/BF16 deviation storage, by speed class
// (|e|^2 = 0,1,2,3): 2^(DEV_LOG2_0 + 2 |e|^2), about 2^10 / w_alpha, so that
// relative deviations down to ~6e-8 stay in FP16's normal range and up to 64
// stay finite.  The factor 4 between classes is what the storage-unit sweeps
// of fpc_collide.hpp rely on.
constexpr int DEV_LOG2_0 = 12;
constexpr float dev_scale(int a) {
  return float(1u << (DEV_LOG2_0 + 2 * (EX[a] * EX[a] + EY[a] * EY[a] + EZ[a] * EZ[a])));
}
static_assert(dev_scale(0) == 4096.0f && dev_scale(1) == 16384.0f && dev_scale(7) == 65536.0f &&
                  dev_scale(19) == 262144.0f,
              "storage scales by speed class");

// Moment index in the paper's order:
// 000,100,010,001,110,101,011,200,020,002,120,102,210,012,201,021,111,220,202,022,
// 211,121,112,122,212,221,222
enum : int {
  K000, K100, K010, K001, K110, K101, K011, K200, K020, K002, K120, K102, K210, K012,
  K201, K021, K111, K220, K202, K022, K211, K121, K112, K122, K212, K221, K222
};

}  // namespace fpc
