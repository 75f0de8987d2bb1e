/*
 * fpc_oracle.c -- plain, slow FP64 CPU oracle of the D3Q27 FPC-LBM time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file: only tests/, the smoke check and the cpu_baseline leg of the
 * benchmark use it.  It shares no code, header, table or constant with the HIP
 * library; every table below is rebuilt here from the paper's printed lists.
 *
 * Source: Schupbach & Premnath, "Fokker-Planck Central Moment Lattice Boltzmann
 * Method for Effective Simulations of Fluid Dynamics" (arXiv 2410.09739).
 *   - velocity set e_alpha:             Sec. 3.5 (construction of the 3D FPC-LBM)
 *   - moment ordering and matrix P:     Sec. 3.5, with Eq. (map-df-rm)
 *   - frame shift F(u), F^-1:           Sec. 3.5, Eq. (rmcm) (binomial expansion)
 *   - Markovian attractor (general):    Eq. (Mvcmattractor3D)
 *   - diffusion tensor choice:          Eq. (diffusion-tensor-parameter-3D)
 *   - body-force sources sigma_mnp:     Eq. (cmupdatesourceD3Q27)
 *   - per-node algorithm Steps 1..7:    Appendix D
 *   - collide/stream form:              Eqs. (LBMsteps-collide), (LBMsteps-stream)
 *
 * Everything is done the obvious way: P is the 27x27 integer matrix of monomials,
 * P^-1 is obtained by Gauss-Jordan elimination, F(u) is filled entry by entry from
 * the binomial theorem, and the collision follows Appendix D Step 3 in the
 * paper's order and notation.  No blocking, fusion or factorisation.
 *
 * Readings where the paper is garbled or silent (the tests and the Python side
 * cite them by these labels):
 *   R2  the equilibrium (initial state, not defined in the paper) is the set of
 *       populations whose central moments are the attractors at rest in the
 *       moving frame, kappa_abc = rho c_a c_b c_c with c = (1, 0, c_s^2): the
 *       discrete Maxwellian, equal to the product form rho prod_d phi(e_d, u_d).
 *   R3  kappa^Mv_122 is evaluated from the general attractor formula, which
 *       yields the product kappa~_110 kappa~_012 (the printed closed form shows
 *       kappa~_011 kappa~_012 there; the continuous form in Sec. 3.4 agrees with
 *       the general formula).
 *   R6  P^-1 is the exact inverse of P; the printed Step 5 row of f~_4
 *       (e_4 = (0, -1, 0)) carries +kappa~'_010 where the exact inverse has
 *       -kappa~'_010 (all other printed rows agree with it).
 *   R7  the third-order decomposition assigns (3s3 - 3m3)/2 to kappa~_021.
 *   R8  sources use the pre-collision central moments with kappa_000 = rho and
 *       the first-order central moments taken as zero (as the 2D source list in
 *       Sec. 2.6 evaluates them).
 *   R10 attractors of order >= 3 use the current (post-collision) lower moments,
 *       the diffusion tensor D'_ij = kappa~_ij / rho, first-order moments = 0.
 *   R11 third-order attractors are zero, as printed.
 *   R12 halfway bounce-back (pull form): if the upstream node x - e_alpha is a
 *       wall node, f_alpha(x, t+1) = f~_opp(alpha)(x, t).
 *   R23 walls: bit 0 of `walls` = halfway bounce-back walls half a link outside
 *       y = 0 and y = ny-1 (R12), bit 1 the same across x, bit 2 across z (the
 *       cubic cavity of Sec. 4 uses all six).  A moving wall above y = ny-1
 *       (velocity `lid`, Sec. 4 lid-driven cavity) adds the momentum
 *       correction 2 w_a rho_w (e_a . U) / c_s^2 with rho_w = 1 to every link
 *       that crosses it, corner and edge links included.
 *   R24 bit 3 of `walls` turns the face above y = ny-1 into the specular
 *       (mirror) symmetry plane of the Sec. 4 half channel: a link crossing it
 *       takes the population that left the tangentially shifted node
 *       (x - e_x, ny-1, z - e_z) with the mirrored velocity (e_x, -e_y, e_z).
 *   R25 the LES of the Sec. 4 half channel (Smagorinsky with van Driest
 *       damping): per node nu_t = (C D)^2 |S|, D = 1 - exp(-y+ / 26), y+ the
 *       distance to the nearest wall in wall units; |S| = sqrt(2 S_ij S_ij)
 *       from the deviatoric non-equilibrium second-order central moments
 *       before collision, S = -omega Pi_dev / (2 rho c_s^2), so
 *       |S| = 3 sqrt(2) Q / (2 rho tau) with Q = |Pi_dev| (Frobenius); the
 *       relaxation time tau = 1/omega of the shear groups (omega_4,5,6,8,9) is
 *       the positive root of tau^2 - tau_0 tau - 9 sqrt(2) (C D)^2 Q / (2 rho);
 *       bulk and higher rates are unchanged.
 *   R22 the comparison model with Maxwellian equilibria (MCM-LBM, Sec. 4, the
 *       doubly periodic shear layer and crossing shear wave studies) relaxes
 *       every non-conserved central moment to the discrete Maxwellian's,
 *       rho c_a c_b c_c with c = (1, 0, c_s^2), with the same rates, grouping
 *       and sources as FPC; only the attractors of order >= 4 differ.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 27

/* Velocity components exactly as listed in Sec. 3.5 (alpha = 0..26). */
static const int EX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
static const int EY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, 1, -1, -1, 1, 1, -1, -1};
static const int EZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1};

/* Exponents (m,n,p) of the 27 moments in the order of the moment vectors of
 * Sec. 3.5: 000,100,010,001,110,101,011,200,020,002,120,102,210,012,201,021,
 * 111,220,202,022,211,121,112,122,212,221,222. */
static const int MNP[Q][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1},
    {2, 0, 0}, {0, 2, 0}, {0, 0, 2}, {1, 2, 0}, {1, 0, 2}, {2, 1, 0}, {0, 1, 2},
    {2, 0, 1}, {0, 2, 1}, {1, 1, 1}, {2, 2, 0}, {2, 0, 2}, {0, 2, 2}, {2, 1, 1},
    {1, 2, 1}, {1, 1, 2}, {1, 2, 2}, {2, 1, 2}, {2, 2, 1}, {2, 2, 2}};

enum {
  K000, K100, K010, K001, K110, K101, K011, K200, K020, K002, K120, K102, K210, K012,
  K201, K021, K111, K220, K202, K022, K211, K121, K112, K122, K212, K221, K222
};

static const double CS2 = 1.0 / 3.0; /* c_s^2 = 1/3 (Sec. 4) */

static double P[Q][Q];    /* m = P f                 */
static double PINV[Q][Q]; /* f = P^-1 m              */
static int IDX[3][3][3];  /* (m,n,p) -> moment index */
static int OPP[Q];        /* e_opp = -e_alpha        */
static int ready = 0;

static int ipow(int b, int e) {
  int r = 1;
  while (e-- > 0) r *= b;
  return r;
}

static double dpow(double b, int e) {
  double r = 1.0;
  while (e-- > 0) r *= b;
  return r;
}

static double binom(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

/* Gauss-Jordan inversion with partial pivoting; returns 0 on success. */
static int invert(int n, const double* a, double* inv) {
  double* w = (double*)malloc(sizeof(double) * n * 2 * n);
  if (!w) return -1;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < 2 * n; ++j)
      w[i * 2 * n + j] = j < n ? a[i * n + j] : (j - n == i ? 1.0 : 0.0);
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (fabs(w[r * 2 * n + c]) > fabs(w[piv * 2 * n + c])) piv = r;
    if (fabs(w[piv * 2 * n + c]) < 1e-12) { free(w); return -2; }
    if (piv != c)
      for (int j = 0; j < 2 * n; ++j) {
        double t = w[c * 2 * n + j];
        w[c * 2 * n + j] = w[piv * 2 * n + j];
        w[piv * 2 * n + j] = t;
      }
    double d = w[c * 2 * n + c];
    for (int j = 0; j < 2 * n; ++j) w[c * 2 * n + j] /= d;
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double s = w[r * 2 * n + c];
      if (s != 0.0)
        for (int j = 0; j < 2 * n; ++j) w[r * 2 * n + j] -= s * w[c * 2 * n + j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) inv[i * n + j] = w[i * 2 * n + n + j];
  free(w);
  return 0;
}

static void setup(void) {
  if (ready) return;
  /* P: rows are the monomials e_x^m e_y^n e_z^p over the 27 velocities. */
  for (int k = 0; k < Q; ++k)
    for (int a = 0; a < Q; ++a)
      P[k][a] = (double)(ipow(EX[a], MNP[k][0]) * ipow(EY[a], MNP[k][1]) * ipow(EZ[a], MNP[k][2]));
  invert(Q, &P[0][0], &PINV[0][0]);
  for (int k = 0; k < Q; ++k) IDX[MNP[k][0]][MNP[k][1]][MNP[k][2]] = k;
  for (int a = 0; a < Q; ++a)
    for (int b = 0; b < Q; ++b)
      if (EX[b] == -EX[a] && EY[b] == -EY[a] && EZ[b] == -EZ[a]) OPP[a] = b;
  ready = 1;
}

/* Frame-shift matrix of Eq. (rmcm): kappa = F(u) m, from the binomial expansion
 * of (e_x - u_x)^m (e_y - u_y)^n (e_z - u_z)^p.  F^-1(u) = F(-u). */
static void frame_matrix(const double u[3], double F[Q][Q]) {
  for (int k = 0; k < Q; ++k) {
    const int m = MNP[k][0], n = MNP[k][1], p = MNP[k][2];
    for (int j = 0; j < Q; ++j) {
      const int i0 = MNP[j][0], j0 = MNP[j][1], k0 = MNP[j][2];
      if (i0 > m || j0 > n || k0 > p) { F[k][j] = 0.0; continue; }
      F[k][j] = binom(m, i0) * binom(n, j0) * binom(p, k0) * dpow(-u[0], m - i0) *
                dpow(-u[1], n - j0) * dpow(-u[2], p - k0);
    }
  }
}

static void matvec(double A[Q][Q], const double* x, double* y) {
  for (int i = 0; i < Q; ++i) {
    double s = 0.0;
    for (int j = 0; j < Q; ++j) s += A[i][j] * x[j];
    y[i] = s;
  }
}

/* Eq. (Mvcmattractor3D): attractor of moment (m,n,p) given the diffusion tensor
 * D' = (D'_200, D'_020, D'_002, D'_110, D'_011, D'_101) and the current central
 * moments pi[] (first-order entries must already be zero, reading R10). */
static double mv_attractor(int m, int n, int p, const double D[6], const double* pi) {
  const double s = (double)(m + n + p);
  double r = 0.0;
  if (m >= 2) r += D[0] * m * (m - 1) / s * pi[IDX[m - 2][n][p]];
  if (n >= 2) r += D[1] * n * (n - 1) / s * pi[IDX[m][n - 2][p]];
  if (p >= 2) r += D[2] * p * (p - 1) / s * pi[IDX[m][n][p - 2]];
  if (m >= 1 && n >= 1) r += 2.0 * D[3] * m * n / s * pi[IDX[m - 1][n - 1][p]];
  if (n >= 1 && p >= 1) r += 2.0 * D[4] * n * p / s * pi[IDX[m][n - 1][p - 1]];
  if (m >= 1 && p >= 1) r += 2.0 * D[5] * m * p / s * pi[IDX[m - 1][n][p - 1]];
  return r;
}

/* central moment (m,n,p) of the discrete Maxwellian (reading R2/R22):
 * rho c_m c_n c_p with c_0 = 1, c_1 = 0, c_2 = c_s^2 */
static double maxwell_central(int m, int n, int p, double rho) {
  const double c[3] = {1.0, 0.0, CS2};
  return rho * c[m] * c[n] * c[p];
}

/* relaxation with source, Appendix D Step 3:
 * kappa~ = kappa + omega (kappa^Mv - kappa) + (1 - omega/2) sigma delta_t, delta_t = 1 */
static double relax(double k, double kmv, double w, double s) {
  return k + w * (kmv - k) + (1.0 - 0.5 * w) * s;
}

/* One collision (Appendix D Steps 7 (for rho,u), 1, 2, 3, 4, 5) at one node.
 * f: 27 pre-collision populations; omega: omega_0..omega_26 (App. D numbering);
 * F: body force; model: 0 = FPC (Markovian attractors), 1 = Maxwellian
 * attractors (MCM, reading R22).  Writes f~ and optionally the pre/post
 * central moments. */
void orc_collide_node(const double* f, const double* omega_in, const double* F, double* ft,
                      double* kappa_pre, double* kappa_post, int model, double les_cd) {
  setup();
  /* Step 7 definitions: rho = sum f, rho u = sum f e + F/2. */
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < Q; ++a) {
    rho += f[a];
    j[0] += f[a] * EX[a];
    j[1] += f[a] * EY[a];
    j[2] += f[a] * EZ[a];
  }
  double u[3];
  for (int d = 0; d < 3; ++d) u[d] = (j[d] + 0.5 * F[d]) / rho;

  /* Step 1: raw moments m = P f.  Step 2: central moments kappa = F(u) m. */
  double m[Q], k[Q];
  double Fu[Q][Q];
  matvec(P, f, m);
  frame_matrix(u, Fu);
  matvec(Fu, m, k);
  if (kappa_pre) memcpy(kappa_pre, k, sizeof k);

  /* LES (reading R25): shear rates from the local deviatoric stress */
  double omega[Q];
  memcpy(omega, omega_in, sizeof omega);
  if (les_cd > 0.0) {
    const double tr = (k[K200] + k[K020] + k[K002]) / 3.0;
    const double dxx = k[K200] - tr, dyy = k[K020] - tr, dzz = k[K002] - tr;
    const double Qs = sqrt(dxx * dxx + dyy * dyy + dzz * dzz +
                           2.0 * (k[K110] * k[K110] + k[K101] * k[K101] + k[K011] * k[K011]));
    const double tau0 = 1.0 / omega_in[4];
    const double tau = 0.5 * (tau0 + sqrt(tau0 * tau0 + 18.0 * sqrt(2.0) * les_cd * les_cd * Qs / rho));
    omega[4] = omega[5] = omega[6] = omega[8] = omega[9] = 1.0 / tau;
  }

  /* Step 3 -- sources sigma_mnp, Eq. (cmupdatesourceD3Q27), reading R8. */
  double ks[Q];
  memcpy(ks, k, sizeof ks);
  ks[K000] = rho;
  ks[K100] = ks[K010] = ks[K001] = 0.0;
  double sg[Q];
  for (int q = 0; q < Q; ++q) {
    const int a = MNP[q][0], b = MNP[q][1], c = MNP[q][2];
    double s = 0.0;
    if (a >= 1) s += a * F[0] / rho * ks[IDX[a - 1][b][c]];
    if (b >= 1) s += b * F[1] / rho * ks[IDX[a][b - 1][c]];
    if (c >= 1) s += c * F[2] / rho * ks[IDX[a][b][c - 1]];
    sg[q] = s;
  }

  /* combined moments of kappa and of sigma */
  const double k2s1 = k[K200] + k[K020] + k[K002], k2d1 = k[K200] - k[K020], k2d2 = k[K200] - k[K002];
  const double s2s1 = sg[K200] + sg[K020] + sg[K002], s2d1 = sg[K200] - sg[K020], s2d2 = sg[K200] - sg[K002];
  const double k3s1 = k[K120] + k[K102], k3m1 = k[K120] - k[K102];
  const double k3s2 = k[K210] + k[K012], k3m2 = k[K210] - k[K012];
  const double k3s3 = k[K201] + k[K021], k3m3 = k[K201] - k[K021];
  const double s3s1 = sg[K120] + sg[K102], s3m1 = sg[K120] - sg[K102];
  const double s3s2 = sg[K210] + sg[K012], s3m2 = sg[K210] - sg[K012];
  const double s3s3 = sg[K201] + sg[K021], s3m3 = sg[K201] - sg[K021];
  const double k4s1 = k[K220] + k[K202] + k[K022], k4d1 = k[K220] + k[K202] - k[K022], k4d2 = k[K220] - k[K202];
  const double s4s1 = sg[K220] + sg[K202] + sg[K022], s4d1 = sg[K220] + sg[K202] - sg[K022], s4d2 = sg[K220] - sg[K202];

  /* attractors up to second order: D'_ii = c_s^2, D'_ij = 0 (order <= 2) */
  double mv[Q];
  memset(mv, 0, sizeof mv);
  const double Deq[6] = {CS2, CS2, CS2, 0.0, 0.0, 0.0};
  double pi_eq[Q];
  memset(pi_eq, 0, sizeof pi_eq);
  pi_eq[K000] = rho;
  mv[K000] = rho;
  for (int q = 1; q < 10; ++q) mv[q] = mv_attractor(MNP[q][0], MNP[q][1], MNP[q][2], Deq, pi_eq);
  /* third-order attractors are zero (reading R11) */
  const double mv2s1 = mv[K200] + mv[K020] + mv[K002], mv2d1 = mv[K200] - mv[K020], mv2d2 = mv[K200] - mv[K002];
  const double mv3 = 0.0;

  /* relax zeroth to second order */
  double kt[Q];
  memset(kt, 0, sizeof kt);
  kt[K000] = relax(k[K000], mv[K000], omega[0], sg[K000]);
  kt[K100] = relax(k[K100], mv[K100], omega[1], sg[K100]);
  kt[K010] = relax(k[K010], mv[K010], omega[2], sg[K010]);
  kt[K001] = relax(k[K001], mv[K001], omega[3], sg[K001]);
  kt[K110] = relax(k[K110], mv[K110], omega[4], sg[K110]);
  kt[K101] = relax(k[K101], mv[K101], omega[5], sg[K101]);
  kt[K011] = relax(k[K011], mv[K011], omega[6], sg[K011]);
  const double kt2s1 = relax(k2s1, mv2s1, omega[7], s2s1);
  const double kt2d1 = relax(k2d1, mv2d1, omega[8], s2d1);
  const double kt2d2 = relax(k2d2, mv2d2, omega[9], s2d2);
  kt[K200] = (kt2s1 + kt2d1 + kt2d2) / 3.0;
  kt[K020] = (kt2s1 - 2.0 * kt2d1 + kt2d2) / 3.0;
  kt[K002] = (kt2s1 + kt2d1 - 2.0 * kt2d2) / 3.0;

  /* relax third order, then decompose (reading R7 for kappa~_021) */
  const double kt3s1 = relax(k3s1, mv3, omega[10], s3s1);
  const double kt3m1 = relax(k3m1, mv3, omega[11], s3m1);
  const double kt3s2 = relax(k3s2, mv3, omega[12], s3s2);
  const double kt3m2 = relax(k3m2, mv3, omega[13], s3m2);
  const double kt3s3 = relax(k3s3, mv3, omega[14], s3s3);
  const double kt3m3 = relax(k3m3, mv3, omega[15], s3m3);
  kt[K111] = relax(k[K111], mv3, omega[16], sg[K111]);
  kt[K120] = 0.5 * (kt3s1 + kt3m1);
  kt[K102] = 0.5 * (kt3s1 - kt3m1);
  kt[K210] = 0.5 * (kt3s2 + kt3m2);
  kt[K012] = 0.5 * (kt3s2 - kt3m2);
  kt[K201] = 0.5 * (kt3s3 + kt3m3);
  kt[K021] = 0.5 * (kt3s3 - kt3m3);

  /* "current" state seen by the higher attractors: post-collision moments with
   * the first-order central moments at zero (reading R10). */
  double cur[Q];
  memcpy(cur, kt, sizeof cur);
  cur[K100] = cur[K010] = cur[K001] = 0.0;
  const double Dh[6] = {kt[K200] / rho, kt[K020] / rho, kt[K002] / rho,
                        kt[K110] / rho, kt[K011] / rho, kt[K101] / rho};

  /* fourth order: attractors from post-collision second order */
  for (int q = K220; q <= K112; ++q)
    mv[q] = model == 1 ? maxwell_central(MNP[q][0], MNP[q][1], MNP[q][2], rho)
                       : mv_attractor(MNP[q][0], MNP[q][1], MNP[q][2], Dh, cur);
  const double mv4s1 = mv[K220] + mv[K202] + mv[K022], mv4d1 = mv[K220] + mv[K202] - mv[K022], mv4d2 = mv[K220] - mv[K202];
  const double kt4s1 = relax(k4s1, mv4s1, omega[17], s4s1);
  const double kt4d1 = relax(k4d1, mv4d1, omega[18], s4d1);
  const double kt4d2 = relax(k4d2, mv4d2, omega[19], s4d2);
  kt[K211] = relax(k[K211], mv[K211], omega[20], sg[K211]);
  kt[K121] = relax(k[K121], mv[K121], omega[21], sg[K121]);
  kt[K112] = relax(k[K112], mv[K112], omega[22], sg[K112]);
  kt[K220] = (kt4s1 + kt4d1 + 2.0 * kt4d2) / 4.0;
  kt[K202] = (kt4s1 + kt4d1 - 2.0 * kt4d2) / 4.0;
  kt[K022] = (kt4s1 - kt4d1) / 2.0;
  for (int q = K220; q <= K112; ++q) cur[q] = kt[q];

  /* fifth order: attractors from post-collision second and third order */
  for (int q = K122; q <= K221; ++q)
    mv[q] = model == 1 ? maxwell_central(MNP[q][0], MNP[q][1], MNP[q][2], rho)
                       : mv_attractor(MNP[q][0], MNP[q][1], MNP[q][2], Dh, cur);
  kt[K122] = relax(k[K122], mv[K122], omega[23], sg[K122]);
  kt[K212] = relax(k[K212], mv[K212], omega[24], sg[K212]);
  kt[K221] = relax(k[K221], mv[K221], omega[25], sg[K221]);
  for (int q = K122; q <= K221; ++q) cur[q] = kt[q];

  /* sixth order: attractor from post-collision second and fourth order */
  mv[K222] = model == 1 ? maxwell_central(2, 2, 2, rho) : mv_attractor(2, 2, 2, Dh, cur);
  kt[K222] = relax(k[K222], mv[K222], omega[26], sg[K222]);
  if (kappa_post) memcpy(kappa_post, kt, sizeof kt);

  /* Step 4: m~ = F^-1 kappa~ with F^-1(u) = F(-u).  Step 5: f~ = P^-1 m~. */
  const double mu[3] = {-u[0], -u[1], -u[2]};
  double mt[Q];
  frame_matrix(mu, Fu);
  matvec(Fu, kt, mt);
  matvec(PINV, mt, ft);
}

/* Equilibrium used for initial states: the populations whose central moments
 * are the attractors evaluated at equilibrium, kappa_abc = rho c_a c_b c_c with
 * c_0 = 1, c_1 = 0, c_2 = c_s^2 (Sec. 3.5 attractor list with the second-order
 * moments at their equilibrium value), mapped back by F(-u) and P^-1. */
void orc_feq(double rho, const double* u, double* feq) {
  setup();
  const double c[3] = {1.0, 0.0, CS2};
  double k[Q], m[Q];
  double Fu[Q][Q];
  for (int q = 0; q < Q; ++q) k[q] = rho * c[MNP[q][0]] * c[MNP[q][1]] * c[MNP[q][2]];
  const double mu[3] = {-u[0], -u[1], -u[2]};
  frame_matrix(mu, Fu);
  matvec(Fu, k, m);
  matvec(PINV, m, feq);
}

/* ---- accessors for the tests ------------------------------------------- */
void orc_lattice(int* ex, int* ey, int* ez, int* opp, int* mnp) {
  setup();
  for (int a = 0; a < Q; ++a) {
    ex[a] = EX[a];
    ey[a] = EY[a];
    ez[a] = EZ[a];
    opp[a] = OPP[a];
    for (int d = 0; d < 3; ++d) mnp[a * 3 + d] = MNP[a][d];
  }
}

void orc_matrices(const double* u, double* p, double* pinv, double* fu, double* finv) {
  setup();
  double A[Q][Q];
  memcpy(p, P, sizeof P);
  memcpy(pinv, PINV, sizeof PINV);
  frame_matrix(u, A);
  memcpy(fu, A, sizeof A);
  const double mu[3] = {-u[0], -u[1], -u[2]};
  frame_matrix(mu, A);
  memcpy(finv, A, sizeof A);
}

double orc_attractor(int m, int n, int p, const double* D, const double* pi) {
  setup();
  return mv_attractor(m, n, p, D, pi);
}

/* ---- whole-lattice operations.  Layout: SoA f[alpha][z][y][x],
 *      node index i = x + nx (y + ny z), N = nx ny nz. ------------------- */

void orc_init(int nx, int ny, int nz, const double* rho, const double* u, double* f) {
  setup();
  const int64_t N = (int64_t)nx * ny * nz;
  for (int64_t i = 0; i < N; ++i) {
    double fe[Q];
    const double ui[3] = {u[i], u[N + i], u[2 * N + i]};
    orc_feq(rho[i], ui, fe);
    for (int a = 0; a < Q; ++a) f[a * N + i] = fe[a];
  }
}

/* Collision at every node (Steps 1-5); g may alias nothing. */
/* C D of reading R25 at layer y: les = {C_s, u_tau / nu (0: no damping), A+}
 * or NULL; the wall distance is that to the nearest y wall (walls bit 0),
 * the symmetry plane (bit 3) excluded. */
static double les_cd(const double* les, int walls, int ny, int y) {
  if (!les || les[0] <= 0.0) return 0.0;
  double d = 1.0;
  if ((walls & 1) && les[1] > 0.0) {
    double yw = y + 0.5;
    if (!(walls & 8) && ny - 0.5 - y < yw) yw = ny - 0.5 - y;
    d = 1.0 - exp(-yw * les[1] / les[2]);
  }
  return les[0] * d;
}

void orc_collide(int nx, int ny, int nz, const double* f, double* g, const double* omega,
                 const double* F, int model, int walls, const double* les) {
  setup();
  const int64_t N = (int64_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    double fi[Q], fo[Q];
    for (int a = 0; a < Q; ++a) fi[a] = f[a * N + i];
    const int y = (int)((i / nx) % ny);
    orc_collide_node(fi, omega, F, fo, NULL, NULL, model, les_cd(les, walls, ny, y));
    for (int a = 0; a < Q; ++a) g[a * N + i] = fo[a];
  }
}

/* rest weights w_a = f^eq(1, 0), for the moving-wall correction */
static double WREST[Q];
static int wrest_ready = 0;
static void setup_wrest(void) {
  if (wrest_ready) return;
  const double zero[3] = {0.0, 0.0, 0.0};
  orc_feq(1.0, zero, WREST);
  wrest_ready = 1;
}

/* Streaming, Eq. (LBMsteps-stream) / Appendix D Step 6, pull form, at node i:
 * fi[a] = g_a(x - e_a), periodic wrap across the faces without walls,
 * halfway bounce-back across the faces with walls (readings R12, R23). */
static void pull_node(int nx, int ny, int nz, int walls, const double* lid, const double* g, int64_t i,
                      double* fi) {
  const int64_t N = (int64_t)nx * ny * nz;
  const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((int64_t)nx * ny));
  for (int a = 0; a < Q; ++a) {
    int xs = x - EX[a], ys = y - EY[a], zs = z - EZ[a];
    const int outx = (walls & 2) && (xs < 0 || xs >= nx);
    const int outy = (walls & 1) && (ys < 0 || ys >= ny);
    const int outz = (walls & 4) && (zs < 0 || zs >= nz);
    if (outy && (walls & 8) && ys >= ny && !outx && !outz) {
      /* specular reflection at the symmetry plane (reading R24) */
      const int xm = (xs % nx + nx) % nx, zm = (zs % nz + nz) % nz;
      int am = 0;
      for (int b = 0; b < Q; ++b)
        if (EX[b] == EX[a] && EY[b] == -EY[a] && EZ[b] == EZ[a]) am = b;
      fi[a] = g[am * N + (xm + (int64_t)nx * (y + (int64_t)ny * zm))];
      continue;
    }
    if (outx || outy || outz) {
      double v = g[OPP[a] * N + i];
      if (lid && (walls & 1) && ys >= ny)
        v += 2.0 * WREST[a] * (EX[a] * lid[0] + EY[a] * lid[1] + EZ[a] * lid[2]) / CS2;
      fi[a] = v;
      continue;
    }
    xs = (xs % nx + nx) % nx;
    ys = (ys % ny + ny) % ny;
    zs = (zs % nz + nz) % nz;
    fi[a] = g[a * N + (xs + (int64_t)nx * (ys + (int64_t)ny * zs))];
  }
}

void orc_stream(int nx, int ny, int nz, int walls, const double* lid, const double* g, double* f) {
  setup();
  setup_wrest();
  const int64_t N = (int64_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    double fi[Q];
    pull_node(nx, ny, nz, walls, lid, g, i, fi);
    for (int a = 0; a < Q; ++a) f[a * N + i] = fi[a];
  }
}

/* The same streaming written in push form, as a cross-check of the pull
 * form: every node sends g_a(x) to x + e_a; a population whose destination
 * lies beyond a walled face returns to x as the opposite velocity (with the
 * lid correction when it crosses the moving lid), and one crossing the
 * symmetry plane lands on (x + e_x, ny-1, z + e_z) with the mirrored
 * velocity. */
void orc_stream_push(int nx, int ny, int nz, int walls, const double* lid, const double* g, double* f) {
  setup();
  setup_wrest();
  const int64_t N = (int64_t)nx * ny * nz;
  for (int64_t i = 0; i < N; ++i) {
    const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((int64_t)nx * ny));
    for (int a = 0; a < Q; ++a) {
      const double val = g[a * N + i];
      int xd = x + EX[a], yd = y + EY[a], zd = z + EZ[a];
      const int outx = (walls & 2) && (xd < 0 || xd >= nx);
      const int outy = (walls & 1) && (yd < 0 || yd >= ny);
      const int outz = (walls & 4) && (zd < 0 || zd >= nz);
      if (outy && (walls & 8) && yd >= ny && !outx && !outz) {
        int am = 0;
        for (int b = 0; b < Q; ++b)
          if (EX[b] == EX[a] && EY[b] == -EY[a] && EZ[b] == EZ[a]) am = b;
        xd = (xd % nx + nx) % nx;
        zd = (zd % nz + nz) % nz;
        f[am * N + (xd + (int64_t)nx * (y + (int64_t)ny * zd))] = val;
        continue;
      }
      if (outx || outy || outz) {
        double v = val;
        /* arrives as OPP[a]; crossed the lid if it left through the top */
        if (lid && (walls & 1) && yd >= ny)
          v += 2.0 * WREST[OPP[a]] * (EX[OPP[a]] * lid[0] + EY[OPP[a]] * lid[1] + EZ[OPP[a]] * lid[2]) / CS2;
        f[OPP[a] * N + i] = v;
        continue;
      }
      xd = (xd % nx + nx) % nx;
      yd = (yd % ny + ny) % ny;
      zd = (zd % nz + nz) % nz;
      f[a * N + (xd + (int64_t)nx * (yd + (int64_t)ny * zd))] = val;
    }
  }
}

/* nsteps of: stream, then collide (one full time step in the paper's order,
 * seen from the post-collision state).  g holds the post-collision state on
 * entry and on exit. */
int orc_run(int nx, int ny, int nz, int walls, const double* lid, const double* omega, const double* F, double* g,
            int nsteps, int model, const double* les) {
  setup();
  const int64_t N = (int64_t)nx * ny * nz;
  double* f = (double*)malloc(sizeof(double) * Q * N);
  if (!f) return -1;
  for (int s = 0; s < nsteps; ++s) {
    orc_stream(nx, ny, nz, walls, lid, g, f);
    orc_collide(nx, ny, nz, f, g, omega, F, model, walls, les);
  }
  free(f);
  return 0;
}

/* One step (stream then collide) evaluated only at the listed nodes, reading
 * the full post-collision state g; out is [27][nsel]. */
void orc_step_nodes(int nx, int ny, int nz, int walls, const double* lid, const double* omega, const double* F,
                    const double* g, const int64_t* sel, int64_t nsel, double* out, int model, const double* les) {
  setup();
  setup_wrest();
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < nsel; ++s) {
    double fi[Q], fo[Q];
    pull_node(nx, ny, nz, walls, lid, g, sel[s], fi);
    const int y = (int)((sel[s] / nx) % ny);
    orc_collide_node(fi, omega, F, fo, NULL, NULL, model, les_cd(les, walls, ny, y));
    for (int a = 0; a < Q; ++a) out[a * nsel + s] = fo[a];
  }
}

/* threads the OpenMP loops above will use (for reporting the baseline) */
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
