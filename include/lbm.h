/*
 * lbm.h -- C ABI of the MI355X (gfx950) D3Q27 Fokker-Planck central-moment
 * lattice Boltzmann library (FPC-LBM, Schupbach & Premnath, arXiv 2410.09739).
 *
 * The library advances a box, periodic or bounded by walls on any faces, with
 * the fused stream-and-collide update of the paper:
 *   - collision of Appendix D Steps 1-5: raw moments (Step 1), central moments
 *     (Step 2, Eq. rmcm), relaxation of each central moment towards its
 *     Markovian attractor (Step 3, Eqs. Mvcmattractor3D and
 *     diffusion-tensor-parameter-3D, attractor list of Sec. 3.5) with the
 *     body-force sources of Eq. (cmupdatesourceD3Q27), and the maps back
 *     (Steps 4 and 5);
 *   - streaming, Eq. (LBMsteps-stream) / Appendix D Step 6, with halfway
 *     bounce-back at the walls, the moving-lid correction and the specular
 *     symmetry plane of the Sec. 4 cavity and half-channel studies;
 *   - options used by those studies: the central-moment scheme with Maxwellian
 *     attractors that Sec. 4 compares against (lbm_config.attractor) and
 *     Smagorinsky LES with van Driest damping (lbm_config.les_*);
 *   - macroscopic fields of Appendix D Step 7: rho = sum f,
 *     rho u = sum f e + F/2, P = rho c_s^2, c_s^2 = 1/3.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid: nx * ny * nz nodes, node index i = x + nx * (y + ny * z), x fastest.
 * Populations: 27 per node in the order of the paper's velocity list (Sec. 3.5),
 *   host arrays are structure-of-arrays f[alpha * N + i], N = nx ny nz.
 * Time levels: the library stores the post-collision populations f~(t) of the
 *   last completed step.  lbm_init stores f^eq(rho, u) as f~(0).  One call of
 *   lbm_step(c, 1) streams f~(t) (Step 6), takes rho and u (Step 7) and collides
 *   (Steps 1-5) to f~(t+1).  lbm_moments reports the Step 7 fields of the
 *   pre-collision state at t: rho = sum f~, rho u = sum f~ e - F/2 (the
 *   collision adds exactly F to sum f e).
 * Walls: walls_y = 1 puts no-slip walls half a link below y = 0 and half a
 *   link above y = ny - 1 (walls_x, walls_z likewise across x and z); faces
 *   without walls are periodic.  The wall above y = ny - 1 may move
 *   (lid_velocity) or be replaced by a symmetry plane (sym_top).
 * Storage forms: the distributions are held as deviations f - w_alpha from the
 *   D3Q27 lattice weights (8/27, 2/27, 1/54, 1/216), in FP64, FP32, FP16 or
 *   BF16.  FP16 and BF16 values carry an exact power-of-two scale per weight
 *   class and are rounded stochastically by default (see lbm_storage);
 *   arithmetic is FP64 for LBM_F64 and FP32 otherwise.  lbm_init, lbm_set_f
 *   round to nearest even.
 * Streams: every device operation is enqueued on the configured HIP stream.
 *   Device memory the caller passes in must be ready on that stream: data
 *   written on another stream must be synchronised first (or the work ordered
 *   with an event) by the caller.
 * Errors: functions return LBM_OK (0) or a negative code; lbm_last_error gives
 *   a text.  No entry point throws, aborts or exits.
 * Ownership: the library owns the device memory it allocates (two state
 *   buffers of 27 * N values plus small scratch); every pointer the caller
 *   passes stays the caller's and is never retained past the call.
 * Threads: one context must not be used by two host threads at once.  The
 *   error text of a call without a context (lbm_last_error(NULL),
 *   lbm_mlp_last_error(NULL)) is kept per host thread.
 */
#ifndef LBM_H
#define LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_OK 0
#define LBM_EINVAL (-1)    /* invalid argument or configuration            */
#define LBM_ENOMEM (-2)    /* device or host allocation failed             */
#define LBM_EHIP (-3)      /* HIP runtime error (text in lbm_last_error)   */
#define LBM_EUNSTABLE (-4) /* diagnostics found non-finite values or rho<=0 */
#define LBM_ESTATE (-5)    /* call out of order (e.g. step before init)    */

#define LBM_Q 27
#define LBM_CLOSURE_NIN 27
#define LBM_CLOSURE_NHID 64
#define LBM_CLOSURE_NOUT 6
/* W1[64][27] b1[64] W2[64][64] b2[64] W3[6][64] b3[6] */
#define LBM_CLOSURE_NPARAM 6342

/* Storage forms.  LBM_F16DEV / LBM_BF16DEV round every stored value
 * stochastically (hardware conversion with a counter-based random word of
 * node and step: unbiased, reproducible); the _RNE forms round to nearest even. */
typedef enum {
  LBM_F64 = 0,
  LBM_F32 = 1,
  LBM_F16DEV = 2,
  LBM_BF16DEV = 3,
  LBM_F16DEV_RNE = 4,
  LBM_BF16DEV_RNE = 5
} lbm_storage;

/* How the 27 relaxation rates omega_0..omega_26 (Appendix D numbering) are set.
 * In all modes omega_4,5,6,8,9 come from the shear viscosity through
 * Eq. (transportcoeff3DFPCLBM), 1/omega = nu / c_s^2 + 1/2, and omega_7 is
 * omega_bulk (bulk viscosity zeta = (2/3) c_s^2 (1/omega_7 - 1/2)), except in
 * LBM_OMEGA_EXPLICIT.
 *   LBM_OMEGA_PAPER        omega_0..3 = 1 (no effect), omega_10..26 = omega_higher
 *                          (the paper's runs use 1 for these and for omega_7).
 *   LBM_OMEGA_ORDER_SCALED moments of order n >= 3 take the order-scaled rate of
 *                          Eq. (FPcoll3d), omega_n = (n/2) omega_2, through the
 *                          Henon correction: 1/omega_n - 1/2 = (2/n)(1/omega_2 - 1/2).
 *   LBM_OMEGA_EXPLICIT     omega[] is used as given.
 * Every rate must lie in (0, 2). */
typedef enum { LBM_OMEGA_PAPER = 0, LBM_OMEGA_ORDER_SCALED = 1, LBM_OMEGA_EXPLICIT = 2 } lbm_omega_mode;

/* Attractors of the central moments of order >= 4.
 *   LBM_ATTRACTOR_FPC      the Markovian attractors of FPC-LBM, Eq. (Mvcmattractor3D)
 *                          with the diffusion tensor of Eq. (diffusion-tensor-parameter-3D),
 *                          built from the post-collision lower moments (Appendix D Step 3).
 *   LBM_ATTRACTOR_MAXWELL  the discrete Maxwellian's central moments rho c_a c_b c_c,
 *                          c = (1, 0, c_s^2): the central-moment scheme with Maxwellian
 *                          equilibria (MCM-LBM) that Sec. 4 compares against, e.g. in the
 *                          crossing shear wave study.  Orders <= 3, rates and sources are
 *                          the same in both.  Not available with the learned closure. */
typedef enum { LBM_ATTRACTOR_FPC = 0, LBM_ATTRACTOR_MAXWELL = 1 } lbm_attractor;

typedef struct {
  int32_t nx, ny, nz;   /* >= 1 each; N = nx*ny*nz must be < 2^31              */
  int32_t storage;      /* lbm_storage                                          */
  int32_t walls_y;      /* 0: periodic in y; 1: halfway bounce-back walls in y  */
  int32_t omega_mode;   /* lbm_omega_mode                                       */
  double nu;            /* shear viscosity, lattice units (> 0 unless EXPLICIT) */
  double omega_bulk;    /* omega_7                                              */
  double omega_higher;  /* omega_10..26 in LBM_OMEGA_PAPER                      */
  double omega[LBM_Q];  /* LBM_OMEGA_EXPLICIT only                              */
  double force[3];      /* body force per unit volume, lattice units, dt = 1    */
  void* hip_stream;     /* hipStream_t to run on; NULL: the library makes one   */
  int32_t attractor;    /* lbm_attractor (default LBM_ATTRACTOR_FPC)            */
  int32_t walls_x;      /* 0: periodic in x; 1: halfway bounce-back walls half a */
  int32_t walls_z;      /*   link outside the first and last layer (same for z)  */
  double lid_velocity[3]; /* velocity of the wall above y = ny-1 (needs walls_y; */
                        /* Sec. 4 lid-driven cavity): every link through it gets */
                        /* the momentum correction 2 w_a (e_a . U) / c_s^2;      */
                        /* zeros = resting wall.  Not with the learned closure.  */
  int32_t sym_top;      /* 1: the face above y = ny-1 is a specular symmetry     */
                        /* plane (Sec. 4 half channel; needs walls_y for the     */
                        /* wall below y = 0, no lid)                            */
  double les_cs;        /* Smagorinsky constant C (Sec. 4 channel LES); 0 = off */
  double les_wall_units;/* u_tau / nu for the van Driest damping                */
                        /* D = 1 - exp(-y+ / les_aplus), y+ from the nearest y   */
                        /* wall half a link outside; 0 = no damping (D = 1)     */
  double les_aplus;     /* van Driest constant A+ (default 26)                  */
} lbm_config;

typedef struct {
  double mass;            /* sum rho                                              */
  double momentum[3];     /* sum rho u (Step 7 definition)                        */
  double kinetic_energy;  /* 1/2 sum rho |u|^2                                    */
  double enstrophy;       /* 1/2 sum |curl u|^2, curl u by centred differences   */
                          /* (q(i+1) - q(i-1))/2 of the Step 7 velocity; periodic */
                          /* axes wrap; ghost value -u across a resting wall,     */
                          /* 2U - u across the moving lid, mirrored tangential u  */
                          /* across the symmetry plane                            */
  double wall_force[3];   /* force of the fluid on the walls: sum over the links  */
                          /* from a fluid node into a wall (any walled face; the  */
                          /* symmetry plane takes none) of 2 f~_alpha e_alpha;    */
                          /* at a moving lid the momentum correction of the       */
                          /* bounced population is not included; zero without     */
                          /* walls                                                */
  double max_speed;       /* max |u|                                              */
  double min_rho;         /* min rho                                              */
  int64_t n_nonfinite;    /* nodes with a non-finite population                   */
  int64_t step;           /* completed time steps                                 */
} lbm_diag;

typedef struct lbm_ctx lbm_ctx;

/* Fills cfg with defaults: 0 sizes, LBM_F32, periodic, LBM_OMEGA_PAPER,
 * nu = 1/6, omega_bulk = omega_higher = 1, zero force, NULL stream,
 * LBM_ATTRACTOR_FPC, no x/z walls, resting walls, no symmetry plane, no LES
 * (les_aplus = 26). */
void lbm_config_default(lbm_config* cfg);

/* Host-only: the 27 rates the configuration implies (no GPU needed).
 * Returns LBM_EINVAL (with no output written) if any rate falls outside (0,2). */
int lbm_omega_table(const lbm_config* cfg, double omega_out[LBM_Q]);

/* Validates cfg, allocates the two device state buffers and scratch on the
 * current HIP device and clears the buffers on the context's stream; returns
 * once that clear has finished.  *out receives the context (NULL on error; the
 * error text is then available from lbm_last_error(NULL)). */
int lbm_create(const lbm_config* cfg, lbm_ctx** out);

/* Stores f~(0) = f^eq(rho, u) at every node, where f^eq has the equilibrium
 * central moments rho c_a c_b c_c (c_0 = 1, c_1 = 0, c_2 = c_s^2) of the
 * attractor list of Sec. 3.5 about velocity u.  rho: host array [N] or NULL
 * (rho = 1); u: host array [3][N] (SoA) or NULL (u = 0).  Resets the step count.
 * Synchronous. */
int lbm_init(lbm_ctx* c, const double* rho, const double* u);

/* Enqueues n >= 0 fused stream-and-collide steps; returns once they are queued. */
int lbm_step(lbm_ctx* c, int64_t n);

/* Blocks until all work queued on the context's stream has finished. */
int lbm_synchronize(lbm_ctx* c);

/* Step 7 fields of the current time level to host arrays rho [N] and u [3][N]
 * (either may be NULL), summed in FP64 from the stored populations whatever
 * the storage form.  Synchronous. */
int lbm_moments(lbm_ctx* c, double* rho, double* u);

/* Same fields into caller-owned device memory, enqueued on the stream:
 * rho_dev [N], u_dev [3][N]; element type double if f64 != 0 (summed in FP64),
 * else float (summed in the storage form's arithmetic type). */
int lbm_moments_device(lbm_ctx* c, void* rho_dev, void* u_dev, int32_t f64);

/* FP64 reductions over the current state (deterministic order).  Synchronous.
 * Returns LBM_EUNSTABLE (after filling *out) if a population is non-finite or
 * some rho <= 0. */
int lbm_diagnostics(lbm_ctx* c, lbm_diag* out);

/* Checkpoint / parity access to the stored post-collision populations f~ as
 * host FP64 [27][N].  lbm_set_f rounds to the storage form (round to nearest
 * even) and marks the context initialised.  Synchronous. */
int lbm_get_f(lbm_ctx* c, double* f);
int lbm_set_f(lbm_ctx* c, const double* f);

/* The stored post-collision populations of listed nodes only (probe points,
 * or parity checks of grids too large to copy whole): nodes[count] flat
 * indices i = x + nx (y + ny z), host; f host FP64 [27][count], the values
 * lbm_get_f would give at those nodes.  count = 0 does nothing; an index
 * outside [0, N) is LBM_EINVAL.  Synchronous. */
int lbm_get_f_nodes(lbm_ctx* c, const int64_t* nodes, int64_t count, double* f);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving or monitoring loops, harnesses that forbid hipMalloc): the same as
 * lbm_get_f_nodes, with identical results, but it allocates nothing.  The
 * node list and the populations are staged in a fixed device array of
 * LBM_NOALLOC_MAX_NODES * (8 + 27 * 8) bytes (917,504) that the library holds
 * on every GPU it runs on until the process ends (its address is looked up
 * once per device by lbm_create).  count > LBM_NOALLOC_MAX_NODES is
 * LBM_EINVAL; the other errors are those of lbm_get_f_nodes.  All calls on one
 * GPU share that array: calls that overlap in time on one GPU (from several
 * host threads or contexts) race and must be serialised by the caller.  The
 * host copies use the caller's pointers as given (pageable memory is copied
 * through the runtime).  Synchronous. */
#define LBM_NOALLOC_MAX_NODES 4096
int lbm_get_f_nodes_noalloc(lbm_ctx* c, const int64_t* nodes, int64_t count, double* f);

/* Bit-exact checkpoint of the raw storage: one state buffer as the library
 * keeps it in device memory (deviations f - w in the storage type, FP16/BF16
 * scaled; blocked by 64-node x segments, each holding its 27 directions, nx
 * padded to a multiple of 64, padding zero).  Opaque apart from its size;
 * restore it into a context created with the same configuration.  nbytes must
 * equal lbm_state_bytes(c).  Synchronous. */
int64_t lbm_state_bytes(const lbm_ctx* c);
int lbm_get_raw(lbm_ctx* c, void* host, int64_t nbytes);
int lbm_set_raw(lbm_ctx* c, const void* host, int64_t nbytes);

/* The HIP stream the context runs on (a hipStream_t). */
void* lbm_stream(const lbm_ctx* c);

/* Completed time steps since lbm_init / lbm_set_f / lbm_set_raw. */
int64_t lbm_step_count(const lbm_ctx* c);

/* Sets the step counter (e.g. after lbm_set_raw, so that a resumed run draws
 * the same stochastic-rounding words as an uninterrupted one). */
int lbm_set_step_count(lbm_ctx* c, int64_t steps);

/* Releases every resource of c (NULL is ignored).  Synchronizes first. */
void lbm_destroy(lbm_ctx* c);

/* Last error text of c, or of the last failed lbm_create when c is NULL.
 * Valid until the next call on the same context. */
const char* lbm_last_error(const lbm_ctx* c);

/* ---------------------------------------------------------------------------
 * Learned second-order closure (not part of the paper: a learned eddy
 * viscosity on top of its second-order relaxation).
 * A per-node network 27 -> 64 -> 64 -> 6 (ReLU hidden layers) maps features of
 * the node's pre-collision central moments (Appendix D Step 2) to eddy
 * viscosities nu_t,j of the six second-order groups relaxed with omega_4..9
 * (110, 101, 011, 2s1, 2d1, 2d2), applied through Eq. (transportcoeff3DFPCLBM)
 * as 1/omega_j,eff = 1/omega_j + 3 clamp(nu_t,j, 0, 1/3).
 * Features: x_000 = rho - 1; x_100 = x_010 = x_001 = 0 (the first-order central
 * moments are -F/2 at every node); for the other 23 moments, in the paper's
 * order, (kappa_abc - rho c_a c_b c_c) / rho * 3^((a+b+c)/2).
 * Parameters: LBM_CLOSURE_NPARAM floats W1[64][27] b1[64] W2[64][64] b2[64]
 * W3[6][64] b3[6] (row-major, W[out][in]) acting on raw features.  The fused
 * kernel rounds weights and activations to BF16 and accumulates in FP32 on
 * the matrix cores.
 */

/* Enables the closure in lbm_step (params != NULL, copied) or disables it
 * (NULL).  Requires nx % 64 == 0.  Synchronous. */
int lbm_set_closure(lbm_ctx* c, const float* params);

/* Features the next collision would see at every node, to caller device memory
 * x_dev [N][27] (float).  Enqueued on the context's stream. */
int lbm_closure_features(lbm_ctx* c, float* x_dev);

/* The fused kernel's BF16 MFMA evaluation of the network on given features:
 * x_dev [n][27] -> nu_dev [n][6] (device, float).  Synchronous on hip_stream
 * (NULL: the null stream).  Errors: lbm_mlp_last_error(NULL). */
int lbm_closure_eval(const float* params, const float* x_dev, float* nu_dev, int64_t n, void* hip_stream);

/* 2x2x2 box filter of the current state of c (nx, ny, nz even) onto the
 * coarse grid (nx/2, ny/2, nz/2), caller device memory, FP64:
 * rho_dev [Nc] (mean density), u_dev [3][Nc] (Favre velocity avg(rho u)/avg(rho)),
 * tau_dev [6][Nc] (sub-filter stress avg(rho u_i u_j) - rho u_i u_j; xx, yy, zz,
 * xy, xz, yz), and, unless sbar_dev is NULL, sbar_dev [6][Nc] (Favre-filtered
 * fine strain rate in coarse lattice units, 2 avg(rho S) / avg(rho), S the
 * centred-difference strain of the fine velocity as in lbm_closure_targets;
 * periodic and y-wall lattices only, else LBM_EINVAL).  Fine rho, u are the
 * Step 7 fields.  Enqueued on the stream. */
int lbm_coarsen(lbm_ctx* c, double* rho_dev, double* u_dev, double* tau_dev, double* sbar_dev);

/* lbm_init from device fields rho_dev [N], u_dev [3][N] (FP64).  Synchronous. */
int lbm_init_device(lbm_ctx* c, const double* rho_dev, const double* u_dev);

/* Eddy-viscosity targets on the grid of c from filtered fields (as written by
 * lbm_coarsen): per node y_dev[i][6] (float) =
 * max(0, S_j (nu_j (Sbar_j - S_j) - tau_j / (2 rho)) / (S_j^2 + eps^2)) for the
 * groups 110, 101, 011 (tau_j, S_j, Sbar_j: the xy, xz, yz entries;
 * nu_j = (1/omega_{4+j} - 1/2) / 3, the viscosity of c for the group), and 0 for
 * 2s1, 2d1, 2d2: the eddy viscosity that makes the coarse node carry the
 * filtered fine stress (sub-filter plus viscous) in the least-squares sense.
 * S is the strain rate of u by centred differences (periodic, or an
 * antisymmetric ghost across the walls); eps = eps_rel * rms(S), rms over the
 * 3 N entries of S_ii^2 + 2 S_ij^2.  Periodic and y-wall lattices only.
 * Synchronous. */
int lbm_closure_targets(lbm_ctx* c, const double* rho_dev, const double* u_dev, const double* tau_dev,
                        const double* sbar_dev, double eps_rel, float* y_dev);

/* Training of the closure network on the GPU (FP32 forward and backward
 * kernels, Adam).  Inputs are standardised, (x - mu) / sigma (sigma = 0 drops a
 * feature), targets scaled by 1 / s_y; lbm_mlp_export folds both into
 * parameters for lbm_set_closure.  Loss: mean over the batch and the 6 outputs
 * of the squared error.  All data pointers are device memory, float,
 * x [n][27], y [n][6]. */
typedef struct lbm_mlp lbm_mlp;
int lbm_mlp_create(uint64_t seed, void* hip_stream, lbm_mlp** out); /* He-uniform init from seed */
int lbm_mlp_set_params(lbm_mlp* m, const float* p);                /* host, standardised space; resets Adam */
int lbm_mlp_get_params(lbm_mlp* m, float* p);                      /* host */
int lbm_mlp_set_normalisation(lbm_mlp* m, const float* mu, const float* sigma, float s_y); /* host; finite, sigma >= 0, s_y > 0 */
int lbm_mlp_get_normalisation(lbm_mlp* m, float* mu, float* sigma, float* s_y);             /* host */
/* mu, sigma per feature (population std; sigma below 1e-7 of the largest -> 0)
 * and s_y = rms of all targets, computed on the device. */
int lbm_mlp_fit_normalisation(lbm_mlp* m, const float* x_dev, const float* y_dev, int64_t n);
/* full-batch loss and gradient (host grad[LBM_CLOSURE_NPARAM], may be NULL) */
int lbm_mlp_loss_grad(lbm_mlp* m, const float* x_dev, const float* y_dev, int64_t n, double* loss, float* grad);
/* `steps` Adam steps (beta 0.9, 0.999, eps 1e-8) on minibatches of `batch`
 * samples drawn with replacement by a counter-based generator of (seed, step,
 * slot); loss_out (host, `steps` entries) may be NULL.  Synchronous. */
int lbm_mlp_train(lbm_mlp* m, const float* x_dev, const float* y_dev, int64_t n, int32_t batch, int32_t steps,
                  float lr, uint64_t seed, double* loss_out);
int lbm_mlp_export(lbm_mlp* m, float* params_raw); /* host, for lbm_set_closure */
void lbm_mlp_destroy(lbm_mlp* m);
const char* lbm_mlp_last_error(const lbm_mlp* m);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
