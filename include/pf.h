/* libpf: pseudospectral phase-field ImEx-ARK hot path for MI355X (gfx950).
 *
 * The library advances the state vector y = (c, eta_1, eta_2, eta_3) of one
 * Cahn-Hilliard composition and three Allen-Cahn order parameters, coupled by
 * homogeneous-modulus (Khachaturyan) elasticity on a periodic 3D grid, with
 * additive ImEx Runge-Kutta methods.  It follows the paper's statement of the
 * problem: the ImEx ODE y' = f^I(t,y) + f^E(t,y) in reciprocal space
 * (Methods, "Time integration", Eq. imex_ode), stiff linear terms implicit and
 * solved per wavevector (Eqs. composition, order), the stage and update
 * formulas of Eq. ARK_method, the embedded error of Eq. ARK_embedding and the
 * WRMS acceptance test of Eqs. wrms_norm / wrms_weights.
 *
 * Conventions (every entry point):
 *  - Real-space fields are float64, C order [z][y][x] (x fastest);
 *    eta is stacked [3][z][y][x].
 *  - Reciprocal-space arrays are complex128 (interleaved re, im), layout
 *    [4][nz][ny][kp] with kp = pf_kspace_pitch(ctx) >= nx/2 + 1; entries with
 *    kx >= nx/2 + 1 are padding (ignored on input, undefined on output).
 *    Field order c, eta_1, eta_2, eta_3.  Forward transform unnormalised,
 *    u~(k) = sum_r u(r) exp(-i k.r), k_i = 2 pi m_i / (N_i dx).
 *  - Pointers marked "device" must be device memory of the GPU current at
 *    pf_init; pointers marked "host or device" are selected by on_device.
 *    The caller owns every pointer it passes; libpf owns its workspace and
 *    frees it in pf_finalize.
 *  - All work is ordered on the HIP stream given to pf_init (NULL = default
 *    stream).  Entry points that return host values synchronise that stream.
 *  - Errors are returned as pf_status codes; nothing is thrown across the
 *    ABI.  A context is not thread-safe.
 */
#ifndef PF_H_
#define PF_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pf_ctx pf_ctx;

typedef enum {
  PF_OK = 0,
  PF_ERR_ARG = -1,              /* invalid argument or parameter */
  PF_ERR_OOM = -2,              /* device allocation failed */
  PF_ERR_HIP = -3,              /* a HIP runtime call failed */
  PF_ERR_UNSUPPORTED_SIZE = -4, /* grid size not in the supported set */
  PF_ERR_STEP_FAIL = -5,        /* too many consecutive rejected steps */
  PF_ERR_NONFINITE = -6,        /* a step produced NaN/Inf (state unchanged) */
  PF_ERR_STATE = -7             /* call not valid in the context's state */
} pf_status;

typedef enum { PF_FP64 = 0, PF_MIXED = 1 } pf_precision;

/* ImEx-ARK pairs (Methods, "Time integration"; the orders of the paper's
 * order study, Results, "Improved performance via time integration
 * approach"): IMEX Euler as a 2-stage pair (1 explicit RHS per step, no
 * embedding); ARK2 of Giraldo, Kelly & Constantinescu 2013 (3, first-order
 * embedding); ARK3(2)4L[2]SA (4) and ARK4(3)6L[2]SA (6) of Kennedy &
 * Carpenter 2003.  Adaptive stepping needs an embedded pair. */
typedef enum { PF_IMEX_EULER = 1, PF_ARK2 = 2, PF_ARK324L = 3, PF_ARK436L = 4 } pf_method;

/* Model, discretisation and integrator parameters.
 * Model (Methods, "Phase-field model formulation", dimensionless stand-in):
 *   f = W (c-c_m)^2 (1-H) + W (c-c_p)^2 H + w sum_v eta_v^2 (1-eta_v)^2,
 *   H = sum_v h(eta_v), h(e) = e^3 (6e^2 - 15e + 10),
 *   gradient energy kappa_c/2 |grad c|^2 + kappa_eta/2 sum_v |grad eta_v|^2,
 *   elastic energy with cubic stiffness (C11, C12, C44) and the diagonal
 *   eigenstrain eps_star[v][axis] of variant v (mechanical equilibrium,
 *   Eq. u_gov, with one stiffness for all phases, solved per wavevector).
 *   dc/dt = div(M grad dF/dc) (Eq. x_gov), deta_v/dt = -L dF/deta_v (Eq. phi_gov).
 * Split: f^I_c = -M k^2 (a_c + kappa_c k^2) c~ with a_c = 2W when
 *   implicit_bulk_c = 1 (default) else 0; f^I_eta = -L kappa_eta k^2 eta~.
 * Sizes: nx, ny, nz each one of the compiled line lengths 8, 16, 24, 32, 40,
 *   48, 56, 64, 80, 96, 128, 160, 168, 192, 256, 320, 336, 384, 504, 512
 *   (multiples of 8 with prime factors 2, 3, 5, 7; the factor-7 lengths are
 *   the paper's 168^3, 336^3 and 504^3 grids); see pf_size_supported. */
typedef struct {
  int32_t nx, ny, nz;
  double dx;
  double W, w, kappa_c, kappa_eta, M, L, c_m, c_p;
  double C11, C12, C44;
  double eps_star[3][3];    /* [variant][axis x,y,z], diagonal eigenstrains */
  double eps_bar[3];        /* prescribed diagonal mean strain (mode 0) */
  int32_t mean_strain_mode; /* 0: prescribed eps_bar, 1: stress-free */
  int32_t implicit_bulk_c;  /* 1: 2W k^2 implicit (default), 0: explicit */
  int32_t precision;        /* pf_precision */
  int32_t method;           /* pf_method */
  int32_t adaptive;         /* 1: embedded-error step control (ARK2, ARK324L, ARK436L) */
  double dt0, rtol, atol, dt_min, dt_max;
  int32_t max_rejects;      /* consecutive rejections before PF_ERR_STEP_FAIL */
  /* Vector the WRMS norm of Eqs. wrms_norm / wrms_weights is taken over:
   * 0 (default): the 4 fields' reciprocal-space coefficients scaled to a
   *   unitary transform, each half-spectrum mode counted with its
   *   multiplicity, weights (rtol |Y_{n-1}| + atol)^-1 per coefficient;
   * 1: the 4 real fields point by point, weights (rtol |y_{n-1}(r)| + atol)^-1
   *   (the paper applies the test to the change of the fields; two extra
   *   inverse 3D transforms of 4 fields per attempted step, single grids only). */
  int32_t norm_space;
  /* Inhomogeneous elasticity (Eq. u_gov with the Reuss average of the
   * phases' stiffness; Methods, "MEUMAPPS C++ and the MEUMAPPS-SS
   * application": the Hu-Chen iteration; Results, "Improved performance via
   * time integration approach": its tight 1e-16 and loose 1e-6 tolerances).
   * 1: local stiffness C(r) = (H S_p + (1 - H) S_m)^-1 between the matrix
   * stiffness (C11, C12, C44) and the precipitate stiffness (C11p, C12p,
   * C44p, shared by every variant, cubic in the grid axes), H = sum_v
   * h(eta_v); mechanical equilibrium by the polarisation iteration with the
   * reference stiffness (C_m + C_p) / 2, started from its homogeneous
   * solution at every RHS evaluation and stopped when the largest change of
   * a strain component is <= el_tol or after el_max_iter updates.  Needs
   * precision FP64 and mean_strain_mode 0; single grids only.  0 (default):
   * one stiffness (C11, C12, C44), solved exactly per wavevector. */
  int32_t elastic_inhom;
  double C11p, C12p, C44p;
  double el_tol;
  int32_t el_max_iter;
} pf_params;

typedef struct {
  int64_t steps;       /* accepted steps */
  int64_t attempts;    /* attempted steps */
  int64_t rejects;     /* rejected attempts */
  int64_t n_rhs;       /* explicit RHS evaluations */
  double t;            /* current time */
  double dt_last;      /* last accepted step size */
  double dt_next;      /* proposed next step size */
  double dt_min_seen, dt_max_seen;
  double err_last;     /* WRMS error estimate of the last attempt */
  double mass;         /* mean of c (k = 0 coefficient / N^3) */
  double elapsed_ms;   /* device time spent in pf_advance / pf_ark_step */
  double F;            /* total free energy (Eq. 1 on the grid; see pf_free_energy) */
  double vf;           /* precipitate volume fraction: mean of H = sum_v h(eta_v) */
  double vf_threshold; /* fraction of points with max_v eta_v > 1/2 */
  int64_t el_iterations; /* elastic_inhom: iteration updates over all RHS evaluations */
  int64_t el_last;       /* elastic_inhom: updates in the last RHS evaluation */
} pf_stats;

/* Fills p with the defaults of the stand-in model (Methods, "Phase-field
 * model formulation", restricted to one stiffness and a per-variant double
 * well): W=w=kappa=M=L=1, c_m=0.02, c_p=0.25, C=(250,150,120), eigenstrain
 * 0.0286 along the variant axis and 0.0067 on the others, dx=1, ARK4(3)6L
 * (the fourth-order pair of Methods, "Time integration"), FP64, fixed step
 * 1e-2, k-space WRMS.  PF_ERR_ARG for NULL p, else PF_OK. */
pf_status pf_default_params(pf_params* p);

/* Returns 1 if n is a supported grid length (the list under pf_params),
 * else 0: the line lengths the 3D real FFT of the pseudospectral
 * discretisation (Methods, "MEUMAPPS C++ and the MEUMAPPS-SS application")
 * is compiled for.  Never fails. */
int32_t pf_size_supported(int32_t n);

/* Creates a context for the grid and model in *p on the current device and
 * allocates its workspace: the state vector and the stage derivative arrays
 * of the ImEx-ARK pair (Eq. ARK_method), FFT temporaries, reductions.  The
 * state is the reciprocal-space vector the integrator advances (Methods,
 * "Time integration": the state is held in the fields' reciprocal-space
 * coefficients, device-resident throughout).  hip_stream: a hipStream_t or
 * NULL (default stream).  On success *out owns the workspace; release it
 * with pf_finalize.  Errors: PF_ERR_ARG (NULL pointer or bad parameter),
 * PF_ERR_UNSUPPORTED_SIZE, PF_ERR_OOM, PF_ERR_HIP (no usable device). */
pf_status pf_init(const pf_params* p, void* hip_stream, pf_ctx** out);

/* Frees the context and its workspace (NULL is a no-op). */
void pf_finalize(pf_ctx* ctx);

/* Row pitch kp (complex elements) of every reciprocal-space array (the
 * half spectrum of the real transform, padded; 0 for NULL). */
int64_t pf_kspace_pitch(const pf_ctx* ctx);

/* Bytes of device workspace the context holds (0 for NULL). */
int64_t pf_workspace_bytes(const pf_ctx* ctx);

/* Sets the state vector from real-space fields: composition c and order
 * parameters eta_1..3 (Methods, "Time integration": the state is built from
 * the composition and order-parameter fields), transformed to reciprocal
 * space.  c: N = nz*ny*nx values; eta: 3N values; host or device per
 * on_device (both caller-owned, read only).  Resets t to t0 and the step
 * controller's memory of a rejection.  Errors: PF_ERR_ARG, PF_ERR_HIP. */
pf_status pf_set_state(pf_ctx* ctx, const double* c, const double* eta,
                       int32_t on_device, double t0);

/* Writes the real-space state into c (N values) and eta (3N values), host or
 * device per on_device (inverse transform of the reciprocal-space state,
 * Methods, "MEUMAPPS C++ and the MEUMAPPS-SS application").  Errors:
 * PF_ERR_ARG, PF_ERR_HIP. */
pf_status pf_get_state(pf_ctx* ctx, double* c, double* eta, int32_t on_device);

/* Copies the reciprocal-space state vector (Methods, "Time integration") to
 * / from caller-owned device memory y_hat (layout above); set resets t to
 * t0.  Errors: PF_ERR_ARG, PF_ERR_HIP. */
pf_status pf_get_state_hat(pf_ctx* ctx, void* y_hat_device);
pf_status pf_set_state_hat(pf_ctx* ctx, const void* y_hat_device, double t0);

/* One evaluation of the split right-hand side at the reciprocal-space state
 * y_hat (device, read only): fI_hat = f^I(y), fE_hat = f^E(y) (device,
 * written).  Autonomous: t is accepted for interface symmetry.  This is the
 * stage right-hand side of Eq. ARK_stage: inverse 3D FFT of the state,
 * pointwise driving forces, forward FFT of h(eta_v), per-wavevector elastic
 * solve, inverse FFT of the elastic potentials, forward FFT of the AC
 * driving forces.  Does not change the context's state. */
pf_status pf_rhs(pf_ctx* ctx, double t, const void* y_hat, void* fI_hat, void* fE_hat);

/* Attempts one step of size dt from the current state (Eq. ARK_method).
 * With adaptive control the step is accepted iff the WRMS norm of the
 * embedded error estimate is <= 1; otherwise always (if finite).  On
 * acceptance the state and t advance.  Outputs (any may be NULL): the
 * controller's next step size, the WRMS error (0 without embedding) and the
 * acceptance flag.  Returns PF_ERR_NONFINITE (state unchanged) if the
 * attempt produced NaN/Inf in a fixed-step run. */
pf_status pf_ark_step(pf_ctx* ctx, double dt, double* dt_next, double* err_wrms,
                      int32_t* accepted);

/* Advances to t_final: fixed steps of dt0 or the adaptive controller, the
 * last step clipped to land on t_final.  Fills *out if non-NULL.
 * PF_ERR_STEP_FAIL after max_rejects consecutive rejections. */
pf_status pf_advance(pf_ctx* ctx, double t_final, pf_stats* out);

/* Counters of the integrator (accepted / attempted / rejected steps and
 * explicit RHS evaluations, the cost measure of Results, "Improved
 * performance via time integration approach"), step sizes, and the state's
 * diagnostics: mass, total free energy F and volume fraction (as
 * pf_free_energy and pf_diagnostics; about the cost of one RHS evaluation).
 * pf_advance fills its *out the same way.  Errors: PF_ERR_ARG, PF_ERR_HIP. */
pf_status pf_get_stats(pf_ctx* ctx, pf_stats* out);

/* Current time (0 for NULL); pf_set_dt sets the next attempted step size
 * (PF_ERR_ARG unless dt > 0). */
double pf_get_time(const pf_ctx* ctx);
pf_status pf_set_dt(pf_ctx* ctx, double dt);

/* Mean of c, mean of H = sum_v h(eta_v) (precipitate volume fraction, with
 * the interpolation function h of Methods, "Phase-field model formulation")
 * and the fraction of points with max_v eta_v > 0.5, from the current state,
 * in FP64.  Output pointers may be NULL.  Errors: PF_ERR_ARG, PF_ERR_STATE
 * (no state set), PF_ERR_HIP. */
pf_status pf_diagnostics(pf_ctx* ctx, double* mass, double* vf, double* vf_threshold);

/* Total free energy of the current state (Eq. 1 with the stand-in model's
 * bulk density f, isotropic gradient energies and the elastic energy at
 * mechanical equilibrium, Eq. u_gov), in FP64 on the grid:
 *   F = dx^3 [ sum_r f(c, eta) + 1/(2 N^3) sum_k m(k) k^2 (kappa_c |c~|^2
 *       + kappa_eta sum_v |eta~_v|^2) + 1/(2 N^3) sum_k m(k) sum_vw
 *       B_vw(k) Re(th~_v conj th~_w) + mean-strain terms ],
 * th_v = h(eta_v), m(k) the half-spectrum multiplicity, B the per-wavevector
 * elastic kernel (its k = 0 value per mean_strain_mode); with a prescribed
 * mean strain the terms N^3/2 eps_bar:C:eps_bar - eps_bar:C:sum_v
 * eps*_v th~_v(0).  F is the Lyapunov functional of the gradient flow
 * (Eqs. x_gov, phi_gov).  Errors: PF_ERR_ARG, PF_ERR_STATE, PF_ERR_HIP. */
pf_status pf_free_energy(pf_ctx* ctx, double* F);

/* Standalone 3D real FFT of nf fields (the transform every stage uses to
 * move fields between real and reciprocal space, Methods, "MEUMAPPS C++ and
 * the MEUMAPPS-SS application"; errors PF_ERR_ARG, PF_ERR_HIP).
 * dir = -1: real [nf][nz][ny][nx] -> reciprocal [nf][nz][ny][kp] (unnormalised);
 * dir = +1: reciprocal -> real, scaled by 1/(nx ny nz).
 * in/out: device; nf in 1..4; in and out must not overlap.  The inverse
 * overwrites `in` (it is used as the intermediate). */
pf_status pf_fft3d(pf_ctx* ctx, int32_t dir, int32_t nf, void* in, void* out);

/* Per-kernel-class timing with HIP events on the context's stream (the
 * profile breakdown of Results, "Improved performance via GPU acceleration",
 * by kernel class).
 * pf_profile_enable(ctx, on) clears the counters and turns recording on/off.
 * Classes 0 .. pf_profile_classes()-1 are named by pf_profile_name (never
 * NULL; "" for an invalid class).  pf_profile_get returns the summed device
 * milliseconds, the number of launches and the summed algorithmic bytes
 * (bytes each launch must read and write once: valid half-spectrum entries
 * of every array it touches) of a class.  Intended for measurement, not for
 * use under graph capture. */
pf_status pf_profile_enable(pf_ctx* ctx, int32_t on);
int32_t pf_profile_classes(void);
const char* pf_profile_name(int32_t cls);
pf_status pf_profile_get(pf_ctx* ctx, int32_t cls, double* total_ms, int64_t* launches, double* bytes);

/* Autotuner for the FFT tile plans (the paper notes that the parallel-loop
 * tiling was left untuned per architecture, Results, "Improved performance
 * via GPU acceleration").  Every column (y/z) pass kind
 * ("colfft", "stage_invz", "zpass_elastic", "zpass_fwd_ac") has two tile
 * variants (kx columns per work-group; see pf_tuning_get); "colfft" has a
 * third for lines of 128 or more: the variant-1 tile in a persistent
 * work-group whose loader wavefronts fetch the next tile while the others
 * transform the current one.  pf_autotune times each variant `reps` times on
 * this context's own buffers and keeps the fastest; it overwrites the stage
 * derivative arrays (call it between steps, never inside one) and leaves the
 * state untouched.  pf_tuning_set forces a variant (PF_ERR_ARG for one that
 * does not exist for this grid); pf_tuning_ms returns the last timing of a
 * variant (0 if never timed).  pf_tuning_get reports the variant in use,
 * its kx columns per work-group and the first (= last) radix of the z-line
 * plan that kind's kernel runs on this grid.  Kinds are
 * 0 .. pf_tuning_kinds()-1; pf_tuning_name never returns NULL ("" for an
 * invalid kind). */
pf_status pf_autotune(pf_ctx* ctx, int32_t reps);
int32_t pf_tuning_kinds(void);
const char* pf_tuning_name(int32_t kind);
pf_status pf_tuning_get(pf_ctx* ctx, int32_t kind, int32_t* variant, int32_t* tile_cols,
                        int32_t* end_radix, double* ms_v0, double* ms_v1);
pf_status pf_tuning_set(pf_ctx* ctx, int32_t kind, int32_t variant);
pf_status pf_tuning_ms(pf_ctx* ctx, int32_t kind, int32_t variant, double* ms);

/* ---- Batched ensembles (many independent simulations of uneven sizes) ----
 * Ensembles of simulations are the use the paper points faster runs at
 * (Discussion: uncertainty quantification over many runs).
 * n members, each with its own pf_params (cubic grids of 32, 48, 64, 96 or
 * 128 points; one embedded method (PF_ARK2, PF_ARK324L or PF_ARK436L), one
 * precision and one adaptivity setting for all; norm_space 0).  Every pass of the stage cycle is one launch covering all members;
 * accept / reject and the next step size are decided on the device per
 * member; one attempted step of all members is captured once as a hipGraph
 * and replayed.  stream: a hipStream_t or NULL (then the ensemble creates its
 * own non-blocking stream).  Errors as for pf_init. */
typedef struct pf_ens pf_ens;
pf_status pf_ensemble_init(int32_t n, const pf_params* per_member, void* stream, pf_ens** out);
void pf_ensemble_finalize(pf_ens* ens);
int32_t pf_ensemble_size_supported(int32_t n);
int64_t pf_ensemble_workspace_bytes(const pf_ens* ens);
int64_t pf_ensemble_kspace_pitch(const pf_ens* ens, int32_t member);
/* Per-member state access, as pf_set_state / pf_get_state / pf_get_state_hat /
 * pf_diagnostics / pf_free_energy on member m (0-based; PF_ERR_ARG out of
 * range); set_state resets the member's time, step size (dt0), controller
 * memory and counters. */
pf_status pf_ensemble_set_state(pf_ens* ens, int32_t m, const double* c, const double* eta,
                                int32_t on_device, double t0);
pf_status pf_ensemble_get_state(pf_ens* ens, int32_t m, double* c, double* eta, int32_t on_device);
pf_status pf_ensemble_get_state_hat(pf_ens* ens, int32_t m, void* y_hat_device);
pf_status pf_ensemble_diagnostics(pf_ens* ens, int32_t m, double* mass, double* vf, double* vf_threshold);
pf_status pf_ensemble_free_energy(pf_ens* ens, int32_t m, double* F);
/* Advances every member to its t_final[m] (host array of n values), at most
 * max_steps attempted steps (graph replays), with the step control of
 * pf_advance per member (Eqs. ARK_embedding, wrms_norm, wrms_weights; a
 * later call with larger t_final resumes from each member's proposed step).
 * Fills per_member[n] if non-NULL (counters, step sizes, and each member's
 * mass, F and volume fraction as pf_get_stats).
 * PF_ERR_STEP_FAIL if a member hit max_rejects consecutive rejections,
 * PF_ERR_NONFINITE for a non-finite fixed-step member, PF_ERR_STATE if
 * max_steps ran out first. */
pf_status pf_ensemble_advance(pf_ens* ens, const double* t_final, int32_t max_steps, pf_stats* per_member);
/* Autotuner: for each pass kind, time work-groups of 128 and 256 threads on
 * the whole ensemble and keep the faster (the step graph is re-captured).
 * The stage kind is timed over all stages of one step; ms128 / ms256 from
 * pf_ensemble_tuning_get are per timed launch sequence. */
pf_status pf_ensemble_autotune(pf_ens* ens, int32_t reps);
int32_t pf_ensemble_tuning_kinds(void);
const char* pf_ensemble_tuning_name(int32_t kind);
pf_status pf_ensemble_tuning_get(pf_ens* ens, int32_t kind, int32_t* block_threads, double* ms128,
                                 double* ms256);
pf_status pf_ensemble_tuning_set(pf_ens* ens, int32_t kind, int32_t block_threads);

/* ---- Fourier neural operator surrogate (learned form) --------------------
 * A learned form beside the method (the paper has no learned component; it
 * advances ensemble members where the plain integrator of Methods, "Time
 * integration" would, and that integrator judges it).
 * Maps the real-space state (cin = 4 fields c, eta_1..3 on an n^3 grid,
 * planar [field][z][y][x]) to the state a fixed time later: the network
 * predicts the increment divided by a per-channel scale.  Layers:
 * v0 = x W_lift + b_lift; v_{l+1} = GELU(K_l v_l + v_l W_l + b_l) (the last
 * layer without GELU), K_l = inverse truncated DFT . per-mode complex width x
 * width matrix . forward truncated DFT (kx < modes; ky, kz among the `modes`
 * lowest non-negative and negative frequencies); out = GELU(v_L P1 + c1) P2 + c2.
 * BF16 weights and activations, FP32 accumulation (MFMA), FP32 master
 * weights with Adam.  Parameters are one flat float32 vector in the order
 * W_lift (cin x width), b_lift, per layer {R_re, R_im ([2m][2m][m][width][width]),
 * W (width x width), b}, P1 (width x hidden), c1, P2 (hidden x cout), c2.
 * Constraints: n % 8 == 0, 8 <= n <= 256, width % 4 == 0 (<= 128), modes even,
 * 2 modes <= n, hidden % 8 == 0 (<= 128), cin, cout <= 8. */
typedef struct {
  int32_t n, width, modes, layers, hidden, cin, cout;
} pf_fno_config;
typedef struct pf_fno pf_fno;
/* Creates a network with zero parameters and its device workspace
 * (activations, spectral blocks, gradients, Adam moments) on the current
 * device; hip_stream a hipStream_t or NULL.  Release with pf_fno_destroy
 * (NULL is a no-op).  Errors: PF_ERR_ARG (config outside the constraints),
 * PF_ERR_OOM, PF_ERR_HIP. */
pf_status pf_fno_create(const pf_fno_config* cfg, void* hip_stream, pf_fno** out);
void pf_fno_destroy(pf_fno* f);
/* Number of parameters (0 for NULL). */
int64_t pf_fno_num_params(const pf_fno* f);
/* Host float32 arrays of pf_fno_num_params values (caller-owned); set also
 * resets Adam.  Errors for the calls below: PF_ERR_ARG for NULL pointers,
 * PF_ERR_HIP for a failed HIP call.  Device arrays are caller-owned and
 * ordered on the network's stream. */
pf_status pf_fno_set_params(pf_fno* f, const float* host_params);
pf_status pf_fno_get_params(pf_fno* f, float* host_params);
/* Loads trained weights from a host buffer of `bytes` bytes holding the flat
 * parameter vector (order as above) either as float32 (bytes = 4 x
 * pf_fno_num_params) or as bfloat16 (bytes = 2 x pf_fno_num_params; widened
 * to the float32 master copy exactly).  Resets Adam.  PF_ERR_ARG for any
 * other size or a NULL pointer. */
pf_status pf_fno_load(pf_fno* f, const void* host_weights, size_t bytes);
/* per-channel output scale (cout host floats); the target is (y - x) / scale */
pf_status pf_fno_set_scale(pf_fno* f, const float* host_scale);
/* per-channel input normalisation (cin host floats each): the network sees
 * (x - shift) / scale, formed before rounding to bf16 (default 0 and 1);
 * PF_ERR_ARG for a scale that is not positive and finite */
pf_status pf_fno_set_input_norm(pf_fno* f, const float* host_shift, const float* host_scale);
/* network output for x (device float32 [cin][n^3]) into out (device float32
 * [n^3][cout], point-major) */
pf_status pf_fno_forward(pf_fno* f, const float* x, float* out);
/* forward + mean-squared loss against the target (y - x) / scale (x, y device
 * float32 [cin][n^3]) + backward; gradients are ADDED to the gradient buffer */
pf_status pf_fno_grad(pf_fno* f, const float* x, const float* y, double* loss);
pf_status pf_fno_get_grad(pf_fno* f, float* host_grad);
pf_status pf_fno_zero_grad(pf_fno* f);
/* Adam step with the accumulated gradient times grad_scale; zeroes it */
pf_status pf_fno_adam_step(pf_fno* f, float lr, float beta1, float beta2, float eps, float grad_scale);
/* One training step on a batch: zero the gradient, forward + loss + backward
 * for each of the `batch` pairs (x, y each device float32
 * [batch][cin][n^3], the state and the state a fixed time later), then one
 * Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the gradient averaged
 * over the batch and learning rate lr.  *loss (may be NULL) receives the
 * batch's mean loss before the update.  PF_ERR_ARG for batch < 1, NULL x/y
 * or lr not positive and finite. */
pf_status pf_fno_train_step(pf_fno* f, const float* x, const float* y, int32_t batch, float lr, float* loss);
/* surrogate advance: next = state + scale * net(state), then the mean of c is
 * restored (the composition is conserved); state / next device float64
 * [cin][n^3] (cin == cout); next may equal state */
pf_status pf_fno_apply(pf_fno* f, const double* state, double* next);
/* Work accounting of the network's kernels: with it on, every launch adds its
 * algorithmic bytes (each operand read once and each result written once, at
 * its storage width: BF16 activations and weights, FP32 outputs, gradients
 * and spectra, FP64 states) and flops (2 per multiply-add) to its kind.
 * Kinds, in this order (PF_FNO_KINDS): 0 truncated-DFT GEMMs (k_lm_gemm),
 * 1 channel-mixing GEMMs (k_cm_gemm), 2 weight-gradient reductions
 * (k_wgrad_mfma), 3 their partial sums (k_sum_partials), 4 per-mode mixing
 * (k_mix_*), 5 GELU backward (k_gelu_bwd), 6 elementwise (input packing,
 * loss, Adam, surrogate update, mass reset).  bytes / flops / launches
 * [kinds] (host) receive the totals since the last reset (kinds beyond
 * PF_FNO_KINDS read 0; kinds == 0 reads nothing); then enable = 1 resets the
 * totals and turns the accounting on, enable = 0 resets and turns it off,
 * enable < 0 leaves both.  Host-side only: no device work, no effect on
 * results.  Errors: PF_ERR_ARG (NULL handle or arrays, kinds < 0). */
#define PF_FNO_KINDS 7
pf_status pf_fno_work(pf_fno* f, int32_t enable, double* bytes, double* flops, int64_t* launches, int32_t kinds);
/* pf_fno_apply for `batch` samples at once (states / nexts device float64
 * [batch][cin][n^3]; nexts may equal states): one network pass whose GEMMs
 * run over every sample's points and lines together, so each sample's result
 * is bit-identical to pf_fno_apply's.  The batched activations (about
 * 0.93 GB per 128^3 sample at width 32, hidden 128) are allocated on the
 * first call and grown when a larger batch comes.  Errors: PF_ERR_ARG (batch
 * < 1, NULL, cin != cout), PF_ERR_OOM, PF_ERR_HIP. */
pf_status pf_fno_apply_batch(pf_fno* f, const double* states, double* nexts, int32_t batch);

/* Counters of the checked surrogate advance.  since_check and plain_left are
 * carried between calls: zero the struct before a member's first call and
 * pass the same struct to continue it. */
typedef struct {
  int32_t surrogate;    /* surrogate advances taken */
  int32_t checks;       /* surrogate advances recomputed by the plain solver */
  int32_t fallbacks;    /* checks whose error exceeded the tolerance */
  int32_t plain;        /* advances run by the plain solver after a fallback */
  int32_t since_check;  /* surrogate advances since the last check */
  int32_t plain_left;   /* plain advances still owed after a fallback */
  double err_last;      /* relative L2 error of c at the last check */
  double err_max;       /* largest checked error */
  double ms_surrogate;  /* wall time in surrogate advances */
  double ms_plain;      /* wall time in checks and plain advances */
} pf_fno_stats;

/* Advances one member by n_adv intervals of length delta.  Each interval is
 * one surrogate advance, except that every check_every-th surrogate advance is
 * also recomputed by the plain solver `plain` (pf_advance over delta from the
 * same input, with that context's method, tolerances and step control); if
 * ||c_net - c_plain|| / ||c_plain|| exceeds tol (or is not finite) the plain
 * result replaces it and the next check_every intervals are run by the plain
 * solver.  state: device float64 [4][n^3] (c, eta_1..3), updated in place.
 * plain: a context on the same n^3 grid and device (its state and time are
 * overwritten; its stream must be ordered with the network's).  Synchronous. */
pf_status pf_fno_advance(pf_fno* f, pf_ctx* plain, double* state, int32_t n_adv, double delta,
                         int32_t check_every, double tol, pf_fno_stats* stats);
/* The checked advance inside a batched ensemble: the `count` members listed
 * (0-based, distinct, each on the network's n^3 grid) advance by n_adv
 * intervals of length delta with the rules of pf_fno_advance (every
 * check_every-th surrogate advance of a member recomputed by the plain
 * solver from the same input; above tol the plain result replaces it and the
 * member runs check_every intervals on the plain solver).  Per interval, every
 * listed member goes through ONE batched network pass (pf_fno_apply_batch)
 * and every check and plain interval runs in ONE pf_ensemble_advance of the
 * ensemble's own batched solver (with the ensemble's method, tolerances and
 * step control; members not listed stay where they are).  Each member ends
 * at its starting time plus n_adv delta, keeping its proposed step size.
 * stats[count]: as pf_fno_advance's, carried between calls; ms_surrogate and
 * ms_plain are the whole call's network and plain wall times, the same in
 * every member's entry.  Synchronous.  Errors: PF_ERR_ARG (bad index,
 * duplicate, size mismatch, cin or cout != 4, delta <= 0, check_every < 1,
 * tol < 0), PF_ERR_OOM, PF_ERR_HIP, and the ensemble's own errors. */
pf_status pf_fno_ensemble_advance(pf_fno* f, pf_ens* ens, const int32_t* members, int32_t count, int32_t n_adv,
                                  double delta, int32_t check_every, double tol, pf_fno_stats* stats);
/* ||a - b||_2 / ||b||_2 over n device float64 values (||a - b|| if b == 0),
 * the error measure of the surrogate's checks; ordered on hip_stream (NULL =
 * default); synchronises that stream.  Allocates its partial sums (device
 * and pinned host) per call.  Errors: PF_ERR_ARG (NULL pointer, n < 1),
 * PF_ERR_OOM, PF_ERR_HIP. */
pf_status pf_rel_l2(const double* a, const double* b, int64_t n, void* hip_stream, double* out);
/* For callers that cannot allocate (code under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc): pf_rel_l2 without any allocation.
 * Same arguments, kernel and summation order as pf_rel_l2 (bit-identical
 * result).  Its partial sums (512 pairs, 8 KiB) live in a file-scope device
 * array of the library, one per GPU, held until the process ends; the host
 * copy of the partials is a stack array.  The array's address is looked up
 * once per device on the first call there.  Every call on a GPU shares that
 * GPU's array: calls that overlap on one GPU (other threads or streams) race
 * and must be serialised by the caller.  Accepts 1 <= n <= 2^41 (each
 * thread's partial sum then adds at most 2^24 squares); PF_ERR_ARG beyond
 * that or for NULL pointers, PF_ERR_HIP for a failed HIP call (more than 64
 * devices included).  Synchronises hip_stream. */
pf_status pf_rel_l2_noalloc(const double* a, const double* b, int64_t n, void* hip_stream, double* out);

/* Streaming-bandwidth probe (a measurement aid, not part of the method): on
 * hip_stream (NULL = default) times a device copy of `bytes`, a read-only sum
 * over `bytes`, and a kernel reading eleven arrays of `bytes` and writing one
 * (the shape of the ARK4 update), best of `reps`; returns algorithmic GB/s of
 * each.  Allocates and frees 12 x bytes of device memory; synchronises the
 * stream.  PF_ERR_ARG for bytes < 1 MiB or reps < 1. */
pf_status pf_bandwidth_probe(int64_t bytes, int32_t reps, void* hip_stream, double* copy_gbs, double* read_gbs,
                             double* multi_gbs);

/* Human-readable status name; never NULL. */
const char* pf_status_string(pf_status s);

/* Identifier of the sources the library was built from (a hash over the
 * kernel, runtime and header sources, fixed at build time); never NULL.
 * Bindings compare it with the sources beside them to refuse a stale build. */
const char* pf_build_id(void);

#ifdef __cplusplus
}
#endif

#endif /* PF_H_ */
