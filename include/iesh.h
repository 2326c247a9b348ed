/*
 * iesh.h -- C ABI of the MI355X (gfx950) ensemble engine for independent
 * electron surface hopping (IESH) on discretised Newns-Anderson models.
 *
 * The library advances many independent trajectories by the IESH time step
 * of Gardner et al., "Efficient implementation and performance analysis of
 * the independent electron surface hopping method for dynamics at metal
 * surfaces": per step and trajectory it
 *   (a) diagonalises the one-electron Hamiltonian H(x) (Sec. II.B, Eq.
 *       single_electron_discrete_electronic_hamiltonian),
 *   (b) forms nonadiabatic couplings and Hellmann-Feynman forces (Sec. II.B,
 *       Eq. classical_hamiltonian and the coupling definition after Eq.
 *       electronic_schrodinger_equation),
 *   (c) propagates the N orbitals with the exponential integrator (Sec. II.C,
 *       Eq. exponential_integrator),
 *   (d) evaluates the hop probabilities from Slater-determinant ratios
 *       (Sec. II.B, Eqs. hopping_probability and hopping_rate), samples a
 *       hop, rescales the velocity and completes velocity Verlet.
 *
 * Conventions (atomic units, hbar = 1):
 *   n = M + 1 one-electron states: index 0 is the impurity |d>, 1..M the bath.
 *   Adiabatic orbitals are ordered by ascending energy; the gauge makes the
 *   impurity component of every orbital positive.
 *   D[j][k] = <j| d/dx |k> = (Q^T dH/dx Q)[j][k] / (lambda_k - lambda_j).
 *   The orbital equation of motion is i dc/dt = (diag(lambda) - i v D) c.
 *   g(a -> b) = max(-2 dt v D[b][a] Re W[b][r(a)], 0), W = C S^-1,
 *   S = C[s, :], r(a) the position of a in the sorted occupied set s.
 *   Step order: half kick, drift, orbital propagation with the propagator
 *   frozen at the midpoint geometry and velocity, eigen-solve at the new
 *   geometry, half kick, hop (probabilities from the new orbitals, couplings
 *   and velocity; one uniform per trajectory and step; rows of occupied
 *   orbitals ascending, then targets ascending), rescaling along D[b][a] or
 *   frustration (no change), force refresh after an accepted hop.
 *   Hop uniforms: Philox4x32-10 with counter (step lo, step hi, trajectory,
 *   0) and key (seed lo, seed hi); u = ((w1 << 32 | w0) >> 11) * 2^-53.
 *
 * Ownership and threading: every buffer passed in is owned by the caller and
 * is not retained after the call returns.  A context is used by one host
 * thread at a time.  All device work runs on the stream given at creation
 * (NULL: a stream created and owned by the context).  Functions return IESH_OK or a negative error
 * code; no C++ exception crosses the ABI.  iesh_last_error() describes the
 * last failure on a context.  Numerical failures of single trajectories do
 * not fail a call: they set that trajectory's status word and freeze it.
 */
#ifndef IESH_H
#define IESH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---------------------------------------------------- */
#define IESH_OK 0
#define IESH_EINVAL (-1)   /* invalid argument                               */
#define IESH_ENOMEM (-2)   /* device allocation failed                       */
#define IESH_EDEVICE (-3)  /* HIP runtime / kernel launch error              */
#define IESH_ESTATE (-4)   /* call not valid in the current context state   */
#define IESH_ENOTSUP (-5)  /* combination not supported by the library        */

/* ---- per-trajectory status bits (iesh_traj_status) -------------------- */
#define IESH_TRAJ_OK 0
#define IESH_TRAJ_EXITED 1      /* crossed the exit plane; frozen            */
#define IESH_TRAJ_NONCONV 2     /* secular-equation root did not converge    */
#define IESH_TRAJ_SINGULAR_S 4  /* occupied overlap S singular: hop skipped  */
#define IESH_TRAJ_NONFINITE 8   /* non-finite position or velocity; frozen   */
#define IESH_TRAJ_STEPCAP 16    /* reached run.max_steps; frozen             */

/* ---- enumerations ------------------------------------------------------- */
enum iesh_model_kind {
  /* Double-well model (Sec. III.B): U0 = m w^2 x^2/2,
     U1 = m w^2 (x-g)^2/2 + dG, h = U1 - U0 + eps_d, V_k constant.
     params: [0] omega, [1] g, [2] dG, [3] eps_d.                           */
  IESH_MODEL_HARMONIC = 0,
  /* Desorption / scattering model (Sec. III.C, Eqs. U0, U1, Vk):
     U0 = De (exp(-a(x-x0)) - 1)^2 + c,
     U1 = D1 exp(-2a'(x-x0)) - D2 exp(-a'(x-x0)) + Vinf,
     V_k(x) = Vbar_k [(1-q)/2 (1 - tanh((x - xt)/at)) + q].
     params: [0] De, [1] x0, [2] a, [3] D1, [4] D2, [5] a', [6] Vinf, [7] q,
             [8] at, [9] xt, [10] c, [11] eps_d.                            */
  IESH_MODEL_MORSE_TANH = 1,
  /* Several nuclear coordinates R_1 .. R_D (D = n_dof <= IESH_MAX_DOF), for a
     molecule with internal and surface-normal modes; the functional forms are
     this library's choice (the paper's models are one-dimensional):
       U0(R) = sum_nu D_nu (1 - exp(-a_nu (R_nu - r_nu)))^2,
       h(R)  = U1 - U0 + eps_d = Delta + eps_d + sum_nu g_nu (R_nu - r_nu),
       V_k(R) = Vbar_k f(R),  f(R) = exp(-sum_nu (R_nu - c_nu)^2 / (4 s_nu^2))
     (so Gamma(R) = Gamma f^2 is a Gaussian in R).  params: [0] Delta,
     [1] eps_d; dof: n_dof rows of (mass, D, a, r, g, c, s).               */
  IESH_MODEL_MULTI_DOF = 2,
  /* A one-electron Hamiltonian of any symmetric structure, affine in one
     coordinate: H(x) = H0 + x H1, dH/dx = H1 (the caller's matrices, field
     dense), n = n_bath + 1 <= IESH_DENSE_MAX_N, state 0 the impurity |d>
     for the observables; U0 = m omega^2 (x - x_c)^2 / 2.  Eigenvectors are
     sign-fixed so that their first nonzero component is positive (the
     impurity component unless it vanishes), which is continuous along a
     path as long as no impurity component passes through zero.  Each
     solve starts from the trajectory's previous eigenvectors (every 256th
     step of a trajectory from scratch), so a run resumed from a saved state
     agrees with the uninterrupted run to rounding, not bit for bit.  eps, w,
     Gamma and lead are not used; no bias.  params: [0] omega, [1] x_c.     */
  IESH_MODEL_DENSE = 3
};

enum iesh_precision {
  IESH_FP64 = 0,  /* every step in FP64                                       */
  IESH_MIXED = 1  /* orbitals and propagation in FP32; eigen-solve, overlap
                     inverse, hop probabilities and rescaling in FP64;
                     FP64 Loewdin re-orthonormalisation every lowdin_every   */
};

enum iesh_mem_kind { IESH_MEM_HOST = 0, IESH_MEM_DEVICE = 1 };

enum iesh_bath_kind {
  IESH_BATH_TRAPEZOID = 0,           /* eps_k = a + (k-1)(b-a)/M (App. A)    */
  IESH_BATH_TRAPEZOID_MIDPOINT = 1,  /* eps_k = a + (k-1/2)(b-a)/M           */
  IESH_BATH_GAUSS_LEGENDRE = 2       /* M/2 Gauss-Legendre nodes on [a, eps_f]
                                        and M/2 on [eps_f, b] (App. A)        */
};

enum iesh_band_placement {
  IESH_BAND_CENTRED = 0,  /* the band [mu - W/2, mu + W/2] follows the chemical
                             potential (wide-band limit); Gauss-Legendre split at mu */
  IESH_BAND_FIXED = 1     /* the band stays [-W/2, W/2]; Gauss-Legendre split at mu  */
};

/* ---- descriptors -------------------------------------------------------- */
/* Bath of a workload (iesh_bath). */
typedef struct iesh_bath_desc {
  int32_t kind;       /* enum iesh_bath_kind                                   */
  int32_t M;          /* bath levels over all leads (a multiple of n_leads;
                         Gauss-Legendre needs M / n_leads even)                */
  int32_t n_leads;    /* 1, or 2: two leads on one grid                         */
  int32_t placement;  /* enum iesh_band_placement                               */
  double W;           /* band width > 0                                         */
  double mu;          /* chemical potential (0: the band centred on 0)          */
} iesh_bath_desc;

typedef struct iesh_model_desc {
  int32_t kind;        /* enum iesh_model_kind                                */
  int32_t n_bath;      /* M >= 1; n = M + 1 <= IESH_MAX_STATES                */
  int32_t n_elec;      /* N electrons, 1 <= N <= min(n - 1, IESH_MAX_ELEC)     */
  int32_t n_dof;       /* nuclear coordinates: 1 (0 means 1) except for
                          IESH_MODEL_MULTI_DOF (1 .. IESH_MAX_DOF); all models
                          of a context have the same count                     */
  const double* eps;   /* host, M bath energies, ascending; equal energies are
                          allowed (two leads on one grid): a group of g equal
                          levels has g - 1 eigenstates at that energy with no
                          impurity component and no coupling to any other
                          state, found by deflation (the secular function keeps
                          one pole per distinct energy, with the summed weight) */
  const double* w;     /* host, M quadrature weights > 0 (V_k = sqrt(Gamma w_k / 2 pi)) */
  double mass;         /* nuclear mass > 0 (one coordinate)                   */
  double Gamma;        /* hybridisation Gamma > 0 (Eq. hybridization)          */
  double params[16];   /* model constants, layout per iesh_model_kind         */
  const double* dof;   /* host, IESH_MODEL_MULTI_DOF: n_dof rows of 7 doubles
                          (mass > 0, D, a, r, g, c, s > 0); else unused       */
  const int32_t* lead; /* host, M labels 0 or 1 (two leads), or NULL (one lead).
                          Only iesh_init_thermal with run.bias != 0 reads them */
  const double* dense; /* host, IESH_MODEL_DENSE: H0 then H1, each n x n
                          row-major and symmetric; else unused (NULL)       */
} iesh_model_desc;

typedef struct iesh_run_desc {
  int32_t n_traj;        /* number of trajectories >= 1                        */
  int32_t precision;     /* enum iesh_precision                                 */
  double dt;             /* time step > 0                                       */
  double kT;             /* temperature of the initial Fermi occupations >= 0  */
  uint64_t seed;         /* key of the hop uniforms                             */
  int32_t lowdin_every;  /* IESH_MIXED: re-orthonormalise every L steps (0: never).
                            Each Loewdin step also measures the orthonormality
                            defect ||C^H C - I||_F the period left (before its
                            correction); the exact no-hop bound allows the
                            stored orbitals a defect of max(1e-3, 4 x that
                            measurement) (1e-8 on the FP64 path).  With 0 the
                            defect is never measured, so the mixed path then
                            evaluates the determinant ratios at every step, as
                            with hop_filter_off = 1 (same results, slower)       */
  int32_t record_every;  /* observables every R steps in iesh_run (0: none)    */
  int32_t exit_enabled;  /* freeze trajectories once x > exit_x (coordinate exit_dof) */
  int32_t compact_every; /* iesh_run: every this many steps, move frozen trajectories
                            behind the active ones so that the step kernels visit
                            only active slots (0: never)                         */
  double exit_x;
  int64_t max_steps;     /* freeze a trajectory after this many steps (0: no cap) */
  int32_t elec_substeps; /* electronic sub-steps per nuclear step, 1..64 (0 = 1):
                            sub-step j of S propagates dt/S with the propagator
                            frozen at x_n + (j + 1/2)/S (x_{n+1} - x_n) (Sec. II.C,
                            sub-stepping of the electronic integrator); hop
                            probabilities stay once per nuclear step            */
  int32_t hop_filter_off; /* 1: evaluate the determinant ratios at every step
                            instead of skipping steps whose exact no-hop bound
                            lies below the uniform (same results, slower)     */
  double bias;           /* V: lead 0 at chemical potential mu + V/2, lead 1 at
                            mu - V/2 for the initial occupations (Sec. III.C, an
                            external bias as a shift of the chemical potential);
                            != 0 needs kT > 0 and lead labels in every model    */
  int32_t exit_dof;      /* coordinate compared with exit_x (0 .. n_dof - 1)     */
  int32_t dt_levels;     /* 0: fixed step dt.  K in 1..30: adaptive step (Sec. II.C
                            bounds the step by the hopping probabilities): after
                            each step a trajectory's next step is the largest
                            dt / 2^k, k = 0..K, for which the step's hop-probability
                            total, rescaled to it (g is proportional to the step),
                            stays <= hop_gmax; dt / 2^K when none does.  Each
                            trajectory keeps its own clock (iesh_traj_clock); the
                            hop uniforms still follow the step count           */
  double hop_gmax;       /* threshold of the adaptive step (> 0 when dt_levels > 0) */
  int32_t eig_max_iter;  /* secular iterations per root, 0..128 (0 = 128).  A small
                            cap is a test hook: roots that do not converge set
                            IESH_TRAJ_NONCONV and freeze their trajectory.
                            IESH_MODEL_DENSE: at most this many perturbative
                            updates of a warm eigen-solve (6 when larger) before
                            the Jacobi sweeps take over                        */
  int32_t reserved3;
} iesh_run_desc;

#define IESH_MAX_STATES 336   /* n = M + 1 limit of the library               */
#define IESH_MAX_ELEC 168     /* N limit of the library                       */
#define IESH_MAX_DOF 6        /* nuclear coordinates per trajectory            */
#define IESH_DENSE_MAX_N 96   /* n limit of IESH_MODEL_DENSE (its eigen-solve
                                 keeps the matrix and the rotations in LDS)    */
#define IESH_JACOBI_MAX_N IESH_MAX_STATES  /* order limit of iesh_eigh_batched */
#define IESH_JACOBI_LDS_N 96  /* orders up to this keep the matrix in LDS      */
#define IESH_NOALLOC_SCRATCH_BYTES (64u << 20)  /* fixed device scratch of
                                                   iesh_eigh_batched_noalloc  */

/* Observables written per record and trajectory by iesh_run, in this order. */
#define IESH_OBS_PD_SURF 0   /* sum_{a in s} Q[0][a]^2                         */
#define IESH_OBS_PD_WF 1     /* sum_n |sum_a Q[0][a] C[a][n]|^2                */
#define IESH_OBS_EKIN 2      /* m v^2 / 2                                      */
#define IESH_OBS_EPOT 3      /* U0(x) + sum_{a in s} lambda_a                  */
#define IESH_OBS_ETOT 4
#define IESH_N_OBS 5

/* Hop event record (iesh_events). */
typedef struct iesh_event {
  int64_t step;      /* global step index of the hop attempt                   */
  int32_t traj;
  int32_t a;         /* orbital left (adiabatic index)                         */
  int32_t b;         /* orbital entered                                        */
  int32_t accepted;  /* 1 accepted, 0 frustrated                               */
  double margin;     /* min |cumulative sum - xi| over the sums formed         */
  double g_total;    /* sum of all hop probabilities of this step              */
} iesh_event;

typedef struct iesh_ctx iesh_ctx;

/* ---- lifecycle ------------------------------------------------------------ */

/* Create a context for run->n_traj trajectories.  traj_model[t] in
   [0, n_models) selects the model (bath size class) of trajectory t; NULL
   means every trajectory uses models[0].  Copies every descriptor array.
   hip_stream is a hipStream_t (NULL: the context creates and owns a stream).  Validates: sorted eps,
   w > 0, N within limits, dt > 0, mass > 0, kT >= 0.  Allocates all device
   memory up front. */
int iesh_create(const iesh_model_desc* models, int32_t n_models, const int32_t* traj_model,
                const iesh_run_desc* run, void* hip_stream, iesh_ctx** out);

/* Free everything.  NULL is accepted. */
int iesh_destroy(iesh_ctx* ctx);

/* Bath discretisation of Appendix A on the band [a, b] (eps_f splits the
   Gauss-Legendre halves; M must be even for it).  Writes M energies and
   weights to host arrays.  Pure host computation. */
int iesh_discretize(int32_t kind, int32_t M, double a, double b, double eps_f, double* eps,
                    double* w);

/* Bath levels of a workload (App. A), placed for the chemical potential mu
   (Sec. II.B, the paragraph on the chemical potential): a grid of
   M / n_leads levels on the band of desc->placement by iesh_discretize
   (Gauss-Legendre halves split at mu); with two leads (each coupled with
   Gamma / 2, so that the total hybridisation stays Gamma) every grid level
   is listed twice, lead 0 first, each copy with half its weight.  Writes M
   energies (ascending) and weights, lead labels (may be NULL) and *n_below
   (may be NULL), the number of levels strictly below mu: the electron count
   that fills the bath up to the chemical potential.  Pure host computation;
   IESH_EINVAL for a bad descriptor. */
int iesh_bath(const iesh_bath_desc* desc, double* eps, double* w, int32_t* lead, int32_t* n_below);

/* ---- state ----------------------------------------------------------------
   Layouts (both for host and device buffers):
     x, v   : n_traj blocks of n_dof doubles (the context's coordinate count)
     C      : n_traj blocks; block t holds N_t * n_t complex doubles,
              orbital-major (C[t][j][i] = coefficient of adiabatic state i in
              orbital j), interleaved (re, im); blocks are packed with the
              stride n_max * N_max complex values of the context
              (iesh_query_sizes), i.e. element (t, j, i) sits at complex
              offset t * n_max * N_max + j * n_t + i.
     occ    : n_traj blocks of stride N_max int32, block t holds N_t sorted
              occupied adiabatic indices.
   mem_kind says whether the pointers are host or device (same device as the
   context) memory.  set_state also recomputes the forces and clears status
   words and the hop event log; the step counter is kept.  During a run each
   eigen-solve starts from the trajectory's previous solution, after
   set_state from the uploaded geometry's own, so a run resumed from a saved
   state agrees with the uninterrupted run to rounding, not bit for bit. */
int iesh_set_state(iesh_ctx* ctx, const double* x, const double* v, const double* C,
                   const int32_t* occ, int32_t mem_kind);
int iesh_get_state(iesh_ctx* ctx, double* x, double* v, double* C, int32_t* occ,
                   int32_t mem_kind);

/* Initial state from positions and velocities (host arrays): occupations
   sampled at run.kT over the adiabatic energies at x (fixed N: chemical
   potential by bisection, one uniform per level from Philox stream 1 at
   counter attempt*n + level, accept when exactly N levels are occupied;
   kT = 0 or 4096 failed attempts give the lowest N), orbitals = occupied
   adiabatic unit vectors (Sec. III.C).  With run.bias = V != 0 the
   occupation probability of orbital j is
     q0_j^2 f(lambda_j - mu) + w0_j f(lambda_j - mu - V/2) + w1_j f(lambda_j - mu + V/2),
   w_l = the orbital's weight on the levels of lead l, and mu is found by the
   same bisection. */
int iesh_init_thermal(iesh_ctx* ctx, const double* x, const double* v);

/* Global step counter (the hop-uniform counter of the next step). */
int iesh_set_step(iesh_ctx* ctx, int64_t step);
int iesh_get_step(const iesh_ctx* ctx, int64_t* step);

/* ---- dynamics ------------------------------------------------------------- */

/* One step of every active trajectory; asynchronous on the context stream. */
int iesh_step(iesh_ctx* ctx);

/* n_steps steps (replayed from a captured HIP graph).  If obs_out is not
   NULL and run.record_every > 0, writes floor(n_steps / record_every)
   records of n_traj * IESH_N_OBS doubles (host memory) taken after every
   record_every-th step of this call; a trajectory that is frozen (status
   word with EXITED, NONCONV, NONFINITE or STEPCAP) when a record falls due
   takes no step and gets NaN in that record.  Synchronises before
   returning. */
int iesh_run(iesh_ctx* ctx, int64_t n_steps, double* obs_out);

/* ---- queries ---------------------------------------------------------------- */

/* Hop probabilities at the current state without sampling: for
   trajectories traj0 .. traj0+ntraj-1 (one model class), writes N_t * n_t
   doubles per trajectory (row r = occupied orbital s[r], column b = target
   state; 0 for occupied targets), packed with stride N_max * n_max.
   Couplings and energies are those at the current x, velocity the current v. */
int iesh_hop_probs(iesh_ctx* ctx, int32_t traj0, int32_t ntraj, double* g_out, int32_t mem_kind);

/* Adiabatic energies and impurity amplitudes Q[0][j] > 0 at the current x
   (host arrays, n_t values per trajectory packed with stride n_max). */
int iesh_adiabatic(iesh_ctx* ctx, int32_t traj0, int32_t ntraj, double* lam_out, double* q0_out);

/* Status words (n_traj int32, host). */
int iesh_traj_status(iesh_ctx* ctx, int32_t* status_out);

/* Step clock of every trajectory (host arrays of n_traj, global trajectory
   order; either may be NULL): elapsed time and the step its next step will
   take.  Without an adaptive step, time = steps taken * dt.  Synchronises. */
int iesh_traj_clock(iesh_ctx* ctx, double* time_out, double* dt_out);

/* Copy up to cap hop events (sorted by step, then trajectory) recorded
   since the last set_state / clear into out (host); *count receives the
   number of events that occurred (may exceed cap and IESH_EVENT_CAP).  The
   device log holds IESH_EVENT_CAP events; once more occurred, the events of
   the step in which the log overflowed are dropped as well (which of them
   found a slot depends on the order the work-groups ran in), so the events
   copied are exactly all events of the steps before that one. */
#define IESH_EVENT_CAP (1 << 20)
int iesh_events(iesh_ctx* ctx, iesh_event* out, int64_t cap, int64_t* count);
int iesh_clear_events(iesh_ctx* ctx);

/* Per-trajectory step caps (host array of n_traj, global order; 0: none):
   a trajectory freezes with IESH_TRAJ_STEPCAP once it has taken that many
   steps, in addition to run->max_steps.  Kept until changed; state uploads
   do not reset them. */
int iesh_set_step_caps(iesh_ctx* ctx, const int64_t* caps);

/* Per bath-size class (model index cls), 8 int32 values: number of
   trajectories, live slots (the step kernels visit slots [0, live); the
   others hold frozen trajectories after compaction), n, N, orbital tiles of
   16 columns per propagation work-group (chosen by timing at creation),
   propagation work-groups per trajectory, n rounded up to 16, 0.  Does not
   synchronise. */
int iesh_class_info(const iesh_ctx* ctx, int32_t cls, int32_t* info);

typedef struct iesh_sizes {
  int32_t n_traj, n_models, n_max, N_max;
  int64_t device_bytes;
  int32_t n_dof;  /* nuclear coordinates per trajectory */
  int32_t reserved;
} iesh_sizes;
int iesh_query_sizes(const iesh_ctx* ctx, iesh_sizes* out);

/* ---- measurement ------------------------------------------------------------
   Per-kernel timing: while enabled, every kernel launched by iesh_step,
   iesh_run and the adjoint calls is bracketed by HIP events on the context stream (iesh_run then
   launches eagerly instead of replaying its graph).  Enabling or disabling
   clears the accumulated times and the work counters. */
#define IESH_TIMER_EIG 0     /* eigen-solves, couplings, Chebyshev set-up, Verlet */
#define IESH_TIMER_PROP 1    /* orbital propagation                              */
#define IESH_TIMER_HOP 2     /* hop probabilities, hop, rescaling, observables   */
#define IESH_TIMER_LOWDIN 3  /* Loewdin re-orthonormalisation (mixed path)       */
#define IESH_TIMER_FILTER 4  /* exact no-hop bound that skips the ratio kernel    */
/* adjoint calls (iesh_adjoint_forward / _backward):                          */
#define IESH_TIMER_ADJ_PROP 5  /* propagations: forward, recompute, Chebyshev and
                                  adjoint Clenshaw vectors                     */
#define IESH_TIMER_ADJ_PHI 6   /* contraction of the adjoint and Chebyshev vectors */
#define IESH_TIMER_ADJ_EIG 7   /* eigen-solves and their reverse, loss terms    */
#define IESH_TIMER_ADJ_HOP 8   /* hop-probability term and its reverse          */
#define IESH_N_TIMERS 9
int iesh_timing(iesh_ctx* ctx, int32_t enable);
/* Milliseconds and launch counts per timer (host arrays of IESH_N_TIMERS)
   since the last read; synchronises. */
int iesh_timing_read(iesh_ctx* ctx, double* ms, int64_t* launches);
/* Algorithmic work since iesh_timing was last called: the number of
   Chebyshev terms summed over all propagated trajectory-steps (one
   propagation of a trajectory costs 4 K n^2 N real flops for K terms) and
   the number of trajectory-steps. */
int iesh_work(iesh_ctx* ctx, int64_t* sum_cheb_terms, int64_t* traj_steps);
/* The same two sums for the trajectories of one bath-size class (model index
   cls), for per-class work: one propagation of a trajectory of that class
   costs 4 K n^2 N real flops with its own n and N. */
int iesh_class_work(iesh_ctx* ctx, int32_t cls, int64_t* sum_cheb_terms, int64_t* traj_steps);

/* Trajectory-steps since iesh_timing was last called whose hop
   probabilities had to be evaluated from the determinant ratios (the others
   were completed by the exact no-hop bound); synchronises. */
int iesh_hop_evals(iesh_ctx* ctx, int64_t* full_evals);

/* Orthonormality defect of the mixed path's FP32 orbitals, as measured by the
   Loewdin steps (run.lowdin_every): per_traj (host, n_traj, global order, may
   be NULL) receives ||C^H C - I||_F of each trajectory before its last
   correction (0 before the first, and on FP64 contexts); max_seen (may be
   NULL) the largest measurement since the last set_state / init_thermal;
   violations (may be NULL) the number of measurements that exceeded the
   defect the exact no-hop bound allowed over the period before them (the
   allowance is max(1e-3, 4 x the previous measurement)): a nonzero count
   means the bound may have skipped a hop in those periods.  Synchronises. */
int iesh_orthonormality_defect(iesh_ctx* ctx, double* per_traj, double* max_seen,
                               int64_t* violations);

/* ---- adjoint along prescribed nuclear paths -------------------------------
   Reverse-mode gradient of an electronic loss with respect to the model
   parameters, for trajectories whose nuclear path x_0 .. x_T is given.  The
   orbitals start as the N lowest adiabatic states at x_0 and follow the
   orbital equation of motion above (Sec. II.C, Eq. exponential_integrator),
   with the propagator frozen at the midpoint (x_n + x_{n+1}) / 2 and the
   velocity (x_{n+1} - x_n) / dt over step n; no hops (the occupations stay
   n0).  Loss of trajectory t with term weights terms = (c_P, c_E, c_G, c_F):
     L_t = c_P (1/T) sum_{s=1..T} P(s) + c_E E_exc(T) + c_G (1/T) sum_s G(s)
           + c_F (1/T) sum_s F(s),
     P(s) = sum_o |sum_a q0_a(x_s) C_ao(s)|^2   (impurity population, Sec. III.B),
     E_exc = sum_a lambda_a(x_T) (rho_a - n0_a), rho_a = sum_o |C_ao(T)|^2,
     G(s) = sum over occupied a, unoccupied b of the hop probabilities
            g_ab = max(-2 dt v_s D_ba Re W_b,r(a), 0) (Eqs. hopping_probability
            and hopping_rate, W = C_U S^-1), v_s = (x_s - x_{s-1}) / dt,
     F(s) = -dU0/dx(x_s) - h' sum_{a in n0} q0_a(x_s)^2 (Hellmann-Feynman
            force, Eq. classical_hamiltonian).
   A singular S at some step drops that step's G term (value and gradient).  Gradients are exact for the discrete
   propagation (Chebyshev series, Sec. II.C) with the series centre and
   radius held fixed.  Supported: IESH_FP64 contexts whose models are all
   IESH_MODEL_HARMONIC.  Parameter layout of one gradient row (model of the
   trajectory, M bath levels): [eps_d, Gamma, eps_1 .. eps_M, omega, g, dG];
   the bath weights w and the mass are constants.

   iesh_adjoint_forward: path (host) [n_traj][n_steps + 1] positions;
   n_steps >= 1; the orbitals are stored every ckpt_every steps (>= 1) and
   recomputed inside each segment by the backward pass (device memory of the
   segment buffer: (ckpt_every + 1) copies of the orbitals).  terms (host, 4
   doubles) or NULL for (1, 1, 0, 0).  loss_out (host, n_traj, may be NULL)
   receives L_t.  Replaces the ensemble state (positions
   follow the path, v is set from it, occupations n0) and releases the
   buffers of any earlier forward pass.  IESH_ENOTSUP for unsupported
   contexts, IESH_EINVAL for a non-finite path.

   iesh_adjoint_backward: dloss (host, n_traj) weights w_t; grad_out (host)
   [n_traj][n_max + 4] receives w_t dL_t/dtheta in the first M_t + 5 entries
   of row t (the rest zero).  May be called again with other weights;
   IESH_ESTATE before a forward pass.  Both calls synchronise. */
int iesh_adjoint_forward(iesh_ctx* ctx, const double* path, int32_t n_steps, int32_t ckpt_every,
                         const double* terms, double* loss_out);
int iesh_adjoint_backward(iesh_ctx* ctx, const double* dloss, double* grad_out);

/* Wait for all work on the context stream; reports asynchronous errors. */
int iesh_sync(iesh_ctx* ctx);

/* ---- dense eigen-solver ------------------------------------------------------
   Eigen-decomposition of `batch` general dense symmetric matrices of order n
   (1 <= n <= IESH_JACOBI_MAX_N): the fallback for a one-electron Hamiltonian
   that is not an arrowhead (Eq. single_electron_discrete_electronic_hamiltonian
   for H of any structure).  Cyclic two-sided Jacobi rotations, FP64, one
   work-group per matrix with the matrix in LDS up to IESH_JACOBI_LDS_N, in a
   device workspace beyond (2 m (m + 1) doubles per matrix, m = n rounded up to
   even; the call allocates it, waits for the kernel and frees it).
     H      : batch x n x n row-major (only symmetric input is meaningful)
     lam    : batch x n eigenvalues, ascending
     Q      : batch x n x n row-major, column j = eigenvector of lam[j]; the
              first component above 1e-12 of the column's largest is positive
     sweeps : batch int32 sweeps used (-1: not converged in 60 sweeps), or NULL
   mem_kind: IESH_MEM_HOST (the call copies, runs and synchronises) or
   IESH_MEM_DEVICE (pointers on the current device; asynchronous on
   hip_stream, NULL = the null stream).  Argument errors return IESH_EINVAL
   before any device call; iesh_last_error(NULL) gives the reason. */
int iesh_eigh_batched(const double* H, int32_t n, int32_t batch, double* lam, double* Q,
                      int32_t* sweeps, int32_t mem_kind, void* hip_stream);

/* The same decomposition for callers that cannot allocate device memory
   (code under HIP graph capture, tight serving loops, harnesses that forbid
   hipMalloc): calls no hipMalloc, hipFree or allocating library routine.
   The work space of orders above IESH_JACOBI_LDS_N comes from a fixed array
   of IESH_NOALLOC_SCRATCH_BYTES in device memory that each GPU the library
   runs on holds until the process ends; a batch whose work space
   (2 m (m + 1) doubles per matrix, m = n rounded up to even) exceeds it is
   rejected with IESH_EINVAL (split it), before any device call.  Every call
   on one GPU shares that array: calls that overlap on one GPU (other streams
   or host threads) race, calls on one stream are ordered by it.
     H, lam, Q, sweeps : device pointers on the current device, layouts as in
                         iesh_eigh_batched (sweeps may be NULL)
     hip_stream        : hipStream_t (NULL = the null stream); the call only
                         enqueues the kernel and does not synchronise.
   Argument errors return IESH_EINVAL, launch errors IESH_EDEVICE;
   iesh_last_error(NULL) gives the reason. */
int iesh_eigh_batched_noalloc(const double* H, int32_t n, int32_t batch, double* lam, double* Q,
                              int32_t* sweeps, void* hip_stream);

/* Description of the last failure on ctx; with ctx = NULL, the reason the
   last context-free call (iesh_create, iesh_eigh_batched) on the calling
   thread failed.  iesh_create checks every
   argument before its first device call, so argument errors (IESH_EINVAL)
   are reported without touching a GPU. */
const char* iesh_last_error(const iesh_ctx* ctx);
int iesh_version(int* major, int* minor, int* patch);

#ifdef __cplusplus
}
#endif
#endif /* IESH_H */
