/*
 * tsph.h -- C ABI of the MI355X (gfx950) Tree+SPH per-step force engine.
 *
 * The library evaluates, for one time-step of a self-gravitating gas + dark
 * matter particle system, the quantities of EvoL's force pass (Merlin et al.,
 * "EvoL: the new Padova T-SPH parallel code for cosmological simulations -
 * I", arXiv:0912.1786):
 *
 *   - the Barnes-Hut oct-tree over Morton-sorted particles with monopole and
 *     quadrupole node moments (Sect. 2.2) and the Dubinski opening test
 *     (Eq. opcrit);
 *   - the self-consistent smoothing length h of gas particles and softening
 *     length eps of all particles from eta = h n^(1/3) (Sect. 2.1 Eqs. rho0,
 *     etan, iter; Sect. 3 Eqs. hn, nsum; Sect. 3.2), with the mass density,
 *     the grad-h terms Omega*, zeta (Eq. drhodr) and the softening terms
 *     Upsilon, xi (Eq. zeta);
 *   - the gravitational acceleration with the symmetrised spline-softened
 *     near field and its adaptive-softening correction terms (Eq. dLgravdr,
 *     App. B);
 *   - the variable-mass SPH acceleration and heating with Monaghan-Gingold
 *     viscosity (Eqs. motionvarmass, thermalvarmass, mu_visc; App. B);
 *   - the kick-drift-kick leapfrog with predicted velocities (Sect. 4.1), the
 *     global time-step criteria (Sect. 4.2) and energy/momentum diagnostics.
 *
 * Conventions
 *   - Units with G = params.G (1 by default).
 *   - Particles are in *caller order*; gas particles are indices [0, n_gas),
 *     every per-particle array has n entries (entries of the non-gas
 *     particles in gas-only arrays are ignored on input and written as 0).
 *   - Every pointer inside tsph_state is a DEVICE pointer to FP64 data owned
 *     by the caller.  The library never frees or reallocates them.
 *   - A context owns all scratch memory (keys, permutation, nodes, lists,
 *     flags), sized once by tsph_create for capacity_n particles.  No
 *     compute call allocates memory.
 *   - A context is used from one host thread and one stream at a time.
 *     Separate contexts may run concurrently on separate streams.
 *   - Stream arguments are hipStream_t values passed as void* (NULL = the
 *     default stream).  Calls enqueue work and return; they do not wait for
 *     the device except where stated.
 *   - No C++ exception crosses the ABI.  Errors are returned as tsph_status;
 *     tsph_last_error gives the text of the last failure on a context.
 *   - Device-side conditions (list overflow, non-convergence, non-finite
 *     values) set bits in a device flag word that tsph_read_flags returns.
 */
#ifndef TSPH_H
#define TSPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TSPH_OK = 0,
  TSPH_EINVAL = -1,     /* invalid argument (null pointer, size, parameter)   */
  TSPH_ENOMEM = -2,     /* device allocation failed in tsph_create            */
  TSPH_EHIP = -3,       /* a HIP runtime call failed                          */
  TSPH_ECAPACITY = -4,  /* n exceeds the context capacity                     */
  TSPH_ENOCONV = -5,    /* a length solve did not converge (tsph_read_flags)  */
  TSPH_EOVERFLOW = -6   /* a device list or the node array overflowed        */
} tsph_status;

enum { TSPH_SOFT_ADAPTIVE = 0,        /* eps solved, correction terms on (Sect. 2.1) */
       TSPH_SOFT_CONSTANT = 1,        /* eps given by the caller, no corrections     */
       TSPH_SOFT_ADAPTIVE_NOCORR = 2  /* eps solved, correction terms off            */ };
/* Arithmetic of the walks (Sect. 2.2 gravity, Sect. 3 SPH).  TSPH_FP32_BULK
 * evaluates the gravity interactions (far nodes and particle pairs) in single
 * precision on coordinates taken relative to the walk batch's centre, and the
 * SPH force pairs in single precision on the double-precision displacement
 * rounded once; single-precision sums per staged tile of at most 64
 * interactions are carried into double-precision totals.  Positions,
 * velocities, node centres of mass, the walks' acceptance and neighbour
 * tests (so the interaction sets are the FP64 form's), the length solves and
 * densities, the integrator and the diagnostics stay FP64. */
enum { TSPH_FP64 = 0, TSPH_FP32_BULK = 1 };
enum { TSPH_KD_FIRST = 0, TSPH_KD_SECOND = 1 };

/* device flag bits */
#define TSPH_FLAG_NODE_CAPACITY 0x1u  /* tree needed more nodes than reserved        */
#define TSPH_FLAG_STACK_OVERFLOW 0x2u /* a walk stack overflowed (result invalid)    */
#define TSPH_FLAG_LIST_OVERFLOW 0x4u  /* a candidate list overflowed (result invalid) */
#define TSPH_FLAG_NOCONV 0x8u         /* an h/eps solve did not converge             */
#define TSPH_FLAG_NONFINITE 0x10u     /* a non-finite input position or mass, or a   *
                                       * constant softening length that is not > 0  *
                                       * (results invalid)                          */
#define TSPH_FLAG_INTERNAL 0x20u      /* an internal index check failed (bug)        */
/* The work-item store of the near-field hand-off (split_leaves) ran out: some
 * walk batches evaluated their whole gravity near field or SPH candidate set
 * themselves.  The results stay valid, but their last bits then depend on
 * which batches got items first (not bitwise reproducible from run to run). */
#define TSPH_FLAG_HANDOFF_CAPACITY 0x40u
/* A periodic box too small for the kernels: some smoothing or softening
 * reach 2h or 2eps is at least half the box side, where the nearest images
 * no longer hold a particle's whole kernel (results invalid). */
#define TSPH_FLAG_PERIOD 0x80u

typedef struct {
  double G;            /* gravitational constant                               */
  double theta;        /* opening parameter; 0 opens every node (direct sum)   */
  int32_t quadrupole;  /* 1: far nodes carry quadrupoles (Sect. 2.2)           */
  int32_t soft_mode;   /* TSPH_SOFT_*                                          */
  double eta_h;        /* h = eta_h n_gas^(-1/3)  (N_nei = 4 pi/3 (2 eta)^3)   */
  double eta_eps;      /* eps = eta_eps n_all^(-1/3)                           */
  double gamma;        /* adiabatic index, P = (gamma - 1) rho u               */
  double alpha, beta;  /* viscosity coefficients (Sect. 3.3)                   */
  double av_eps2;      /* eta^2 = av_eps2 * hbar^2 in mu_ij (0.01)             */
  int32_t tc92;        /* 1: Thomas & Couchman gradient in the SPH pairs       */
  int32_t h_maxit;     /* Newton iterations per solve                          */
  double h_tol;        /* stop when |dh| < h_tol * h_start                      */
  double kappa;        /* candidate search radius 2 h_guess (1 + kappa); a    *
                        * margin that saves walks when h grows (the results  *
                        * do not depend on it)                               */
  int32_t leaf_size;   /* particles per tree leaf (1..64)                      */
  int32_t group_size;  /* sinks per walk group (leaf_size..64)                 */
  int32_t precision;   /* TSPH_FP64 or TSPH_FP32_BULK                           */
  int32_t gravity;     /* 1: self-gravity on                                   */
  int32_t hydro;       /* 1: SPH on                                            */
  int32_t split_leaves; /* load balance (0: off).  A walk batch evaluates at
                          * most this many opened leaves of its gravity near
                          * field itself; the rest go, in work items of 64 to
                          * 127 leaves, to other wavefronts and are summed back
                          * in a fixed order.  A batch whose density candidates
                          * span more leaves (or overflow the on-chip list) is
                          * solved one sink per wavefront, the lanes sharing
                          * the sink's candidates.  An SPH batch evaluates a
                          * quarter of that many candidate particles itself
                          * and hands its further leaves on in the same way
                          * as the gravity near field.                        */
  double eta_dt;       /* time-step coefficient of the Sect. 4.2 criteria      */
  int32_t max_members; /* independent systems one context can hold
                          * (tsph_set_members); 1 by default                  */
  int32_t grav_corr_literal; /* 1: the correction terms with the mass weighting
                          * printed in Sect. 2.1 (Eq. zeta sums d phi/d eps
                          * without masses; Eq. dLgravdr weights both terms of
                          * a pair by m_j); 0 (default): the weighting that
                          * makes the force the gradient of the softened
                          * Lagrangian for unequal masses (the two agree for
                          * equal masses)                                     */
  int32_t soften_cells;  /* 1: softened cells (Sect. 2.2): a node that passes
                          * the opening test but lies within the softening
                          * reach 2 max(eps) acts as one softened particle at
                          * its centre of mass, with the mass-weighted mean
                          * eps of its particles and their correction terms
                          * gathered there, instead of being opened; 0
                          * (default): such nodes are opened down to exact
                          * particle pairs                                    */
  /* scheme variants (Sect. 3 to 3.5) */
  int32_t visc_form;   /* TSPH_VISC_MG: Monaghan-Gingold (Eq. mu_visc);
                          TSPH_VISC_SIGNAL: signal velocity, Pi_ij = -alpha
                          v_sig w_ij / rhobar with w_ij = v_ij . x_ij / r and
                          v_sig = 2 cbar - w_ij (Eqs. pvsig, vsig)            */
  int32_t entropy;     /* 1: the state's u holds the entropic function
                          A = P / rho^gamma and dudt its rate, the viscous
                          term of Eq. SPHentr; P = A rho^gamma              */
  double xsph_eta;     /* X-SPH (Eq. xsph): gas particles drift with
                          v + eta sum_j m_j (v_j - v_i) Wbar_ij / rhobar_ij,
                          Wbar the mean of W(r, h_i) and W(r, h_j), taken from
                          the last force pass; 0 (default): plain drift     */
  int32_t h_scheme;    /* TSPH_H_LAGRANGIAN (default): eta = h n^(1/3) with
                          the grad-h terms; TSPH_H_STANDARD: h puts a fixed
                          number N = 4 pi/3 (2 eta_h)^3 (rounded) of gas
                          particles, the sink included, inside 2h (2h midway
                          between the N-th and the next larger distance;
                          equal distances are taken whole), no grad-h terms  */
  int32_t h_weight;    /* density that sets h: TSPH_HW_NUMBER (default,
                          Eq. nsum) or TSPH_HW_MASS (Eq. densitySPH: a
                          neighbour counts m_j / m_i; the grad-h factor is
                          then 1 / Omega_i with Omega_i = 1 + h/(3 rho)
                          sum m dW/dh).  The mass form is taken with
                          TSPH_H_LAGRANGIAN only (TSPH_EINVAL otherwise).
                          rho is Eq. densitySPH in every scheme              */
  /* dissipation switches (Sect. 3.3.1, 3.3.2); each needs the state's
   * alpha / alpha_u arrays where noted */
  int32_t balsara;     /* 1: Pi_ij times (f_i + f_j)/2, f = |div v| / (|div v|
                          + |curl v| + 1e-4 c/h), the curl from the h kernel
                          normalised as the divergence                      */
  int32_t alpha_switch;/* 1: per-particle alpha (state alpha, gas): the pair
                          mean replaces alpha in Pi_ij (both forms) and in the
                          Courant criterion; d alpha/dt = -(alpha -
                          alpha_min)/tau + 0.75 f max(0, -div v) with
                          tau = h / (0.1 v_sig) (Eq. alphaswitch)             */
  int32_t conduction;  /* 1: artificial conductivity: du_i += sum_j m_j Pi^u_ij
                          |Gbar_ij|, Pi^u_ij = -alphabar^u v^u_sig (u_i - u_j)
                          / rhobar, v^u_sig = sqrt(|P_i - P_j| / rhobar), with
                          per-particle alpha_u (state alpha_u, gas),
                          d alpha_u/dt = -(alpha_u - alpha_u_min)/tau + h
                          |lap u| / sqrt(u) (Brookshaw's Laplacian).  Not
                          with entropy (TSPH_EINVAL)                         */
  double alpha_min;    /* floor of alpha (0.01)                               */
  double alpha_u_min;  /* floor of alpha_u (0)                                */
  double period;       /* > 0: periodic box [0, period)^3 (Sect. 4.3).  The
                          positions are taken modulo the side (and wrapped by
                          the drifts); every pair, node and opening test uses
                          the nearest image (SPH included: no ghosts); gravity
                          adds per particle and per accepted node the Ewald
                          correction of the replicas (omega = 2/L, |n|, |h| <
                          5), tabulated on the device for 32 intervals per half
                          box and interpolated trilinearly.  The potential
                          gets no correction.  0: open boundaries          */
} tsph_params;
enum { TSPH_VISC_MG = 0, TSPH_VISC_SIGNAL = 1 };
enum { TSPH_H_LAGRANGIAN = 0, TSPH_H_STANDARD = 1 };
enum { TSPH_HW_NUMBER = 0, TSPH_HW_MASS = 1 };

typedef struct {
  int64_t n, n_gas;
  /* integrator state (FP64, written only by tsph_kick_drift) */
  double *x, *y, *z;
  double *vx, *vy, *vz;
  double *m;
  double *u;                 /* specific internal energy (gas entries)         */
  /* predicted end-of-step velocity and energy used by the forces (Sect. 4.1);
   * written by tsph_kick_drift(TSPH_KD_FIRST); for the first evaluation the
   * caller copies v and u here */
  double *vpx, *vpy, *vpz, *up;
  /* lengths: in = guess (<= 0: cold start; constant eps in TSPH_SOFT_CONSTANT),
   * out = solved value; carried along the drift by tsph_kick_drift */
  double *h, *eps;
  /* outputs */
  double *ax, *ay, *az;      /* total acceleration                              */
  double *dudt;              /* du/dt (gas)                                     */
  double *rho;               /* SPH mass density (gas)                          */
  double *pot;               /* potential per unit mass; may be NULL            */
  /* dissipation coefficients (gas entries; integrator state advanced by
   * tsph_kick_drift with the rates of the last force pass, kept at or above
   * alpha_min / alpha_u_min); required with alpha_switch / conduction, read
   * by balsara-only passes if given, else NULL */
  double *alpha, *alpha_u;
} tsph_state;

/* Create a context on the current HIP device for up to capacity_n particles.
 * Allocates every scratch buffer once.  *out receives the context. */
tsph_status tsph_create(void **out, int64_t capacity_n, const tsph_params *p);
tsph_status tsph_destroy(void *ctx);
/* Replace the parameters (same capacity). */
tsph_status tsph_set_params(void *ctx, const tsph_params *p);
/* Fill p with the defaults: G=1, theta=0.5, quadrupoles, adaptive softening,
 * 50 neighbours, gamma=5/3, alpha=1, beta=2, av_eps2=0.01, TC92 on,
 * h_tol=1e-10, kappa=0.02, leaf 16, group 64, eta_dt=0.1, split_leaves 256,
 * max_members 1. */
void tsph_default_params(tsph_params *p);
/* Device bytes a context of this capacity reserves (host-only, no GPU).  The
 * arena is laid out per particle for any mix of species (gas records are
 * reserved for every particle), so that one context -- a pooled serving
 * shell, an ensemble -- can hold systems of any gas fraction up to its
 * capacity; the gas count therefore does not enter. */
tsph_status tsph_bytes_required(int64_t capacity_n, const tsph_params *p, size_t *bytes);

/* Several independent systems in one context (an ensemble advanced by the
 * same calls).  The state then holds them back to back: system k owns
 * particles [off[k], off[k+1]) with its gas first, [off[k], off[k] + n_gas[k]);
 * the state's n and n_gas must equal off[count] and the sum of n_gas, or the
 * calls fail with TSPH_EINVAL.  Each system gets its own root cube and tree
 * (the trees form one forest: one sort segmented by system, one walk launch
 * over the walk batches of all of them), its own neighbour sets and its own
 * time-step; nothing couples two systems, so each system's results are those
 * it would get in a context of its own with the same parameters, as long as
 * that context would take the same kernel form: the form follows the whole
 * context (gas present, all particles gas).  off and n_gas are host arrays
 * (count + 1 and count entries) copied by the call; count must not exceed
 * max_members; every system needs at least one particle.  count = 1 returns
 * to the single-system default, in which a state of any size is taken.
 * Synchronous (not for a captured stream). */
tsph_status tsph_set_members(void *ctx, int32_t count, const int64_t *off, const int64_t *n_gas);

/* Root cube, Morton keys, radix sort, gather into key order, canonical
 * oct-tree in level order and node moments (Sect. 2.2). */
tsph_status tsph_build_tree(void *ctx, const tsph_state *s, void *stream);
/* Full force pass: tree, h/eps solves and densities, gravity walk, SPH
 * forces.  Reads x, v^p, u^p, m, h, eps; writes h, eps, a, dudt, rho, pot. */
tsph_status tsph_compute_forces(void *ctx, tsph_state *s, void *stream);
/* Leapfrog half steps (Sect. 4.1).  TSPH_KD_FIRST: v^p = v + dt a,
 * u^p = u + dt du/dt, then v += dt/2 a, x += dt v, u += dt/2 du/dt; when
 * the last tsph_compute_forces on this context had the same n, the positive
 * lengths h (gas) and eps follow the drift through the continuity equation
 * (Sect. 2.1: h n^(1/3) = eta, dn/dt = -n div v): h *= 1 + dt/3 div v, with
 * div v from that evaluation (h kernel for h, eps kernel for eps) and the
 * factor clamped to [1/2, 2].  They are starting values for the next solve.
 * TSPH_KD_SECOND: v += dt/2 a, u += dt/2 du/dt. */
tsph_status tsph_kick_drift(void *ctx, tsph_state *s, double dt, int32_t phase, void *stream);
/* The same with dt read on the device from dt_device (one double per
 * system held, e.g. the output of tsph_timestep), so that a captured HIP
 * graph replays with the current time-step.  dt_device must stay valid while the work runs; a
 * negative or non-finite value there makes the kernel do nothing (the
 * state is left unchanged). */
tsph_status tsph_kick_drift_dt(void *ctx, tsph_state *s, const double *dt_device, int32_t phase, void *stream);
/* One leapfrog step of every system the context holds (one, or the members
 * of tsph_set_members), each with its own global time-step, with no host
 * synchronisation: tsph_timestep into dt_device (one double per system,
 * device memory owned by the caller), tsph_kick_drift_dt(TSPH_KD_FIRST),
 * tsph_compute_forces and tsph_kick_drift_dt(TSPH_KD_SECOND) on the stream.
 * Needs a previous force pass on the context (its time-steps and
 * accelerations); enqueues only, so a HIP graph can capture it (a batch of
 * independent simulations advanced by one graph launch per step). */
tsph_status tsph_batch_step(void *ctx, tsph_state *s, double *dt_device, void *stream);

/* The carry of a context from one step to the next: the velocity
 * divergences with which the next drift carries h and eps, the X-SPH
 * velocity correction of that drift, the rates of alpha and alpha_u for the
 * next kicks and the largest |mu_ij| per particle for the Courant criterion
 * (8 n doubles for n particles).  Saving it and
 * loading it into a context (the same or a new one) lets a simulation leave
 * the device between steps and continue bit for bit: after tsph_carry_load
 * the next tsph_timestep / tsph_kick_drift behave as if the force pass had
 * run on that context.  Both are stream-ordered device-to-device copies;
 * save fails with TSPH_EINVAL when the last force pass had a different n.
 * Only for a context holding one system (TSPH_EINVAL otherwise). */
tsph_status tsph_carry_bytes(int64_t n, size_t *bytes);
tsph_status tsph_carry_save(void *ctx, int64_t n, void *dst_device, void *stream);
tsph_status tsph_carry_load(void *ctx, int64_t n, const void *src_device, void *stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * totals of tsph_diagnostics without a context.  No memory is allocated:
 * the partial sums go to a static device buffer of
 * TSPH_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds until
 * the process ends; every call on a GPU shares that GPU's buffer, so calls
 * that overlap on one GPU (other streams, other threads) race and must be
 * serialised by the caller.  count systems lie back to back in the state:
 * system k = particles [off[k], off[k+1]) with its first ngas[k] gas, where
 * off_device (count + 1 int64) and ngas_device (count int64) are DEVICE
 * arrays the host does not read (ranges are clamped to [0, n)); count = 1
 * takes the whole state (s->n particles, the first s->n_gas gas) and
 * ignores the tables.  Writes nine FP64 totals per system to out_device
 * exactly as tsph_diagnostics does (same kernels, same summation order).
 * Errors: TSPH_EINVAL for null pointers or bad sizes, TSPH_ECAPACITY for
 * count > TSPH_NOALLOC_MAX_SYSTEMS, TSPH_EHIP for a failed launch;
 * tsph_noalloc_last_error gives the text (per host thread). */
#define TSPH_NOALLOC_SCRATCH_BYTES (1 << 20)
#define TSPH_NOALLOC_MAX_SYSTEMS 910
tsph_status tsph_diagnostics_noalloc(const tsph_state *s, int32_t count, const int64_t *off_device,
                                     const int64_t *ngas_device, double *out_device, void *stream);
const char *tsph_noalloc_last_error(void);

/* Global time-step (Sect. 4.2): the minimum over particles of
 * eta_dt sqrt(min(eps, h)/|a|) (a non-positive eps, as without gravity, drops
 * out of the min), the Courant criterion
 * eta_dt h / (h |div v| + c + 1.2 (alpha c + beta max_j |mu_ij|)) and
 * eta_dt |u / du/dt|, taken from the state as it stands (call it at the end
 * of a step, after the closing kick and before the next drift: u, c, a,
 * du/dt, h, eps, rho and alpha of the state, div v and max |mu| of the last
 * force pass).  Writes one double per system held to dt_device. */
tsph_status tsph_timestep(void *ctx, const tsph_state *s, double *dt_device, void *stream);

/* Individual power-of-two time-steps (Sect. 4.2.1) of a context holding one
 * system.  Time runs in integer ticks: the largest step dt_max is 2^max_level
 * ticks.  Particle i steps with dt_max / 2^n_i, the largest such step not
 * above its criteria (those of tsph_timestep, n_i <= max_level), shortened to
 * divide the current tick (a longer step only where synchronised).  Each
 * step is a kick-drift-kick leapfrog of the particle's own length; all
 * particles drift to every system time with their half-kicked velocities;
 * the system time advances to the earliest step end, where the particles
 * whose steps end are active.  A force pass evaluates gravity and the SPH
 * sums for the active particles only (walk chunks without an active sink are
 * skipped) and solves the lengths and densities of all gas particles (their
 * neighbours at the current time); inactive particles lend the predicted
 * velocity v_n + a_n (t - t_n) and energy u_n + du_n (t - t_n) of their last
 * synchronised state.  Wake-up (wake = f > 0, a power of two): an active gas
 * particle's step is at most f times the shortest current step among its SPH
 * neighbours (r_ij < 2 max(h_i, h_j)); an inactive gas particle whose step is
 * longer than f times the shortest criterion step w of its active neighbours
 * ends at the current time plus w, its opening half kick redone for the
 * shorter step from its synchronised state (its drift so far is kept).
 * The caller owns the device arrays (n entries, caller order); the library
 * updates them and the host fields t, n_active, n_woken. */
typedef struct {
  double dt_max;          /* largest step (> 0)                                  */
  int32_t max_level;      /* dt_max = 2^max_level ticks, 0..30                   */
  int32_t wake;           /* wake-up factor f: 0 (off) or a power of two <= 64   */
  int64_t t;              /* host: system time in ticks, in [0, 2^max_level);     *
                           * 0 at every synchronisation point                    */
  int64_t n_active;       /* host: particles evaluated by the last call           */
  int64_t n_woken;        /* host: particles woken by the last call               */
  int32_t *t0, *t1;       /* device: step start and end of each particle (ticks)  */
  double *vsx, *vsy, *vsz, *us;  /* device: v and u at the step start            */
} tsph_blocks;
/* First system time (t = 0): every particle active.  Takes x, v, u of the
 * state as the initial condition (v^p = v, u^p = u; h and eps as in
 * tsph_compute_forces), runs a force pass, chooses the steps (with the
 * wake-up) and gives the opening half kicks.  Synchronous (waits for the
 * stream).  TSPH_EINVAL for missing arrays, a bad dt_max, max_level or wake,
 * or a context holding several systems. */
tsph_status tsph_block_start(void *ctx, tsph_state *s, tsph_blocks *b, void *stream);
/* Advance to the next system time: drift every particle there, evaluate the
 * active ones, close their steps, choose their next steps (wake-up included)
 * and open them.  Synchronous: the earliest step end is read back to the
 * host (b->t, b->n_active and b->n_woken are set on return). */
tsph_status tsph_block_advance(void *ctx, tsph_state *s, tsph_blocks *b, void *stream);
/* FP64 totals: out_device[0..8] = E_kin, E_th, V (= 1/2 sum m pot), Px, Py,
 * Pz, Lx, Ly, Lz; nine per system held (system k at out_device[9k]).
 * Needs s->pot from the last force pass. */
tsph_status tsph_diagnostics(void *ctx, const tsph_state *s, double *out_device, void *stream);
/* Return the OR of the device flag bits since the previous call (then clear
 * them); n_noconv receives the number of unconverged length solves.  The
 * copies and the clearing are ordered on the context's last stream, and the
 * call waits for that stream only (not for the whole device). */
tsph_status tsph_read_flags(void *ctx, uint32_t *flags, int64_t *n_noconv);
/* The same flag bits and unconverged count without waiting: dst[0] receives
 * the flag word and dst[1] the count (uint32 each), then both are cleared,
 * all ordered on `stream`.  dst is device memory or pinned host memory that
 * the caller reads once the stream has passed this point.  For callers that
 * must not block, such as a serving loop moving a simulation off the device;
 * the stream must follow the work whose flags are taken (or that work must
 * be complete).  TSPH_EINVAL for a NULL dst. */
tsph_status tsph_take_flags_async(void *ctx, uint32_t *dst, void *stream);

/* Per-phase timing with HIP events recorded on the stream of each
 * tsph_compute_forces call: phase 0 tree build, 1 length solves and
 * densities, 2 gravity walk, 3 SPH forces, 4 output scatter and time-step.
 * tsph_timing(ctx, 1) creates the events and resets the totals (allocates;
 * not for captured streams); tsph_phase_times waits for the recorded calls
 * and returns the summed milliseconds per phase and the number of calls. */
tsph_status tsph_timing(void *ctx, int32_t enable);
tsph_status tsph_phase_times(void *ctx, double *ms_out /* [5] */, int64_t *calls);

/* Machine probes for the roofline denominators; they measure the machine,
 * not an operation of the paper.  TSPH_PROBE_FMA32 / TSPH_PROBE_FMA64:
 * 4096 x 256 threads each run n rounds (1 <= n <= 2^20) of 8 independent
 * FMA chains in FP32 / FP64, compiled as the walk kernels are (packed FP32
 * off); *work = the flops executed; a is one device double that is never
 * written in practice (it keeps the chains alive).  TSPH_PROBE_TRIAD:
 * a[i] = b[i] + 0.5 c[i] for i < n over caller-owned device arrays of n
 * doubles; *work = 24 n bytes moved.  Enqueued on stream (NULL: the default
 * stream) and asynchronous: time it with events on that stream.  TSPH_EINVAL
 * for an unknown kind, a bad n or a null pointer; TSPH_EHIP if the launch
 * fails. */
enum { TSPH_PROBE_FMA32 = 0, TSPH_PROBE_FMA64 = 1, TSPH_PROBE_TRIAD = 2 };
tsph_status tsph_probe(int32_t kind, int64_t n, double *a, const double *b, const double *c, void *stream,
                       double *work);

/* Debug exports (synchronous copies to host memory, for the tests). */
enum { TSPH_DBG_KEYS = 0,      /* uint64[n] sorted Morton keys                         */
       TSPH_DBG_PERM = 1,      /* int32[n] sorted position -> caller index             */
       TSPH_DBG_NODES = 2,     /* int32[7][nnodes] level, first, count, child, nchild,  *
                                * parent, ngas                                          */
       TSPH_DBG_NNODES = 3,    /* int64[1] node count                                  */
       TSPH_DBG_MOMENTS = 4,   /* double[16][nnodes] mass, com(3), quad(6), bmin(3),    *
                                * bmax(3)                                               */
       TSPH_DBG_GROUPS = 5,    /* int32[ngroups] group nodes                           */
       TSPH_DBG_NGROUPS = 6,   /* int64[1]                                             */
       TSPH_DBG_COUNTS = 7,    /* int32[3][n] (caller order) far nodes, near pairs,    *
                                * SPH pairs per particle in the last force pass        */
       TSPH_DBG_NBR = 8,       /* int32[3][n][max] neighbour lists, see below          */
       TSPH_DBG_ROOT = 9,      /* double[4] x0, y0, z0, side (of the first system)     */
       TSPH_DBG_SOLVE = 10,    /* double[19][n] (caller order) nh, omega, zeta, divv,  *
                                * neps, ups, xi, maxmu, divv with the eps kernel,       *
                                * largest signal velocity, viscous heating, X-SPH sum  *
                                * (3, without eta), curl (3), Balsara factor, lap u     */
       TSPH_DBG_BATCHES = 11,  /* int32[nbatches][2] walk batches: group-list ranges   *
                                * [g0, g1) of consecutive sibling groups packed to <= 64 */
       TSPH_DBG_NBATCHES = 12  /* int64[1]                                             */ };
/* Enable per-particle neighbour-list recording (up to max_per_particle
 * entries per particle and kind: density gather r < 2h_i, SPH pairs
 * r < 2max(h_i,h_j), gravity-correction pairs r < 2max(eps_i,eps_j)); lists
 * hold caller indices in the order found, padded with -1; a longer list sets
 * TSPH_FLAG_LIST_OVERFLOW.  max_per_particle = 0 disables.  Allocates. */
tsph_status tsph_debug_lists(void *ctx, int32_t max_per_particle);
tsph_status tsph_debug_export(void *ctx, int32_t what, void *host, size_t cap_bytes,
                              size_t *written);

/* Limit the near-field hand-off (tsph_params.split_leaves) of the following
 * force passes to at most `items` work items (0: the context's full store),
 * so that tests can exhaust it on small inputs; exhaustion raises
 * TSPH_FLAG_HANDOFF_CAPACITY.  Host-only, takes effect at the next call. */
tsph_status tsph_debug_handoff_cap(void *ctx, int64_t items);

const char *tsph_last_error(const void *ctx);
const char *tsph_version(void);
/* Identity of the sources the library was built from: the first 16 hex
 * digits of a SHA-256 over the HIP sources and this header (the binding
 * refuses a library whose identity differs from the sources beside it). */
const char *tsph_source_id(void);

#ifdef __cplusplus
}
#endif
#endif
