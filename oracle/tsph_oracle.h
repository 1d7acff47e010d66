/*
 * tsph_oracle.h -- FP64 CPU oracle for the Tree+SPH per-step force evaluation
 * of EvoL (Merlin et al., "EvoL: the new Padova T-SPH parallel code for
 * cosmological simulations - I").
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, obviously-correct CPU
 * implementation used by the test-suite, by the smoke check and by the CPU
 * baseline leg of the benchmark.  The product path (the HIP library) never
 * links, loads or calls it, and it shares no code, header, table or constant
 * generator with that path.
 *
 * Every floating-point quantity is FP64.  The library must be compiled with
 * -ffp-contract=off so that the neighbour and opening predicates are evaluated
 * with exactly one rounding per operation, in the stated order.
 *
 * Parity status per function is listed in the header comment of
 * tsph_oracle.c.
 */
#ifndef TSPH_ORACLE_H
#define TSPH_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- kernel functions (Sect. 2.1, Sect. 3, App. A/B) -------------------- */
double orc_w(double u);                 /* spline shape w(u), W = w/(pi h^3)      */
double orc_dw(double u);                /* dw/du                                   */
double orc_W(double r, double h);
double orc_dWdr(double r, double h);
double orc_dWdh(double r, double h);
double orc_dWdr_tc92(double r, double h);   /* Thomas & Couchman gradient       */
double orc_phi(double r, double eps);       /* softened potential kernel (<0)   */
double orc_dphidr(double r, double eps);    /* softened force kernel            */
double orc_dphideps(double r, double eps);  /* d phi / d eps at fixed r         */

/* ---- parameters ---------------------------------------------------------- */
enum { ORC_SOFT_ADAPTIVE = 0, ORC_SOFT_CONSTANT = 1, ORC_SOFT_ADAPTIVE_NOCORR = 2 };
enum { ORC_WALK_PARTICLE = 0, ORC_WALK_GROUP = 1, ORC_WALK_DIRECT = 2 };
enum { ORC_NBR_TREE = 0, ORC_NBR_BRUTE = 1 };

typedef struct {
  double G, theta;
  int32_t quadrupole;
  int32_t soft_mode;
  double eta_h, eta_eps;        /* eps = eta n^(-1/3), h = eta n^(-1/3)        */
  double gamma, alpha, beta;    /* EoS and artificial viscosity                 */
  double av_eps2;               /* eta^2 / hbar^2 in mu_ij (0.01)               */
  int32_t tc92;                 /* modified kernel gradient in the SPH pairs   */
  int32_t h_maxit;
  double h_tol, kappa;          /* Newton tolerance; search-radius margin      */
  int32_t leaf_size, group_size;
  int32_t walk_mode, nbr_mode;
  int32_t gravity, hydro;       /* switches (1 = on)                            */
  int32_t batch_size;           /* walk batches: groups packed up to this size  */
  int32_t batch_mode;           /* 0: siblings only, 1: any consecutive groups  */
  int32_t grav_corr_literal;    /* correction terms with the printed mass
                                 * weighting of Eqs. dLgravdr, zeta            */
  int32_t soften_cells;         /* softened cells (Sect. 2.2): a node that
                                 * passes the opening test but lies within the
                                 * softening reach acts as one softened
                                 * particle at its centre of mass              */
  /* scheme variants (Sect. 3, 3.3.1, 3.4, 3.5) */
  int32_t visc_form;            /* ORC_VISC_MG (Eq. mu_visc) or ORC_VISC_SIGNAL
                                 * (Eqs. pvsig, vsig)                          */
  int32_t entropy;              /* 1: the energy variable is the entropic
                                 * function A = P / rho^gamma (Eq. SPHentr)    */
  double xsph_eta;              /* X-SPH velocity smoothing (Eq. xsph); 0: off */
  int32_t h_scheme;             /* ORC_H_LAGRANGIAN (eta = h n^(1/3)) or
                                 * ORC_H_STANDARD (a fixed neighbour count, no
                                 * grad-h terms)                               */
  int32_t h_weight;             /* the density that sets h (Sect. 3, the four
                                 * schemes of the mixed-mass test): ORC_HW_NUMBER
                                 * (number density, Eq. nsum; every neighbour
                                 * counts 1) or ORC_HW_MASS (mass density,
                                 * Eq. densitySPH; neighbour j counts
                                 * m_j / m_i).  rho is Eq. densitySPH either way */
  /* dissipation switches (Sect. 3.3.1, 3.3.2) */
  int32_t balsara;              /* Pi_ij times (f_i + f_j)/2, the Balsara limiter */
  int32_t alpha_switch;         /* per-particle alpha (Eq. alphaswitch)         */
  double alpha_min;             /* its floor (0.01)                             */
  int32_t conduction;           /* artificial thermal conductivity              */
  double alpha_u_min;           /* floor of the conductivity coefficient (0)    */
  /* periodic box [0, L)^3 of side period (0: open), Sect. 4.3: positions are
   * taken modulo L, every pair and node interaction uses the nearest image,
   * and gravity adds the Ewald correction of the replicas, tabulated for
   * omega = 2/L, |n|, |h| < 5, on a grid of ORC_EWALD_GRID intervals per
   * half box and interpolated trilinearly (the potential gets no correction) */
  double period;
} orc_params;
#define ORC_EWALD_GRID 32
enum { ORC_VISC_MG = 0, ORC_VISC_SIGNAL = 1 };
enum { ORC_H_LAGRANGIAN = 0, ORC_H_STANDARD = 1 };
enum { ORC_HW_NUMBER = 0, ORC_HW_MASS = 1 };

/* All arrays are in caller order, length n unless noted.  Gas particles are
 * the indices [0, n_gas).  Output arrays may be NULL when not wanted.       */
typedef struct {
  int64_t n, n_gas;
  const double *x, *y, *z;
  const double *vx, *vy, *vz;   /* velocities used in the forces (predicted)    */
  const double *m;
  const double *u;              /* specific internal energy (predicted), gas     */
  const double *h_in;           /* smoothing-length guesses (<=0: cold start)   */
  const double *eps_in;         /* softening guesses, or the constant values    */
  /* outputs */
  double *h, *nh, *rho, *omega, *zeta, *divv;      /* gas solve                  */
  double *eps, *neps, *ups, *xi;                   /* softening solve            */
  double *ax, *ay, *az, *pot, *dudt, *maxmu;       /* forces                     */
  int64_t *cnt_node, *cnt_pair, *cnt_sph;          /* interaction counts         */
  int32_t *iters;                                  /* Newton passes per particle */
  int64_t n_noconv;                                /* out: unsolved lengths      */
  /* optional sink sample (caller indices): when n_sinks > 0 the gravity and
   * SPH passes run for these sinks only (any walk mode; the batch walk visits
   * only the batches holding a sampled sink); the
   * length solves still cover every particle */
  const int64_t *sinks;
  int64_t n_sinks;
  int64_t *cnt_soft;                               /* near pairs inside 2 max(eps) */
  double *divv_eps;                                /* div v with the eps kernel    */
  double t_phase[4];   /* out: wall seconds of tree, length solves + densities,
                        * gravity and SPH (instrumentation only)              */
  double *xsph_x, *xsph_y, *xsph_z;  /* X-SPH velocity correction (gas)       */
  double *vsig;                      /* max over pairs of the signal velocity  */
  /* dissipation switches: per-particle coefficients in (gas), their rates,
   * the velocity curl (h kernel), the Balsara factor and the Laplacian of u */
  const double *alpha_in, *alpha_u_in;
  double *dalpha, *dalpha_u, *curlx, *curly, *curlz, *fbal, *lapu;
} orc_run;

/* Full force evaluation: tree, h/eps solves, gravity walk, SPH forces.
 * Returns 0 on success, <0 on invalid arguments or allocation failure.     */
int orc_compute_forces(const orc_params *p, orc_run *r);

/* ---- tree (exported for the topology tests) ------------------------------ */
typedef struct orc_tree orc_tree;
orc_tree *orc_tree_build(int64_t n, const double *x, const double *y, const double *z,
                         const double *m, int32_t leaf_size);
void orc_tree_free(orc_tree *t);
int64_t orc_tree_nnodes(const orc_tree *t);
/* root cube: x0[3], log2 side; sorted keys and permutation (sorted -> caller) */
void orc_tree_root(const orc_tree *t, double *x0, int32_t *e);
void orc_tree_keys(const orc_tree *t, uint64_t *keys, int64_t *perm);
void orc_tree_nodes(const orc_tree *t, int32_t *level, uint64_t *prefix, int64_t *first,
                    int64_t *count, int64_t *child, int32_t *nchild, int64_t *parent);
void orc_tree_moments(const orc_tree *t, double *mass, double *com, double *quad,
                      double *centre, double *side, double *delta, double *bmin, double *bmax);
/* groups: maximal nodes holding at most group_size particles, by first particle */
int64_t orc_tree_groups(const orc_tree *t, int32_t group_size, int64_t *group_node);
/* walk batches: runs of consecutive groups (mode 0: consecutive children of
 * one parent only) packed greedily up to batch_size particles; ranges
 * [g0, g1) of the group list */
int64_t orc_tree_batches(const orc_tree *t, int32_t group_size, int32_t batch_size, int32_t mode, int64_t *g0,
                         int64_t *g1);

/* ---- neighbour sets (bit-exact list tests) ---------------------------------
 * kind 0: density gather  {j in gas : r_ij < 2 h_i}, sinks = gas
 * kind 1: SPH force       {j in gas, j != i : r_ij < 2 max(h_i, h_j)}, sinks = gas
 * kind 2: gravity terms   {j, j != i : r_ij < 2 max(eps_i, eps_j)}, sinks = all
 * offsets has n+1 entries (entries for non-sinks are empty); idx receives
 * caller indices in ascending order.  Returns the total count, or -1 if it
 * exceeds cap (offsets are still filled).                                   */
int64_t orc_neighbours(int kind, int mode, int64_t n, int64_t n_gas, const double *x,
                       const double *y, const double *z, const double *len, int32_t leaf_size,
                       int64_t *offsets, int64_t *idx, int64_t cap, double period);

/* ---- Ewald correction (Sect. 4.3) ---------------------------------------------
 * acc[3] = the acceleration per unit mass of the replicas of a unit mass at
 * displacement x (x = the evaluation point minus the mass, |x_k| <= L/2):
 * the Ewald sums over |n| < 5 and 0 < |h| < 5 (integer triplets, Euclidean
 * norms) with splitting parameter omega, minus the direct term -x/|x|^3;
 * zero at x = 0.  orc_ewald_interp: the same from the tabulated grid
 * (omega = 2/L) by trilinear interpolation on |x_k| with the sign of x_k. */
void orc_ewald_exact(double x, double y, double z, double L, double omega, double *acc);
void orc_ewald_interp(double x, double y, double z, double L, double *acc);

/* ---- direct sums, integrator and diagnostics ------------------------------ */
/* V = (G/2) sum_i sum_j m_i m_j phi(r_ij, eps_i), self terms included        */
double orc_potential_energy(int64_t n, const double *x, const double *y, const double *z,
                            const double *m, const double *eps, double G);
/* kick-drift-kick leapfrog; phase 0 = K1/2 + D (+ predicted v, u, and the
 * lengths h (gas) and eps (all) carried along the drift by the continuity
 * equation, h <- h (1 + dt/3 div v) clamped to [1/2, 2], when h / divv_h or
 * eps / divv_e are given), 1 = K1/2 */
void orc_kick_drift(int64_t n, int64_t n_gas, double dt, int32_t phase,
                    double *x, double *y, double *z, double *vx, double *vy, double *vz,
                    double *u, const double *ax, const double *ay, const double *az,
                    const double *dudt, double *vpx, double *vpy, double *vpz, double *up,
                    double *h, double *eps, const double *divv_h, const double *divv_e,
                    const double *xsx, const double *xsy, const double *xsz,
                    double *alpha, const double *dalpha, double alpha_min,
                    double *alpha_u, const double *dalpha_u, double alpha_u_min,
                    double period /* > 0: positions wrapped into [0, period) */);
double orc_timestep(const orc_params *p, int64_t n, int64_t n_gas, const double *vx,
                    const double *vy, const double *vz, const double *u, const double *h,
                    const double *eps, const double *ax, const double *ay, const double *az,
                    const double *dudt, const double *divv, const double *maxmu, double eta_dt,
                    const double *rho /* entropy form: c from A and rho */,
                    const double *alpha /* per-particle alpha, or NULL */);
/* the same criteria per particle into dt_out (INFINITY where none applies) */
double orc_timestep_each(const orc_params *p, int64_t n, int64_t n_gas, const double *vx,
                         const double *vy, const double *vz, const double *u, const double *h,
                         const double *eps, const double *ax, const double *ay, const double *az,
                         const double *dudt, const double *divv, const double *maxmu, double eta_dt,
                         const double *rho, const double *alpha, double *dt_out);
/* out[9] = E_kin, E_th, V, Px, Py, Pz, Lx, Ly, Lz (V from pot: 0.5 sum m pot) */
void orc_diagnostics(int64_t n, int64_t n_gas, const double *x, const double *y, const double *z,
                     const double *vx, const double *vy, const double *vz, const double *m,
                     const double *u, const double *pot, double *out,
                     const double *rho, double gamma, int32_t entropy /* E_th from A and rho */);

void orc_multipole_field(int64_t n, const double *x, const double *y, const double *z,
                         const double *m, double px, double py, double pz, int32_t quadrupole,
                         double *acc, double *pot);
int orc_num_threads(void);
void orc_eval_kernel(int which, int64_t n, const double *r, const double *h, double *out);

#ifdef __cplusplus
}
#endif
#endif
