/*
 * tsph_oracle.c -- FP64 CPU oracle (TEST INFRASTRUCTURE ONLY; see the header).
 *
 * Source of every formula: Merlin et al., "EvoL: the new Padova T-SPH parallel
 * code for cosmological simulations - I" (arXiv:0912.1786).  Section and
 * equation labels below are the paper's.  Where the printed text is garbled or
 * silent the adopted reading is named at the point of use; the full list of
 * readings is kept with the design notes of the repository.
 *
 * Parity status (what pins each part, in tests/test_oracle_*.py):
 *   kernels          closed-form values, continuity, integral of W, finite
 *                    differences of each derivative                  pinned
 *   keys/tree        independent prefix enumeration, partition invariants
 *                                                                     pinned
 *   h / eps solve    lattice self-consistency, brute-force neighbours,
 *                    monotonicity, eps-N_nei relation                 pinned
 *   gravity          theta = 0 equals the O(N^2) sum, quadrupole error order,
 *                    Plummer potential and field, finite differences of the
 *                    softened Lagrangian (correction terms), momentum pinned
 *   SPH forces       finite differences of the thermal energy at fixed
 *                    entropy, exact dE/dt = 0 identity, momentum      pinned
 *   walk batches     defining properties of the greedy sibling packing
 *                    (partition, siblings, size, forced cuts)        pinned
 *   integrator       energy drift scaling with dt^2                   pinned
 *   timestep rule    each criterion of Sect. 4.2 deciding in turn on
 *                    hand-worked values; minimum over particles       pinned
 *   diagnostics      rigid rotation + drift: P = M V, L = M R x V + I w,
 *                    E_kin from the inertia tensor                    pinned
 *   scheme variants  signal-velocity viscosity conserves momentum and
 *                    energy; entropy rate = rescaled viscous heating;
 *                    X-SPH carries no momentum; standard scheme counts
 *                    exactly N; four-scheme mixed-mass lattice        pinned
 *   switches         curl of a rigid rotation, Balsara limits, alpha
 *                    rate closed forms, conduction conserves energy   pinned
 *   periodic box     Ewald sums independent of omega, small-x and
 *                    symmetry limits, table = sums on its grid; lattice
 *                    at rest, translation invariance, nearest-image
 *                    neighbours by brute force                        pinned
 *   (the individual time-steps, oracle/blocksteps.py, are pinned there)
 *
 * Plain loops, no blocking or fusion; OpenMP only distributes independent
 * sinks over threads.
 */
#include "tsph_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXLEVEL 21

/* ===================================================================== */
/* Kernel functions                                                       */
/* ===================================================================== */

/* Cubic spline density kernel, Sect. 2.1 Eq. (spline): W = w(u)/(pi h^3),
 * support 2h.  The printed normalisation writes h for the softening kernel;
 * it is read as 1/(pi eps^3) there (the same shape with the kernel's own
 * length). */
double orc_w(double u)
{
  if (u < 1.0) return 1.0 - 1.5 * u * u + 0.75 * u * u * u;
  if (u < 2.0) { double t = 2.0 - u; return 0.25 * t * t * t; }
  return 0.0;
}

double orc_dw(double u)
{
  if (u < 1.0) return -3.0 * u + 2.25 * u * u;
  if (u < 2.0) { double t = 2.0 - u; return -0.75 * t * t; }
  return 0.0;
}

double orc_W(double r, double h) { return orc_w(r / h) / (M_PI * h * h * h); }

double orc_dWdr(double r, double h) { return orc_dw(r / h) / (M_PI * h * h * h * h); }

/* dW/dh at fixed r = -(3 w + u w')/(pi h^4): chain rule on w(r/h)/(pi h^3). */
double orc_dWdh(double r, double h)
{
  double u = r / h;
  return -(3.0 * orc_w(u) + u * orc_dw(u)) / (M_PI * h * h * h * h);
}

/* Thomas & Couchman (1992) kernel gradient, Sect. 3 footnote to the
 * equations of motion: constant slope inside u < 2/3.  The printed form lacks
 * the 1/h^4 of a 3-D gradient; it is restored here. */
double orc_dWdr_tc92(double r, double h)
{
  double u = r / h, s;
  if (u < 2.0 / 3.0) s = 1.0;
  else if (u < 1.0) s = 0.75 * u * (4.0 - 3.0 * u);
  else if (u < 2.0) { double t = 2.0 - u; s = 0.75 * t * t; }
  else s = 0.0;
  return -s / (M_PI * h * h * h * h);
}

/* Softened potential kernel, Sect. 2.1 Eq. (softphi); phi -> -1/r for u >= 2. */
double orc_phi(double r, double eps)
{
  double u = r / eps;
  if (u < 1.0) {
    double u2 = u * u;
    return ((2.0 / 3.0) * u2 - 0.3 * u2 * u2 + 0.1 * u2 * u2 * u - 1.4) / eps;
  }
  if (u < 2.0) {
    double u2 = u * u;
    return ((4.0 / 3.0) * u2 - u2 * u + 0.3 * u2 * u2 - u2 * u2 * u / 30.0 - 1.6 + 1.0 / (15.0 * u)) / eps;
  }
  return -1.0 / r;
}

/* Softened force kernel d phi/d r, Sect. 2.1 Eq. (softforce); 1/r^2 for u >= 2. */
double orc_dphidr(double r, double eps)
{
  double u = r / eps;
  if (u < 1.0) {
    double u2 = u * u;
    return ((4.0 / 3.0) * u - 1.2 * u2 * u + 0.5 * u2 * u2) / (eps * eps);
  }
  if (u < 2.0) {
    double u2 = u * u;
    return ((8.0 / 3.0) * u - 3.0 * u2 + 1.2 * u2 * u - u2 * u2 / 6.0 - 1.0 / (15.0 * u2)) / (eps * eps);
  }
  return 1.0 / (r * r);
}

/* d phi / d eps at fixed r, Sect. 2.1 Eq. (dphidh).  Derived as
 * -(f + u f')/eps^2 from phi = f(u)/eps; in the outer branch this gives
 * -3/2 u^4 where the paper prints +3/2 u^4 (the printed sign makes the
 * function discontinuous at u = 1 and non-zero at u = 2). */
double orc_dphideps(double r, double eps)
{
  double u = r / eps;
  if (u < 1.0) {
    double u2 = u * u;
    return (-2.0 * u2 + 1.5 * u2 * u2 - 0.6 * u2 * u2 * u + 1.4) / (eps * eps);
  }
  if (u < 2.0) {
    double u2 = u * u;
    return (-4.0 * u2 + 4.0 * u2 * u - 1.5 * u2 * u2 + 0.2 * u2 * u2 * u + 1.6) / (eps * eps);
  }
  return 0.0;
}

/* ===================================================================== */
/* Tree: root cube, Morton keys, canonical oct-tree (Sect. 2.2)            */
/* ===================================================================== */

struct orc_tree {
  int64_t n;
  int32_t leaf_size;
  double x0[3];
  int32_t e;                  /* root cube side = 2^e                        */
  uint64_t *keys;             /* sorted keys                                 */
  int64_t *perm;              /* sorted position -> caller index             */
  double *xs, *ys, *zs, *ms;  /* sorted positions, masses                    */
  int64_t nnodes, cap;
  int32_t *level;
  uint64_t *prefix;
  int64_t *first, *count, *child, *parent;
  int32_t *nchild;
  double *mass, *com, *quad, *centre, *side, *delta, *bmin, *bmax;
  int64_t *leaf_of;           /* sorted position -> leaf node                */
};

/* Power-of-two root cube: x0 = component-wise minimum, side = the maximum
 * extent rounded up to a power of two.  The cube subdivision is the
 * hierarchical partition of Sect. 2.2. */
static void root_cube(int64_t n, const double *x, const double *y, const double *z,
                      double *x0, int32_t *e)
{
  double lo[3] = {x[0], y[0], z[0]}, hi[3] = {x[0], y[0], z[0]};
  for (int64_t i = 1; i < n; i++) {
    if (x[i] < lo[0]) lo[0] = x[i];
    if (x[i] > hi[0]) hi[0] = x[i];
    if (y[i] < lo[1]) lo[1] = y[i];
    if (y[i] > hi[1]) hi[1] = y[i];
    if (z[i] < lo[2]) lo[2] = z[i];
    if (z[i] > hi[2]) hi[2] = z[i];
  }
  double L = 0.0;
  for (int d = 0; d < 3; d++) {
    double ext = hi[d] - lo[d];
    if (ext > L) L = ext;
    x0[d] = lo[d];
  }
  if (L > 0.0) {
    int ex;
    double f = frexp(L, &ex); /* L = f 2^ex, f in [0.5, 1) */
    *e = (f == 0.5) ? ex - 1 : ex;
  } else {
    *e = 0;
  }
}

static uint64_t spread3(uint64_t v)
{
  /* put bit b of v at bit 3b, by a plain loop */
  uint64_t r = 0;
  for (int b = 0; b < ORC_MAXLEVEL; b++) r |= ((v >> b) & 1ull) << (3 * b);
  return r;
}

static uint64_t cell_coord(double xv, double x0, double scale)
{
  double c = floor((xv - x0) * scale);
  if (c < 0.0) c = 0.0;
  if (c > 2097151.0) c = 2097151.0;
  return (uint64_t)c;
}

typedef struct { uint64_t key; int64_t idx; } key_idx;

static int keyidx_cmp(const void *a, const void *b)
{
  const key_idx *p = (const key_idx *)a, *q = (const key_idx *)b;
  if (p->key < q->key) return -1;
  if (p->key > q->key) return 1;
  return (p->idx < q->idx) ? -1 : (p->idx > q->idx);
}

static int tree_push(orc_tree *t, int32_t level, uint64_t prefix, int64_t first, int64_t count,
                     int64_t parent)
{
  if (t->nnodes == t->cap) {
    int64_t nc = t->cap ? 2 * t->cap : 1024;
    t->level = realloc(t->level, nc * sizeof(int32_t));
    t->prefix = realloc(t->prefix, nc * sizeof(uint64_t));
    t->first = realloc(t->first, nc * sizeof(int64_t));
    t->count = realloc(t->count, nc * sizeof(int64_t));
    t->child = realloc(t->child, nc * sizeof(int64_t));
    t->parent = realloc(t->parent, nc * sizeof(int64_t));
    t->nchild = realloc(t->nchild, nc * sizeof(int32_t));
    if (!t->level || !t->prefix || !t->first || !t->count || !t->child || !t->parent || !t->nchild)
      return -1;
    t->cap = nc;
  }
  int64_t k = t->nnodes++;
  t->level[k] = level;
  t->prefix[k] = prefix;
  t->first[k] = first;
  t->count[k] = count;
  t->child[k] = -1;
  t->nchild[k] = 0;
  t->parent[k] = parent;
  return 0;
}

void orc_tree_free(orc_tree *t)
{
  if (!t) return;
  free(t->keys); free(t->perm); free(t->xs); free(t->ys); free(t->zs); free(t->ms);
  free(t->level); free(t->prefix); free(t->first); free(t->count); free(t->child);
  free(t->parent); free(t->nchild);
  free(t->mass); free(t->com); free(t->quad); free(t->centre); free(t->side); free(t->delta);
  free(t->bmin); free(t->bmax); free(t->leaf_of);
  free(t);
}

static void tree_moments(orc_tree *t)
{
  int64_t nn = t->nnodes;
  t->mass = calloc(nn, sizeof(double));
  t->com = calloc(3 * nn, sizeof(double));
  t->quad = calloc(6 * nn, sizeof(double));
  t->centre = calloc(3 * nn, sizeof(double));
  t->side = calloc(nn, sizeof(double));
  t->delta = calloc(nn, sizeof(double));
  t->bmin = calloc(3 * nn, sizeof(double));
  t->bmax = calloc(3 * nn, sizeof(double));
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t k = 0; k < nn; k++) {
    int64_t f = t->first[k], c = t->count[k];
    /* cube geometry from level and prefix: side 2^(e-L); centre
     * x0 + (2 i + 1) side/2 (one rounding, in the addition) */
    int L = t->level[k];
    double s = ldexp(1.0, t->e - L);
    uint64_t ix = 0, iy = 0, iz = 0;
    for (int b = 0; b < L; b++) {
      uint64_t dgt = (t->prefix[k] >> (3 * b)) & 7ull;
      ix |= ((dgt >> 2) & 1ull) << b;
      iy |= ((dgt >> 1) & 1ull) << b;
      iz |= (dgt & 1ull) << b;
    }
    t->side[k] = s;
    t->centre[3 * k + 0] = t->x0[0] + (double)(2 * ix + 1) * (0.5 * s);
    t->centre[3 * k + 1] = t->x0[1] + (double)(2 * iy + 1) * (0.5 * s);
    t->centre[3 * k + 2] = t->x0[2] + (double)(2 * iz + 1) * (0.5 * s);
    /* monopole, centre of mass (Sect. 2.2), tight bounding box */
    double M = 0, sx = 0, sy = 0, sz = 0;
    double lo[3] = {t->xs[f], t->ys[f], t->zs[f]}, hi[3] = {t->xs[f], t->ys[f], t->zs[f]};
    for (int64_t q = f; q < f + c; q++) {
      M += t->ms[q];
      sx += t->ms[q] * t->xs[q];
      sy += t->ms[q] * t->ys[q];
      sz += t->ms[q] * t->zs[q];
      double p[3] = {t->xs[q], t->ys[q], t->zs[q]};
      for (int d = 0; d < 3; d++) {
        if (p[d] < lo[d]) lo[d] = p[d];
        if (p[d] > hi[d]) hi[d] = p[d];
      }
    }
    double cx = sx / M, cy = sy / M, cz = sz / M;
    t->mass[k] = M;
    t->com[3 * k + 0] = cx;
    t->com[3 * k + 1] = cy;
    t->com[3 * k + 2] = cz;
    for (int d = 0; d < 3; d++) { t->bmin[3 * k + d] = lo[d]; t->bmax[3 * k + d] = hi[d]; }
    /* traceless quadrupole about the centre of mass:
     * Q_ab = sum m (3 d_a d_b - |d|^2 delta_ab), order xx, yy, zz, xy, xz, yz */
    double Q[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t q = f; q < f + c; q++) {
      double dx = t->xs[q] - cx, dy = t->ys[q] - cy, dz = t->zs[q] - cz;
      double d2 = dx * dx + dy * dy + dz * dz, mq = t->ms[q];
      Q[0] += mq * (3 * dx * dx - d2);
      Q[1] += mq * (3 * dy * dy - d2);
      Q[2] += mq * (3 * dz * dz - d2);
      Q[3] += mq * 3 * dx * dy;
      Q[4] += mq * 3 * dx * dz;
      Q[5] += mq * 3 * dy * dz;
    }
    for (int a = 0; a < 6; a++) t->quad[6 * k + a] = Q[a];
    /* Dubinski offset delta = |centre of mass - geometric centre| (Eq. opcrit) */
    double ox = cx - t->centre[3 * k], oy = cy - t->centre[3 * k + 1], oz = cz - t->centre[3 * k + 2];
    t->delta[k] = sqrt(ox * ox + oy * oy + oz * oz);
  }
}

orc_tree *orc_tree_build(int64_t n, const double *x, const double *y, const double *z,
                         const double *m, int32_t leaf_size)
{
  if (n <= 0 || leaf_size < 1) return NULL;
  orc_tree *t = calloc(1, sizeof(orc_tree));
  t->n = n;
  t->leaf_size = leaf_size;
  root_cube(n, x, y, z, t->x0, &t->e);
  double scale = ldexp(1.0, ORC_MAXLEVEL - t->e);
  key_idx *ki = malloc(n * sizeof(key_idx));
  for (int64_t i = 0; i < n; i++) {
    uint64_t cx = cell_coord(x[i], t->x0[0], scale);
    uint64_t cy = cell_coord(y[i], t->x0[1], scale);
    uint64_t cz = cell_coord(z[i], t->x0[2], scale);
    ki[i].key = (spread3(cx) << 2) | (spread3(cy) << 1) | spread3(cz);
    ki[i].idx = i;
  }
  /* stable order by (key, original index) */
  qsort(ki, n, sizeof(key_idx), keyidx_cmp);
  t->keys = malloc(n * sizeof(uint64_t));
  t->perm = malloc(n * sizeof(int64_t));
  t->xs = malloc(n * sizeof(double));
  t->ys = malloc(n * sizeof(double));
  t->zs = malloc(n * sizeof(double));
  t->ms = malloc(n * sizeof(double));
  for (int64_t p = 0; p < n; p++) {
    int64_t i = ki[p].idx;
    t->keys[p] = ki[p].key;
    t->perm[p] = i;
    t->xs[p] = x[i];
    t->ys[p] = y[i];
    t->zs[p] = z[i];
    t->ms[p] = m ? m[i] : 1.0;
  }
  free(ki);
  /* canonical oct-tree in level order: a node is (level, key prefix) with a
   * non-zero count; it is split into its non-empty octants (in octant order)
   * when it holds more than leaf_size particles and is above the finest
   * level.  Processing the queue front to back yields nodes ordered by
   * (level, first particle), children of a node contiguous. */
  tree_push(t, 0, 0, 0, n, -1);
  for (int64_t k = 0; k < t->nnodes; k++) {
    int32_t L = t->level[k];
    if (t->count[k] <= leaf_size || L >= ORC_MAXLEVEL) continue;
    int shift = 3 * (ORC_MAXLEVEL - (L + 1));
    int64_t p = t->first[k], end = t->first[k] + t->count[k];
    int64_t c0 = t->nnodes;
    int32_t nc = 0;
    uint64_t pre = t->prefix[k];
    for (uint64_t oct = 0; oct < 8; oct++) {
      int64_t q = p;
      while (q < end && ((t->keys[q] >> shift) & 7ull) == oct) q++;
      if (q > p) {
        if (tree_push(t, L + 1, (pre << 3) | oct, p, q - p, k) != 0) { orc_tree_free(t); return NULL; }
        nc++;
      }
      p = q;
    }
    t->child[k] = c0;
    t->nchild[k] = nc;
  }
  t->leaf_of = malloc(n * sizeof(int64_t));
  for (int64_t k = 0; k < t->nnodes; k++)
    if (t->nchild[k] == 0)
      for (int64_t q = t->first[k]; q < t->first[k] + t->count[k]; q++) t->leaf_of[q] = k;
  tree_moments(t);
  return t;
}

int64_t orc_tree_nnodes(const orc_tree *t) { return t->nnodes; }

void orc_tree_root(const orc_tree *t, double *x0, int32_t *e)
{
  for (int d = 0; d < 3; d++) x0[d] = t->x0[d];
  *e = t->e;
}

void orc_tree_keys(const orc_tree *t, uint64_t *keys, int64_t *perm)
{
  if (keys) memcpy(keys, t->keys, t->n * sizeof(uint64_t));
  if (perm) memcpy(perm, t->perm, t->n * sizeof(int64_t));
}

void orc_tree_nodes(const orc_tree *t, int32_t *level, uint64_t *prefix, int64_t *first,
                    int64_t *count, int64_t *child, int32_t *nchild, int64_t *parent)
{
  int64_t nn = t->nnodes;
  if (level) memcpy(level, t->level, nn * sizeof(int32_t));
  if (prefix) memcpy(prefix, t->prefix, nn * sizeof(uint64_t));
  if (first) memcpy(first, t->first, nn * sizeof(int64_t));
  if (count) memcpy(count, t->count, nn * sizeof(int64_t));
  if (child) memcpy(child, t->child, nn * sizeof(int64_t));
  if (nchild) memcpy(nchild, t->nchild, nn * sizeof(int32_t));
  if (parent) memcpy(parent, t->parent, nn * sizeof(int64_t));
}

void orc_tree_moments(const orc_tree *t, double *mass, double *com, double *quad, double *centre,
                      double *side, double *delta, double *bmin, double *bmax)
{
  int64_t nn = t->nnodes;
  if (mass) memcpy(mass, t->mass, nn * sizeof(double));
  if (com) memcpy(com, t->com, 3 * nn * sizeof(double));
  if (quad) memcpy(quad, t->quad, 6 * nn * sizeof(double));
  if (centre) memcpy(centre, t->centre, 3 * nn * sizeof(double));
  if (side) memcpy(side, t->side, nn * sizeof(double));
  if (delta) memcpy(delta, t->delta, nn * sizeof(double));
  if (bmin) memcpy(bmin, t->bmin, 3 * nn * sizeof(double));
  if (bmax) memcpy(bmax, t->bmax, 3 * nn * sizeof(double));
}

static int is_group(const orc_tree *t, int64_t k, int32_t G)
{
  int fits = (t->count[k] <= G) || (t->nchild[k] == 0);
  int top = (t->parent[k] < 0) || (t->count[t->parent[k]] > G);
  return fits && top;
}

int64_t orc_tree_groups(const orc_tree *t, int32_t G, int64_t *group_node)
{
  /* walk particle positions: the group containing position p starts there */
  int64_t ng = 0;
  int64_t *start = malloc(t->n * sizeof(int64_t));
  for (int64_t p = 0; p < t->n; p++) start[p] = -1;
  for (int64_t k = 0; k < t->nnodes; k++)
    if (is_group(t, k, G)) start[t->first[k]] = k;
  for (int64_t p = 0; p < t->n; p++)
    if (start[p] >= 0) {
      if (group_node) group_node[ng] = start[p];
      ng++;
    }
  free(start);
  return ng;
}

/* Walk batches: consecutive groups that are consecutive children of the same
 * parent are packed greedily, in octant order, into batches of at most B
 * particles.  A batch is the node range [k0, k1) of its member siblings; its
 * particles are one contiguous range and its box is the union of the
 * members' boxes.  Returns the number of batches. */
int64_t orc_tree_batches(const orc_tree *t, int32_t G, int32_t B, int32_t mode, int64_t *bg0, int64_t *bg1)
{
  /* batches are ranges [g0, g1) of the group list (ordered by first
   * particle); mode 0 packs only consecutive children of one parent, mode 1
   * any consecutive groups */
  int64_t ng = orc_tree_groups(t, G, NULL);
  int64_t *gn = malloc((ng + 1) * sizeof(int64_t));
  orc_tree_groups(t, G, gn);
  int64_t nb = 0, fill = 0;
  for (int64_t i = 0; i < ng; i++) {
    int64_t u = gn[i];
    int join = nb > 0 && fill + t->count[u] <= B;
    if (join && mode == 0) join = (u == gn[i - 1] + 1) && t->parent[u] == t->parent[gn[i - 1]];
    if (join) {
      fill += t->count[u];
      if (bg1) bg1[nb - 1] = i + 1;
    } else {
      fill = t->count[u];
      if (bg0) bg0[nb] = i;
      if (bg1) bg1[nb] = i + 1;
      nb++;
    }
  }
  free(gn);
  return nb;
}

/* ===================================================================== */
/* Geometry predicates (one rounding per operation, fixed order)           */
/* ===================================================================== */

static double sq_axis(double lo, double hi, double p)
{
  double d = 0.0;
  if (p < lo) d = lo - p;
  else if (p > hi) d = p - hi;
  return d * d;
}

/* nearest-image component of a displacement in a periodic box of side L
 * (Sect. 4.3; L = 0: open boundaries) */
static double wrapd(double d, double L)
{
  return L > 0.0 ? d - L * nearbyint(d / L) : d;
}

/* the same gaps on a circle of circumference L: the nearest-image distance
 * of the centres less the half-widths */
static double sq_axis_p(double lo, double hi, double p, double L)
{
  if (!(L > 0.0)) return sq_axis(lo, hi, p);
  double c = 0.5 * (lo + hi), w = 0.5 * (hi - lo);
  double t = fabs(wrapd(p - c, L));
  double d = t > w ? t - w : 0.0;
  return d * d;
}

static double box_point_d2(const double *lo, const double *hi, double px, double py, double pz, double L)
{
  double s = sq_axis_p(lo[0], hi[0], px, L);
  s = s + sq_axis_p(lo[1], hi[1], py, L);
  s = s + sq_axis_p(lo[2], hi[2], pz, L);
  return s;
}

static double gap_axis(double lo1, double hi1, double lo2, double hi2)
{
  double d = 0.0;
  if (hi1 < lo2) d = lo2 - hi1;
  else if (hi2 < lo1) d = lo1 - hi2;
  return d * d;
}

static double gap_axis_p(double lo1, double hi1, double lo2, double hi2, double L)
{
  if (!(L > 0.0)) return gap_axis(lo1, hi1, lo2, hi2);
  double c1 = 0.5 * (lo1 + hi1), w1 = 0.5 * (hi1 - lo1);
  double c2 = 0.5 * (lo2 + hi2), w2 = 0.5 * (hi2 - lo2);
  double d = fabs(wrapd(c2 - c1, L)) - w1 - w2;
  if (!(d > 0.0)) d = 0.0;
  return d * d;
}

static double box_box_d2(const double *lo1, const double *hi1, const double *lo2, const double *hi2, double L)
{
  double s = gap_axis_p(lo1[0], hi1[0], lo2[0], hi2[0], L);
  s = s + gap_axis_p(lo1[1], hi1[1], lo2[1], hi2[1], L);
  s = s + gap_axis_p(lo1[2], hi1[2], lo2[2], hi2[2], L);
  return s;
}

static double pair_r2(double xi, double yi, double zi, double xj, double yj, double zj, double L)
{
  double dx = wrapd(xj - xi, L), dy = wrapd(yj - yi, L), dz = wrapd(zj - zi, L);
  return dx * dx + dy * dy + dz * dz;
}

/* ---- Ewald correction (Sect. 4.3) ---------------------------------------- */

/* The acceleration per unit mass of all replicas of a unit mass at
 * displacement x (evaluation point minus mass), with the direct term
 * -x/|x|^3 taken out: the real-space sum over |n| < 5 with erfc and the
 * Gaussian, and the Fourier sum over 0 < |h| < 5, splitting parameter
 * omega.  Zero at x = 0 (by symmetry). */
void orc_ewald_exact(double x, double y, double z, double L, double omega, double *acc)
{
  acc[0] = acc[1] = acc[2] = 0.0;
  if (x == 0.0 && y == 0.0 && z == 0.0) return;
  double r2 = x * x + y * y + z * z, r = sqrt(r2);
  double ax = x / (r2 * r), ay = y / (r2 * r), az = z / (r2 * r);
  for (int nx = -4; nx <= 4; nx++)
    for (int ny = -4; ny <= 4; ny++)
      for (int nz = -4; nz <= 4; nz++) {
        if (nx * nx + ny * ny + nz * nz >= 25) continue;
        double dx = x - nx * L, dy = y - ny * L, dz = z - nz * L;
        double d2 = dx * dx + dy * dy + dz * dz, d = sqrt(d2);
        double f = (erfc(omega * d) + 2.0 * omega * d / sqrt(M_PI) * exp(-omega * omega * d2)) / (d2 * d);
        ax -= dx * f;
        ay -= dy * f;
        az -= dz * f;
      }
  for (int hx = -4; hx <= 4; hx++)
    for (int hy = -4; hy <= 4; hy++)
      for (int hz = -4; hz <= 4; hz++) {
        int h2 = hx * hx + hy * hy + hz * hz;
        if (h2 == 0 || h2 >= 25) continue;
        double c = 2.0 / (L * L) / h2 * exp(-M_PI * M_PI * h2 / (omega * omega * L * L)) *
                   sin(2.0 * M_PI / L * (hx * x + hy * y + hz * z));
        ax -= c * hx;
        ay -= c * hy;
        az -= c * hz;
      }
  acc[0] = ax;
  acc[1] = ay;
  acc[2] = az;
}

/* Tables of the correction on [0, L/2]^3 for omega = 2/L, ORC_EWALD_GRID
 * intervals per axis, built once per L (a few tables kept) */
#define EW_N ORC_EWALD_GRID
#define EW_KEEP 4
static double ew_L[EW_KEEP];
static double *ew_T[EW_KEEP];
static pthread_mutex_t ew_lock = PTHREAD_MUTEX_INITIALIZER;

static const double *ewald_table(double L)
{
  pthread_mutex_lock(&ew_lock);
  const double *T = NULL;
  for (int k = 0; k < EW_KEEP; k++)
    if (ew_T[k] && ew_L[k] == L) T = ew_T[k];
  if (!T) {
    int slot = 0;
    while (slot < EW_KEEP - 1 && ew_T[slot]) slot++;
    free(ew_T[slot]);
    const int n1 = EW_N + 1;
    double *W = malloc((size_t)3 * n1 * n1 * n1 * sizeof(double));
    double step = 0.5 * L / EW_N;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t a = 0; a < (int64_t)n1 * n1 * n1; a++) {
      int i = (int)(a / (n1 * n1)), j = (int)((a / n1) % n1), k = (int)(a % n1);
      double e[3];
      orc_ewald_exact(i * step, j * step, k * step, L, 2.0 / L, e);
      /* odd in its own coordinate: zero on that coordinate plane */
      W[3 * a + 0] = i == 0 ? 0.0 : e[0];
      W[3 * a + 1] = j == 0 ? 0.0 : e[1];
      W[3 * a + 2] = k == 0 ? 0.0 : e[2];
    }
    ew_T[slot] = W;
    ew_L[slot] = L;
    T = W;
  }
  pthread_mutex_unlock(&ew_lock);
  return T;
}

/* trilinear interpolation on |x_k|, the component taking the sign of x_k
 * (the correction is odd in its own coordinate, even in the others) */
static void ewald_interp(const double *T, double L, double x, double y, double z, double *acc)
{
  const int n1 = EW_N + 1;
  double a[3] = {fabs(x), fabs(y), fabs(z)}, f[3];
  int i[3];
  double step = 0.5 * L / EW_N;
  for (int d = 0; d < 3; d++) {
    double u = a[d] / step;
    int k = (int)floor(u);
    if (k > EW_N - 1) k = EW_N - 1;
    if (k < 0) k = 0;
    i[d] = k;
    f[d] = u - k;
  }
  for (int c = 0; c < 3; c++) {
    double v = 0.0;
    for (int b = 0; b < 8; b++) {
      int ox = b >> 2, oy = (b >> 1) & 1, oz = b & 1;
      double w = (ox ? f[0] : 1.0 - f[0]) * (oy ? f[1] : 1.0 - f[1]) * (oz ? f[2] : 1.0 - f[2]);
      v += w * T[3 * (((int64_t)(i[0] + ox) * n1 + (i[1] + oy)) * n1 + (i[2] + oz)) + c];
    }
    acc[c] = v;
  }
  if (x < 0.0) acc[0] = -acc[0];
  if (y < 0.0) acc[1] = -acc[1];
  if (z < 0.0) acc[2] = -acc[2];
}

void orc_ewald_interp(double x, double y, double z, double L, double *acc)
{
  ewald_interp(ewald_table(L), L, x, y, z, acc);
}

/* ===================================================================== */
/* Force evaluation                                                        */
/* ===================================================================== */

typedef struct {
  const orc_params *p;
  const orc_tree *t;
  int64_t n, n_gas;
  /* sorted-order per-particle data */
  double *vx, *vy, *vz, *u;
  char *gas;
  double *h, *nh, *rho, *omega, *zeta, *divv, *divv_e;
  double *eps, *neps, *ups, *xi;
  double *ax, *ay, *az, *pot, *dudt, *maxmu;
  double *P, *cs;
  double *fa;                 /* grad-h factor f_ij = fa_i + zeta_i / (m_j Omega*_i) */
  double *xsx, *xsy, *xsz, *vsig;  /* X-SPH velocity correction, max signal velocity */
  double *curl, *fbal, *lapu, *alpha, *alpha_u, *dalpha, *dalpha_u;  /* dissipation switches */
  int64_t *cnt_node, *cnt_pair, *cnt_sph, *cnt_soft;
  int32_t *iters;
  int64_t noconv;             /* length solves that did not converge        */
  char *active;               /* sinks of the gravity/SPH passes            */
  /* per-node maxima after the solves */
  double *epsmax, *hmax;
  int64_t *ngas;
  /* per-node softened-cell data: mass-weighted mean eps, sum of m xi/Ups */
  double *epsbar, *xsum;
  /* periodic box side (0: open) and its Ewald table */
  double L;
  const double *ewt;
} ctx_t;

typedef struct {
  int64_t *idx;
  int64_t n, cap;
  int64_t *stack;
} cand_t;

static void cand_add(cand_t *c, int64_t q)
{
  if (c->n == c->cap) {
    c->cap = c->cap ? 2 * c->cap : 256;
    c->idx = realloc(c->idx, c->cap * sizeof(int64_t));
  }
  c->idx[c->n++] = q;
}

/* candidates for sink position p: particles (of the solve's set) within R,
 * found through leaves whose bounding box lies closer than R */
static void collect(const ctx_t *C, int64_t p, double R, int gas_only, cand_t *c)
{
  const orc_tree *t = C->t;
  double R2 = R * R, px = t->xs[p], py = t->ys[p], pz = t->zs[p];
  int64_t sp = 0;
  c->n = 0;
  c->stack[sp++] = 0;
  while (sp > 0) {
    int64_t k = c->stack[--sp];
    if (gas_only && C->ngas[k] == 0) continue;
    if (!(box_point_d2(&t->bmin[3 * k], &t->bmax[3 * k], px, py, pz, C->L) < R2)) continue;
    if (t->nchild[k] == 0) {
      for (int64_t q = t->first[k]; q < t->first[k] + t->count[k]; q++) {
        if (gas_only && !C->gas[q]) continue;
        if (pair_r2(px, py, pz, t->xs[q], t->ys[q], t->zs[q], C->L) < R2) cand_add(c, q);
      }
    } else {
      for (int32_t a = t->nchild[k] - 1; a >= 0; a--) c->stack[sp++] = t->child[k] + a;
    }
  }
}

typedef struct { double n, sdh, rho, msdh, mdphi, divv, dphi, curl[3]; } sums_t;

/* number-density sum and its h-derivative over the candidates, Eqs. (rho0),
 * (nsum); self term included (j = i) */
static sums_t kernel_sums(const ctx_t *C, int64_t p, double h, const cand_t *c, int full, int mode)
{
  const orc_tree *t = C->t;
  sums_t s = {0, 0, 0, 0, 0, 0, 0};
  double px = t->xs[p], py = t->ys[p], pz = t->zs[p];
  for (int64_t a = 0; a < c->n; a++) {
    int64_t q = c->idx[a];
    double r2 = pair_r2(px, py, pz, t->xs[q], t->ys[q], t->zs[q], C->L);
    double r = sqrt(r2);
    if (!(r < 2.0 * h)) continue;
    /* x_i - x_j, the nearest image */
    double ex = wrapd(px - t->xs[q], C->L), ey = wrapd(py - t->ys[q], C->L), ez = wrapd(pz - t->zs[q], C->L);
    double W = orc_W(r, h), dWdh = orc_dWdh(r, h);
    s.n += W;
    s.sdh += dWdh;
    if (full) {
      double mq = t->ms[q];
      if (mode == 0) {
        /* gas: mass density, zeta, velocity divergence */
        s.rho += mq * W;
        s.msdh += mq * dWdh;
        if (r > 0.0) {
          double g = orc_dWdr(r, h) / r; /* grad_i W = g (x_i - x_j) */
          double dvx = C->vx[p] - C->vx[q], dvy = C->vy[p] - C->vy[q], dvz = C->vz[p] - C->vz[q];
          s.divv += g * (dvx * ex + dvy * ey + dvz * ez);
          /* curl: v_ij x grad_i W_ij */
          s.curl[0] += g * (dvy * ez - dvz * ey);
          s.curl[1] += g * (dvz * ex - dvx * ez);
          s.curl[2] += g * (dvx * ey - dvy * ex);
        }
      } else {
        /* softening: mass-weighted d phi / d eps (Eq. zeta), and the
         * velocity divergence with the eps kernel */
        s.mdphi += mq * orc_dphideps(r, h);
        s.dphi += orc_dphideps(r, h);
        if (r > 0.0) {
          double g = orc_dWdr(r, h) / r;
          double dvx = C->vx[p] - C->vx[q], dvy = C->vy[p] - C->vy[q], dvz = C->vz[p] - C->vz[q];
          s.divv += g * (dvx * ex + dvy * ey + dvz * ez);
        }
      }
    }
  }
  return s;
}

/* Self-consistent length for one sink (Sect. 2.1 "iterative method",
 * Eq. (iter); Sect. 3 Eq. (hn)).  The relation eta = h n^(1/3) is solved as
 * g(h) = h^3 n(h) - eta^3 = 0; g is non-decreasing in h (each h^3 W term is),
 * so the root is unique and a bracket is kept.  g'(h) = 3 h^2 n Omega*, the
 * printed f' = -(3 n/h) Upsilon rescaled by -h^3.  Safeguarded Newton
 * steps (below); iteration stops when the Newton step is below tol h, and
 * the result is the last evaluated length with its sums.  Candidates cover
 * r < 2 rc, rc = h (1 + kappa), and are gathered again whenever an iterate
 * exceeds rc (Sect. 3.1, enlarged search radius). */
static int solve_length(const ctx_t *C, int64_t p, int gas_only, int mode, double eta, double guess,
                        int cold, cand_t *c, double *h_out, sums_t *s_out, int32_t *iters)
{
  /* with the mass-density relation every neighbour counts m_j / m_i */
  const int mass_w = mode == 0 && C->p->h_weight == ORC_HW_MASS;
  const double imi = 1.0 / C->t->ms[p];
  const orc_params *P = C->p;
  int64_t set_size = gas_only ? C->n_gas : C->n;
  double eta3 = eta * eta * eta;
  if (!((double)set_size / M_PI > eta3) || !(guess > 0.0)) {
    double h = guess > 0.0 ? guess : 1.0;
    collect(C, p, 2.0 * h, gas_only, c);
    *s_out = kernel_sums(C, p, h, c, 1, mode);
    *h_out = h;
    return 0;
  }
  /* Newton from the starting value (half the volume guess on a cold start);
   * the candidates cover r < 2 rc and are gathered again, with the margin
   * kappa, whenever an iterate leaves that radius.  The bracket [lo, hi] of
   * the monotone g catches steps that leave it (bisection, or doubling while
   * no upper end is known, which also bounds every step then). */
  double h = cold ? 0.5 * guess : guess, lo = 0.0, hi = INFINITY, dx_old = INFINITY;
  double rc = h * (1.0 + P->kappa);
  collect(C, p, 2.0 * rc, gas_only, c);
  sums_t s = {0, 0, 0, 0, 0, 0, 0};
  double h_eval = h;
  for (int it = 0; it < P->h_maxit; it++) {
    if (h > rc) {
      rc = h * (1.0 + P->kappa);
      collect(C, p, 2.0 * rc, gas_only, c);
    }
    s = kernel_sums(C, p, h, c, 1, mode);
    h_eval = h;
    (*iters)++;
    double nw = mass_w ? s.rho * imi : s.n, sdw = mass_w ? s.msdh * imi : s.sdh;
    double g = h * h * h * nw - eta3;
    double gp = 3.0 * h * h * nw + h * h * h * sdw;
    if (g < 0.0) lo = h;
    else hi = h;
    /* converged when the Newton step is below the tolerance; otherwise a
     * safeguarded Newton step: one that leaves the bracket, does not halve
     * the previous step, or more than doubles h while no upper end is known
     * (g' vanishes when only the particle itself lies within 2h) is replaced
     * by bisection, or by doubling while no upper end is known */
    double dx = g / gp;
    if (fabs(dx) < P->h_tol * h) {
      /* converged: the step is below tolerance; the quantities are those of
       * the last evaluated length */
      *h_out = h;
      *s_out = s;
      return 1;
    }
    double hn = h - dx;
    if (!(hn > lo && hn < hi) || fabs(dx) > 0.5 * dx_old || (isinf(hi) && hn > 2.0 * h))
      hn = isinf(hi) ? 2.0 * h : 0.5 * (lo + hi);
    dx_old = fabs(hn - h);
    h = hn;
  }
  *h_out = h_eval;
  *s_out = s;
  return 0;
}

static int cmp_double(const void *a, const void *b)
{
  double x = *(const double *)a, y = *(const double *)b;
  return (x > y) - (x < y);
}

/* Standard SPH (Sect. 3): h from a fixed neighbour count instead of the
 * kernel-weighted relation.  With the gas candidates sorted by squared
 * distance, the count reaches nstd at the first shell (all candidates at
 * one distance) whose cumulative weight is at least nstd -- every neighbour
 * counts 1, or m_j / m_i with the mass-density relation -- and 2h lies
 * midway between that shell's distance and the next larger distance.  The
 * neighbour set inside 2h is then that cumulative set: exactly nstd
 * particles, the sink included, unless the shell holds several (a lattice).
 * Returns 0 when there are too few gas particles. */
static int solve_count(const ctx_t *C, int64_t p, int64_t nstd, double guess, cand_t *c, double *h_out,
                       sums_t *s_out)
{
  const orc_tree *t = C->t;
  const int mass_w = C->p->h_weight == ORC_HW_MASS;
  double R = 2.0 * (guess > 0.0 ? guess : 1.0);
  for (;;) {
    collect(C, p, R, 1, c);
    /* (squared distance, weight) sorted by distance */
    double *d = malloc(2 * (c->n + 1) * sizeof(double));
    for (int64_t a = 0; a < c->n; a++) {
      int64_t q = c->idx[a];
      d[2 * a] = pair_r2(t->xs[p], t->ys[p], t->zs[p], t->xs[q], t->ys[q], t->zs[q], C->L);
      d[2 * a + 1] = mass_w ? t->ms[q] / t->ms[p] : 1.0;
    }
    qsort(d, c->n, 2 * sizeof(double), cmp_double);
    double cum = 0.0;
    int64_t k = 0;
    while (k < c->n) {
      /* the whole shell at distance d[2k] */
      double r2k = d[2 * k];
      while (k < c->n && d[2 * k] == r2k) cum += d[2 * k++ + 1];
      if (cum >= (double)nstd) {
        if (k < c->n) {
          double h = 0.25 * (sqrt(r2k) + sqrt(d[2 * k]));
          free(d);
          *h_out = h;
          *s_out = kernel_sums(C, p, h, c, 1, 0);
          return 1;
        }
        break;  /* the next distance lies beyond the gathered radius */
      }
    }
    free(d);
    if ((cum < (double)nstd && c->n >= C->n_gas) || R > 1e30) {
      /* fewer gas particles (or less weight) than the count needs */
      *h_out = 0.5 * R;
      *s_out = kernel_sums(C, p, 0.5 * R, c, 1, 0);
      return 0;
    }
    R *= 2.0;
  }
}

static double cold_guess(const ctx_t *C, int64_t p, int gas_only, double eta)
{
  const orc_tree *t = C->t;
  int64_t k = t->leaf_of[p];
  double cnt = (double)t->count[k];
  if (gas_only && C->ngas[k] > 0) cnt = (double)C->ngas[k];
  double s = t->side[k];
  return eta * cbrt(s * s * s / cnt);
}

static void density_phase(ctx_t *C, const double *h_in, const double *eps_in)
{
  const orc_params *P = C->p;
  const orc_tree *t = C->t;
  int64_t n = C->n;
  int64_t noconv = 0;
#pragma omp parallel reduction(+ : noconv)
  {
    cand_t c = {0};
    c.stack = malloc((8 * 22 * 8 + t->nnodes + 16) * sizeof(int64_t));
#pragma omp for schedule(dynamic, 16)
    for (int64_t p = 0; p < n; p++) {
      int64_t i = t->perm[p];
      /* gas: smoothing length over gas neighbours (Sect. 3, Eqs. hn, nsum) */
      if (P->hydro && C->gas[p]) {
        int cold = !(h_in && h_in[i] > 0.0);
        double guess = cold ? cold_guess(C, p, 1, P->eta_h) : h_in[i];
        double h;
        sums_t s;
        if (P->h_scheme == ORC_H_STANDARD) {
          /* the neighbour number of the relation eta = h n^(1/3) */
          int64_t nstd = llround(4.0 / 3.0 * M_PI * pow(2.0 * P->eta_h, 3.0));
          if (!solve_count(C, p, nstd, guess, &c, &h, &s)) noconv++;
        } else if (!solve_length(C, p, 1, 0, P->eta_h, guess, cold, &c, &h, &s, &C->iters[p])) {
          noconv++;
        }
        C->h[p] = h;
        C->nh[p] = s.n;
        C->rho[p] = s.rho;  /* Eq. densitySPH in every scheme */
        /* grad-h terms, Sect. 3 Eq. (drhodr) and the definitions after it:
         * Omega* = 1 - (dh/dn) sum dW/dh, zeta = (dh/dn) sum m dW/dh,
         * dh/dn = -h/(3 n); the standard scheme neglects them */
        if (P->h_scheme == ORC_H_STANDARD) {
          C->omega[p] = 1.0;
          C->zeta[p] = 0.0;
          C->fa[p] = 1.0;
        } else if (P->h_weight == ORC_HW_MASS) {
          /* h from the mass density: the correction of Springel & Hernquist,
           * f_ij = 1 / Omega_i with Omega_i = 1 + (h/(3 rho)) sum m dW/dh */
          double om = 1.0 + (h / (3.0 * s.rho)) * s.msdh;
          C->omega[p] = om;
          C->zeta[p] = 0.0;
          C->fa[p] = 1.0 / om;
        } else {
          C->omega[p] = 1.0 + (h / (3.0 * s.n)) * s.sdh;
          C->zeta[p] = -(h / (3.0 * s.n)) * s.msdh;
          C->fa[p] = 1.0;
        }
        /* velocity divergence (Sect. 2.1), with the gas kernel */
        C->divv[p] = -s.divv / (s.n * C->omega[p]);
        /* velocity curl with the normalisation of the divergence:
         * curl_i = (1/(n_i Omega_i)) sum_j v_ij x grad_i W_ij(h_i) */
        for (int d = 0; d < 3; d++) C->curl[3 * p + d] = s.curl[d] / (s.n * C->omega[p]);
      }
      /* all species: adaptive softening length over all neighbours
       * (Sect. 2.1, Eq. etan; Sect. 3.2, independent eps and h) */
      if (P->gravity) {
        if (P->soft_mode == ORC_SOFT_CONSTANT) {
          C->eps[p] = eps_in[i];
          C->ups[p] = 1.0;
          C->xi[p] = 0.0;
          C->neps[p] = 0.0;
        } else {
          int cold = !(eps_in && eps_in[i] > 0.0);
          double guess = cold ? cold_guess(C, p, 0, P->eta_eps) : eps_in[i];
          double e;
          sums_t s;
          if (!solve_length(C, p, 0, 1, P->eta_eps, guess, cold, &c, &e, &s, &C->iters[p])) noconv++;
          C->eps[p] = e;
          C->neps[p] = s.n;
          /* Upsilon = 1 - (d eps/dn) sum dW/d eps; xi~ = (d eps/dn) sum m dphi/deps
           * (Eq. zeta with the neighbour mass inside the sum, so that the
           * force is the gradient of the softened Lagrangian for unequal
           * masses) */
          C->ups[p] = 1.0 + (e / (3.0 * s.n)) * s.sdh;
          /* the printed Eq. zeta sums d phi / d eps without masses; that
           * weighting is kept under grav_corr_literal */
          double sphi = P->grav_corr_literal ? s.dphi : s.mdphi;
          C->xi[p] = (P->soft_mode == ORC_SOFT_ADAPTIVE) ? -(e / (3.0 * s.n)) * sphi : 0.0;
          C->divv_e[p] = -s.divv / (s.n * C->ups[p]);
        }
      }
    }
    free(c.idx);
    free(c.stack);
  }
  C->noconv = noconv;
}

/* per-node maxima of eps (all) and h (gas), gas counts */
static void node_maxima(ctx_t *C)
{
  const orc_tree *t = C->t;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t k = 0; k < t->nnodes; k++) {
    double em = 0.0, hm = 0.0;
    for (int64_t q = t->first[k]; q < t->first[k] + t->count[k]; q++) {
      if (C->eps[q] > em) em = C->eps[q];
      if (C->gas[q] && C->h[q] > hm) hm = C->h[q];
    }
    C->epsmax[k] = em;
    C->hmax[k] = hm;
    /* a softened cell's own length and correction weight (Sect. 2.2: a
     * node treated as one particle): the mass-weighted mean eps, and the
     * sum of m_j xi_j / Ups_j over its particles */
    double me = 0.0, mx = 0.0;
    for (int64_t q = t->first[k]; q < t->first[k] + t->count[k]; q++) {
      me += t->ms[q] * C->eps[q];
      mx += t->ms[q] * (C->xi[q] / C->ups[q]);
    }
    C->epsbar[k] = me / t->mass[k];
    C->xsum[k] = mx;
  }
}

/* ---- gravity ----------------------------------------------------------- */

/* periodic box: the replicas of mass m at displacement x (Sect. 4.3) */
static void ewald_add(const ctx_t *C, double m, double dx, double dy, double dz, double *a)
{
  if (!(C->L > 0.0)) return;
  double e[3];
  ewald_interp(C->ewt, C->L, dx, dy, dz, e);
  double G = C->p->G;
  a[0] += G * m * e[0];
  a[1] += G * m * e[1];
  a[2] += G * m * e[2];
}

/* Far-field node: monopole plus traceless quadrupole about the centre of
 * mass (Sect. 2.2), unsoftened. r = x_i - com.
 *   a = -G M r/r^3 + G [Q r / r^5 - 5/2 (r.Q.r) r / r^7]
 *   phi = -G M / r - G/2 (r.Q.r) / r^5 */
static void far_node(const ctx_t *C, int64_t k, double px, double py, double pz, double *a,
                     double *pot)
{
  const orc_tree *t = C->t;
  double G = C->p->G;
  double dx = wrapd(px - t->com[3 * k], C->L), dy = wrapd(py - t->com[3 * k + 1], C->L),
         dz = wrapd(pz - t->com[3 * k + 2], C->L);
  double r2 = dx * dx + dy * dy + dz * dz;
  double r = sqrt(r2), M = t->mass[k];
  double ir3 = 1.0 / (r2 * r);
  a[0] -= G * M * dx * ir3;
  a[1] -= G * M * dy * ir3;
  a[2] -= G * M * dz * ir3;
  *pot -= G * M / r;
  if (C->p->quadrupole) {
    const double *Q = &t->quad[6 * k];
    double qx = Q[0] * dx + Q[3] * dy + Q[4] * dz;
    double qy = Q[3] * dx + Q[1] * dy + Q[5] * dz;
    double qz = Q[4] * dx + Q[5] * dy + Q[2] * dz;
    double rqr = dx * qx + dy * qy + dz * qz;
    double ir5 = ir3 / r2, ir7 = ir5 / r2;
    a[0] += G * (qx * ir5 - 2.5 * rqr * dx * ir7);
    a[1] += G * (qy * ir5 - 2.5 * rqr * dy * ir7);
    a[2] += G * (qz * ir5 - 2.5 * rqr * dz * ir7);
    *pot -= 0.5 * G * rqr * ir5;
  }
  ewald_add(C, M, dx, dy, dz, a);
}

/* Softened pair j -> i (Sect. 2.1 Eq. dLgravdr, App. B):
 *   a_i -= G m_j 1/2 [phi'(r, eps_i) + phi'(r, eps_j)] r_hat
 *   a_i -= G/2 [xi_i/Ups_i dW/dr(r, eps_i) + (m_j/m_i) xi_j/Ups_j dW/dr(r, eps_j)] r_hat
 * with r_hat = (x_i - x_j)/r.  The correction's mass weighting is the one
 * that makes the force the gradient of the softened Lagrangian for unequal
 * masses (xi~ carries the neighbour masses); for equal masses it coincides
 * with the printed form. */
static void near_pair(const ctx_t *C, int64_t p, int64_t q, double *a, double *pot)
{
  const orc_tree *t = C->t;
  double G = C->p->G;
  double dx = wrapd(t->xs[p] - t->xs[q], C->L), dy = wrapd(t->ys[p] - t->ys[q], C->L),
         dz = wrapd(t->zs[p] - t->zs[q], C->L);
  double r2 = dx * dx + dy * dy + dz * dz, r = sqrt(r2);
  double ei = C->eps[p], ej = C->eps[q], mj = t->ms[q];
  *pot += G * mj * 0.5 * (orc_phi(r, ei) + orc_phi(r, ej));
  if (!(r > 0.0)) return;
  ewald_add(C, mj, dx, dy, dz, a);
  double f = G * mj * 0.5 * (orc_dphidr(r, ei) + orc_dphidr(r, ej));
  if (C->p->soft_mode == ORC_SOFT_ADAPTIVE) {
    if (C->p->grav_corr_literal)
      /* Eq. dLgravdr as printed: m_j [xi_i/Ups_i W'(eps_i) + xi_j/Ups_j W'(eps_j)]
       * with xi of Eq. zeta (no masses), the j-gradient taken with eps_j */
      f += 0.5 * G * mj * ((C->xi[p] / C->ups[p]) * orc_dWdr(r, ei) + (C->xi[q] / C->ups[q]) * orc_dWdr(r, ej));
    else
      f += 0.5 * G * ((C->xi[p] / C->ups[p]) * orc_dWdr(r, ei) +
                      (mj / t->ms[p]) * (C->xi[q] / C->ups[q]) * orc_dWdr(r, ej));
  }
  a[0] -= f * dx / r;
  a[1] -= f * dy / r;
  a[2] -= f * dz / r;
}

/* Softened cell k acting on sink p (Sect. 2.2): the node taken as one
 * particle of mass M at its centre of mass with the mass-weighted mean eps
 * of its particles, through the symmetrised softened pair, and the
 * correction terms of its particles gathered there: the sink's term counts
 * each particle of the cell (N of them; with the printed weighting, their
 * mass M), the cell's term is the sum of m_j xi_j / Ups_j. */
static void soft_cell(const ctx_t *C, int64_t k, int64_t p, double *a, double *pot)
{
  const orc_tree *t = C->t;
  double G = C->p->G;
  double dx = wrapd(t->xs[p] - t->com[3 * k], C->L), dy = wrapd(t->ys[p] - t->com[3 * k + 1], C->L),
         dz = wrapd(t->zs[p] - t->com[3 * k + 2], C->L);
  double r = sqrt(dx * dx + dy * dy + dz * dz);
  double ei = C->eps[p], ek = C->epsbar[k], M = t->mass[k];
  ewald_add(C, M, dx, dy, dz, a);
  *pot += G * M * 0.5 * (orc_phi(r, ei) + orc_phi(r, ek));
  double f = G * M * 0.5 * (orc_dphidr(r, ei) + orc_dphidr(r, ek));
  if (C->p->soft_mode == ORC_SOFT_ADAPTIVE) {
    double wi = orc_dWdr(r, ei), wk = orc_dWdr(r, ek), xu = C->xi[p] / C->ups[p];
    if (C->p->grav_corr_literal)
      f += 0.5 * G * (M * xu * wi + C->xsum[k] * wk);
    else
      f += 0.5 * G * ((double)t->count[k] * xu * wi + (C->xsum[k] / t->ms[p]) * wk);
  }
  a[0] -= f * dx / r;
  a[1] -= f * dy / r;
  a[2] -= f * dz / r;
}

/* opening test (Sect. 2.2 Eq. opcrit, Dubinski): accept a node when the sink
 * is farther from its centre of mass than l/theta + delta (strictly), and no
 * particle of the node can lie within the softening reach 2 max(eps_i,
 * eps_node) of the sink ("softening-clear"); accepted nodes are unsoftened. */
/* returns 1 for an accepted (unsoftened) node, 2 for a softened cell (with
 * soften_cells: the opening test passes but the node lies within the
 * softening reach), 0 to open it */
static int accept_point(const ctx_t *C, int64_t k, double px, double py, double pz, double ei)
{
  const orc_params *P = C->p;
  const orc_tree *t = C->t;
  if (!(P->theta > 0.0)) return 0;
  double rm = t->side[k] / P->theta + t->delta[k];
  double d2 = pair_r2(px, py, pz, t->com[3 * k], t->com[3 * k + 1], t->com[3 * k + 2], C->L);
  if (!(d2 > rm * rm)) return 0;
  double s = 2.0 * (ei > C->epsmax[k] ? ei : C->epsmax[k]);
  if (box_point_d2(&t->bmin[3 * k], &t->bmax[3 * k], px, py, pz, C->L) >= s * s) return 1;
  return P->soften_cells ? 2 : 0;
}

static int accept_box(const ctx_t *C, int64_t k, const double *lo, const double *hi, double emax)
{
  const orc_params *P = C->p;
  const orc_tree *t = C->t;
  if (!(P->theta > 0.0)) return 0;
  double rm = t->side[k] / P->theta + t->delta[k];
  double d2 = box_point_d2(lo, hi, t->com[3 * k], t->com[3 * k + 1], t->com[3 * k + 2], C->L);
  if (!(d2 > rm * rm)) return 0;
  double s = 2.0 * (emax > C->epsmax[k] ? emax : C->epsmax[k]);
  if (box_box_d2(lo, hi, &t->bmin[3 * k], &t->bmax[3 * k], C->L) >= s * s) return 1;
  return P->soften_cells ? 2 : 0;
}

static void self_term(const ctx_t *C, int64_t p, double *pot)
{
  *pot += C->p->G * C->t->ms[p] * orc_phi(0.0, C->eps[p]);
}

static void gravity_particle_walk(ctx_t *C)
{
  const orc_tree *t = C->t;
#pragma omp parallel
  {
    int64_t *stack = malloc((8 * 22 * 8 + t->nnodes + 16) * sizeof(int64_t));
#pragma omp for schedule(dynamic, 16)
    for (int64_t p = 0; p < C->n; p++) {
      if (!C->active[p]) continue;
      double a[3] = {0, 0, 0}, pot = 0.0;
      int64_t nnode = 0, npair = 0, nsoft = 0, sp = 0;
      double px = t->xs[p], py = t->ys[p], pz = t->zs[p];
      stack[sp++] = 0;
      while (sp > 0) {
        int64_t k = stack[--sp];
        int acc = accept_point(C, k, px, py, pz, C->eps[p]);
        if (acc == 1) {
          far_node(C, k, px, py, pz, a, &pot);
          nnode++;
        } else if (acc == 2) {
          soft_cell(C, k, p, a, &pot);
          nnode++;
        } else if (t->nchild[k] == 0) {
          for (int64_t q = t->first[k]; q < t->first[k] + t->count[k]; q++)
            if (q != p) {
              near_pair(C, p, q, a, &pot);
              npair++;
              double R = 2.0 * (C->eps[p] > C->eps[q] ? C->eps[p] : C->eps[q]);
              if (pair_r2(px, py, pz, t->xs[q], t->ys[q], t->zs[q], C->L) < R * R) nsoft++;
            }
        } else {
          for (int32_t b = t->nchild[k] - 1; b >= 0; b--) stack[sp++] = t->child[k] + b;
        }
      }
      self_term(C, p, &pot);
      C->ax[p] = a[0]; C->ay[p] = a[1]; C->az[p] = a[2];
      C->pot[p] = pot;
      C->cnt_node[p] = nnode;
      C->cnt_pair[p] = npair;
      C->cnt_soft[p] = nsoft;
    }
    free(stack);
  }
}

/* Group mode: every sink of a walk batch (consecutive sibling groups, each a
 * maximal node of at most group_size particles, packed up to batch_size
 * particles) receives the interaction set found with the batch's bounding box
 * (union of the members' boxes) and its largest eps in the opening test.  The
 * set is a superset of each member's per-particle set, so accuracy is at
 * least that of the per-particle walk. */
static void gravity_group_walk(ctx_t *C)
{
  const orc_tree *t = C->t;
  int32_t G = C->p->group_size, B = C->p->batch_size;
  int64_t nb = orc_tree_batches(t, G, B, C->p->batch_mode, NULL, NULL);
  int64_t ng = orc_tree_groups(t, G, NULL);
  int64_t *gn = malloc((ng + 1) * sizeof(int64_t));
  orc_tree_groups(t, G, gn);
  int64_t *bk0 = malloc((nb + 1) * sizeof(int64_t)), *bk1 = malloc((nb + 1) * sizeof(int64_t));
  orc_tree_batches(t, G, B, C->p->batch_mode, bk0, bk1);
#pragma omp parallel
  {
    int64_t *stack = malloc((8 * 22 * 8 + t->nnodes + 16) * sizeof(int64_t));
    int64_t *acc = malloc((t->nnodes + 1) * sizeof(int64_t));
    int64_t *lvs = malloc((t->nnodes + 1) * sizeof(int64_t));
    int64_t *scl = malloc((t->nnodes + 1) * sizeof(int64_t));
#pragma omp for schedule(dynamic, 4)
    for (int64_t g = 0; g < nb; g++) {
      double lo[3], hi[3], emax = 0.0;
      int64_t k0 = gn[bk0[g]], kl = gn[bk1[g] - 1];
      for (int d = 0; d < 3; d++) { lo[d] = t->bmin[3 * k0 + d]; hi[d] = t->bmax[3 * k0 + d]; }
      for (int64_t i = bk0[g]; i < bk1[g]; i++) {
        int64_t k = gn[i];
        for (int d = 0; d < 3; d++) {
          if (t->bmin[3 * k + d] < lo[d]) lo[d] = t->bmin[3 * k + d];
          if (t->bmax[3 * k + d] > hi[d]) hi[d] = t->bmax[3 * k + d];
        }
        if (C->epsmax[k] > emax) emax = C->epsmax[k];
      }
      int64_t pfirst = t->first[k0];
      int64_t pend = t->first[kl] + t->count[kl];
      /* with a sink sample, only batches holding a sampled sink are walked
       * (the lists are the batch's, so their values are those of a full run) */
      int any = 0;
      for (int64_t p = pfirst; p < pend && !any; p++) any = C->active[p];
      if (!any) continue;
      int64_t na = 0, nl = 0, ns = 0, sp = 0;
      stack[sp++] = 0;
      while (sp > 0) {
        int64_t k = stack[--sp];
        int ab = accept_box(C, k, lo, hi, emax);
        if (ab == 1) acc[na++] = k;
        else if (ab == 2) scl[ns++] = k;
        else if (t->nchild[k] == 0) lvs[nl++] = k;
        else for (int32_t b = t->nchild[k] - 1; b >= 0; b--) stack[sp++] = t->child[k] + b;
      }
      for (int64_t p = pfirst; p < pend; p++) {
        if (!C->active[p]) continue;
        double a[3] = {0, 0, 0}, pot = 0.0;
        int64_t npair = 0;
        double px = t->xs[p], py = t->ys[p], pz = t->zs[p];
        for (int64_t b = 0; b < na; b++) far_node(C, acc[b], px, py, pz, a, &pot);
        for (int64_t b = 0; b < ns; b++) soft_cell(C, scl[b], p, a, &pot);
        for (int64_t b = 0; b < nl; b++) {
          int64_t k = lvs[b];
          for (int64_t q = t->first[k]; q < t->first[k] + t->count[k]; q++)
            if (q != p) { near_pair(C, p, q, a, &pot); npair++; }
        }
        self_term(C, p, &pot);
        C->ax[p] = a[0]; C->ay[p] = a[1]; C->az[p] = a[2];
        C->pot[p] = pot;
        C->cnt_node[p] = na + ns;
        C->cnt_pair[p] = npair;
      }
    }
    free(stack); free(acc); free(lvs); free(scl);
  }
  free(bk0);
  free(bk1);
  free(gn);
}

/* O(N^2): every pair softened and corrected, the definition the tree
 * approximates (theta -> 0). */
static void gravity_direct(ctx_t *C)
{
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t p = 0; p < C->n; p++) {
    if (!C->active[p]) continue;
    double a[3] = {0, 0, 0}, pot = 0.0;
    for (int64_t q = 0; q < C->n; q++)
      if (q != p) near_pair(C, p, q, a, &pot);
    self_term(C, p, &pot);
    C->ax[p] = a[0]; C->ay[p] = a[1]; C->az[p] = a[2];
    C->pot[p] = pot;
    C->cnt_node[p] = 0;
    C->cnt_pair[p] = C->n - 1;
  }
}

/* ---- SPH ---------------------------------------------------------------- */

/* Pair i <- j of the variable-mass Lagrangian SPH equations (Sect. 3 Eqs.
 * motionvarmass, thermalvarmass, Sect. 3.3 Eq. mu_visc; App. B).  Convention:
 * grad_i W_ij(h) = dW/dr(r, h) (x_i - x_j)/r.  With it the equations read
 *   a_i  = -sum_j m_j [A_ij gW(h_i) + A_ji gW(h_j) + Pi_ij Gbar_ij]
 *   du_i =  sum_j m_j [A_ij v_ij . gW(h_i) + 1/2 Pi_ij v_ij . Gbar_ij]
 * A_ij = P_i f_ij / rho_i^2, f_ij = 1 + zeta_i/(m_j Omega*_i),
 * Gbar_ij = 1/2 [f_ij gW(h_i) + f_ji gW(h_j)], v_ij = v_i - v_j; this is the
 * printed set once the 1/m_i of dv/dt and the orientation of the gradient are
 * made consistent (pressure repulsive, compression heating).  Pi_ij is the
 * Monaghan-Gingold term with hbar, cbar, rhobar the arithmetic pair means and
 * eta^2 = av_eps2 hbar^2; it acts only on approaching pairs. */
typedef struct {
  double a[3], du, du_v, mumax, vsig, xs[3];  /* du: pressure + viscous; du_v: viscous */
  double lapu;                                /* Laplacian of u (Brookshaw)              */
} sph_acc_t;

/* Variants (flags of orc_params):
 *   visc_form SIGNAL: Pi_ij = -alpha v_sig w_ij / rhobar with w_ij = v_ij . x_ij / r
 *     and v_sig = 2 cbar - w_ij (Sect. 3.3.1, Eqs. pvsig, vsig), approaching pairs;
 *     mu is still formed for the time-step criterion;
 *   entropy: the energy variable is A = P / rho^gamma and its rate is the
 *     viscous term only, dA_i = (gamma - 1) rho_i^(1 - gamma) sum_j 1/2 m_j
 *     Pi_ij v_ij . Gbar_ij (Sect. 3.4, Eq. SPHentr);
 *   xsph_eta > 0: the X-SPH velocity correction eta sum_j m_j (v_j - v_i)
 *     Wbar_ij / rhobar_ij with Wbar_ij = 1/2 [W(r, h_i) + W(r, h_j)] over the
 *     same pairs (Sect. 3.5, Eq. xsph).
 * The signal velocity of every pair, 2 cbar - min(w_ij, 0), gives the
 * largest one per particle (vsig). */
static void sph_pair(const ctx_t *C, int64_t p, int64_t q, sph_acc_t *acc)
{
  const orc_params *P = C->p;
  const orc_tree *t = C->t;
  double dx = wrapd(t->xs[p] - t->xs[q], C->L), dy = wrapd(t->ys[p] - t->ys[q], C->L),
         dz = wrapd(t->zs[p] - t->zs[q], C->L);
  double r2 = dx * dx + dy * dy + dz * dz;
  if (!(r2 > 0.0)) return;
  double r = sqrt(r2);
  double hi = C->h[p], hj = C->h[q], mi = t->ms[p], mj = t->ms[q];
  double gi = (P->tc92 ? orc_dWdr_tc92(r, hi) : orc_dWdr(r, hi)) / r;
  double gj = (P->tc92 ? orc_dWdr_tc92(r, hj) : orc_dWdr(r, hj)) / r;
  double fij = C->fa[p] + C->zeta[p] / (mj * C->omega[p]);
  double fji = C->fa[q] + C->zeta[q] / (mi * C->omega[q]);
  double Ai = C->P[p] * fij / (C->rho[p] * C->rho[p]);
  double Aj = C->P[q] * fji / (C->rho[q] * C->rho[q]);
  double vx = C->vx[p] - C->vx[q], vy = C->vy[p] - C->vy[q], vz = C->vz[p] - C->vz[q];
  double vd = vx * dx + vy * dy + vz * dz;
  double s = mj * (Ai * gi + Aj * gj);
  double cb = 0.5 * (C->cs[p] + C->cs[q]);
  double rb = 0.5 * (C->rho[p] + C->rho[q]);
  double w = vd / r;
  double e = mj * Ai * gi * vd;
  if (vd < 0.0) {
    double hb = 0.5 * (hi + hj);
    double mu = hb * vd / (r2 + P->av_eps2 * hb * hb);
    /* per-particle alpha: the pair mean replaces alpha (Sect. 3.3.1) */
    double al = P->alpha_switch ? 0.5 * (C->alpha[p] + C->alpha[q]) : P->alpha;
    double Pi = P->visc_form == ORC_VISC_SIGNAL ? -al * (2.0 * cb - w) * w / rb
                                                : (-al * cb * mu + P->beta * mu * mu) / rb;
    if (P->balsara) Pi *= 0.5 * (C->fbal[p] + C->fbal[q]);
    double Gb = 0.5 * (fij * gi + fji * gj);
    s += mj * Pi * Gb;
    double ev = 0.5 * mj * Pi * Gb * vd;
    e += ev;
    acc->du_v += ev;
    if (fabs(mu) > acc->mumax) acc->mumax = fabs(mu);
  }
  acc->du += e;
  double vs = 2.0 * cb - (w < 0.0 ? w : 0.0);
  if (vs > acc->vsig) acc->vsig = vs;
  if (P->conduction) {
    /* artificial conductivity (Sect. 3.3.2): Pi^u = -alphabar^u v^u_sig
     * (u_i - u_j) / rhobar with v^u_sig = sqrt(|P_i - P_j| / rhobar), acting
     * through the averaged gradient's magnitude |Gbar| = |Gb| r; and the
     * Laplacian of u (Brookshaw), -sum_j 2 m_j (u_i - u_j) / rho_j |Gbar| / r:
     * the printed sum without the minus sign is minus the Laplacian, which
     * the source term's |lap u| does not see */
    double Gbm = fabs(0.5 * (fij * gi + fji * gj)) * r;
    double du_ij = C->u[p] - C->u[q];
    double vsu = sqrt(fabs(C->P[p] - C->P[q]) / rb);
    double Piu = -0.5 * (C->alpha_u[p] + C->alpha_u[q]) * vsu * du_ij / rb;
    acc->du += mj * Piu * Gbm;
    acc->lapu -= 2.0 * mj * du_ij / C->rho[q] * Gbm / r;
  }
  if (P->xsph_eta > 0.0) {
    double wb = 0.5 * (orc_W(r, hi) + orc_W(r, hj)) / rb;
    acc->xs[0] -= mj * vx * wb;
    acc->xs[1] -= mj * vy * wb;
    acc->xs[2] -= mj * vz * wb;
  }
  acc->a[0] -= s * dx;
  acc->a[1] -= s * dy;
  acc->a[2] -= s * dz;
}

/* symmetric neighbour condition r < 2 max(h_i, h_j) (Sect. 3.1) */
static int sph_nbr(const ctx_t *C, int64_t p, int64_t q)
{
  const orc_tree *t = C->t;
  double r2 = pair_r2(t->xs[p], t->ys[p], t->zs[p], t->xs[q], t->ys[q], t->zs[q], C->L);
  double R = 2.0 * (C->h[p] > C->h[q] ? C->h[p] : C->h[q]);
  return r2 < R * R;
}

static void sph_phase(ctx_t *C)
{
  const orc_params *P = C->p;
  const orc_tree *t = C->t;
  for (int64_t p = 0; p < C->n; p++) {
    if (!C->gas[p]) continue;
    if (P->entropy) {
      /* the energy variable is A: P = A rho^gamma, c^2 = gamma P / rho */
      C->P[p] = C->u[p] * pow(C->rho[p], P->gamma);
      C->cs[p] = sqrt(P->gamma * C->u[p] * pow(C->rho[p], P->gamma - 1.0));
    } else {
      C->P[p] = (P->gamma - 1.0) * C->rho[p] * C->u[p];
      C->cs[p] = sqrt(P->gamma * (P->gamma - 1.0) * C->u[p]);
    }
  }
  /* Balsara limiter (Sect. 3.3.1): f = |div v| / (|div v| + |curl v| + 1e-4 c / h) */
  for (int64_t p = 0; p < C->n; p++) {
    if (!C->gas[p]) continue;
    double cu = sqrt(C->curl[3 * p] * C->curl[3 * p] + C->curl[3 * p + 1] * C->curl[3 * p + 1] +
                     C->curl[3 * p + 2] * C->curl[3 * p + 2]);
    double dv = fabs(C->divv[p]);
    C->fbal[p] = dv / (dv + cu + 1e-4 * C->cs[p] / C->h[p]);
  }
#pragma omp parallel
  {
    int64_t *stack = malloc((8 * 22 * 8 + t->nnodes + 16) * sizeof(int64_t));
#pragma omp for schedule(dynamic, 16)
    for (int64_t p = 0; p < C->n; p++) {
      if (!C->gas[p] || !C->active[p]) continue;
      sph_acc_t acc;
      memset(&acc, 0, sizeof(acc));
      int64_t npair = 0;
      if (P->nbr_mode == ORC_NBR_BRUTE) {
        for (int64_t q = 0; q < C->n; q++)
          if (q != p && C->gas[q] && sph_nbr(C, p, q)) { sph_pair(C, p, q, &acc); npair++; }
      } else {
        int64_t sp = 0;
        double px = t->xs[p], py = t->ys[p], pz = t->zs[p];
        stack[sp++] = 0;
        while (sp > 0) {
          int64_t k = stack[--sp];
          if (C->ngas[k] == 0) continue;
          double R = 2.0 * (C->h[p] > C->hmax[k] ? C->h[p] : C->hmax[k]);
          if (!(box_point_d2(&t->bmin[3 * k], &t->bmax[3 * k], px, py, pz, C->L) < R * R)) continue;
          if (t->nchild[k] == 0) {
            for (int64_t q = t->first[k]; q < t->first[k] + t->count[k]; q++)
              if (q != p && C->gas[q] && sph_nbr(C, p, q)) { sph_pair(C, p, q, &acc); npair++; }
          } else {
            for (int32_t b = t->nchild[k] - 1; b >= 0; b--) stack[sp++] = t->child[k] + b;
          }
        }
      }
      C->ax[p] += acc.a[0];
      C->ay[p] += acc.a[1];
      C->az[p] += acc.a[2];
      C->dudt[p] = P->entropy ? (P->gamma - 1.0) * pow(C->rho[p], 1.0 - P->gamma) * acc.du_v : acc.du;
      C->maxmu[p] = acc.mumax;
      C->vsig[p] = acc.vsig;
      C->xsx[p] = P->xsph_eta * acc.xs[0];
      C->xsy[p] = P->xsph_eta * acc.xs[1];
      C->xsz[p] = P->xsph_eta * acc.xs[2];
      C->lapu[p] = acc.lapu;
      /* the coefficients' rates (Sect. 3.3.1, 3.3.2): relaxation to the floor
       * over tau = h / (0.1 v_sig), sources 0.75 f max(0, -div v) and
       * h |lap u| / sqrt(u) */
      double tau = acc.vsig > 0.0 ? C->h[p] / (0.1 * acc.vsig) : INFINITY;
      if (P->alpha_switch) {
        double src = 0.75 * C->fbal[p] * (C->divv[p] < 0.0 ? -C->divv[p] : 0.0);
        C->dalpha[p] = -(C->alpha[p] - P->alpha_min) / tau + src;
      }
      if (P->conduction) {
        double src = C->u[p] > 0.0 ? C->h[p] * fabs(acc.lapu) / sqrt(C->u[p]) : 0.0;
        C->dalpha_u[p] = -(C->alpha_u[p] - P->alpha_u_min) / tau + src;
      }
      C->cnt_sph[p] = npair;
    }
    free(stack);
  }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static double wall_seconds(void)
{
#ifdef _OPENMP
  return omp_get_wtime();
#else
  return 0.0;
#endif
}

int orc_compute_forces(const orc_params *p, orc_run *r)
{
  if (!p || !r || r->n <= 0 || r->n_gas < 0 || r->n_gas > r->n) return -1;
  if (!r->x || !r->y || !r->z || !r->m) return -1;
  if (p->gravity && p->soft_mode == ORC_SOFT_CONSTANT && !r->eps_in) return -1;
  if (p->conduction && p->entropy) return -1;  /* conduction acts on u */
  if (!(p->period >= 0.0)) return -1;
  int64_t n = r->n;
  double t0 = wall_seconds();
  /* a periodic box takes the positions modulo its side (Sect. 4.3) */
  const double L = p->period;
  double *wx = NULL, *wy = NULL, *wz = NULL;
  const double *px = r->x, *py = r->y, *pz = r->z;
  if (L > 0.0) {
    wx = malloc(n * sizeof(double));
    wy = malloc(n * sizeof(double));
    wz = malloc(n * sizeof(double));
    for (int64_t i = 0; i < n; i++) {
      wx[i] = r->x[i] - L * floor(r->x[i] / L);
      wy[i] = r->y[i] - L * floor(r->y[i] / L);
      wz[i] = r->z[i] - L * floor(r->z[i] / L);
    }
    px = wx;
    py = wy;
    pz = wz;
  }
  orc_tree *t = orc_tree_build(n, px, py, pz, r->m, p->leaf_size);
  free(wx);
  free(wy);
  free(wz);
  if (!t) return -2;
  ctx_t C;
  memset(&C, 0, sizeof(C));
  C.p = p;
  C.L = L;
  C.ewt = (L > 0.0 && p->gravity) ? ewald_table(L) : NULL;
  C.t = t;
  C.n = n;
  C.n_gas = r->n_gas;
  C.vx = calloc(n, sizeof(double)); C.vy = calloc(n, sizeof(double)); C.vz = calloc(n, sizeof(double));
  C.u = calloc(n, sizeof(double));
  C.gas = calloc(n, 1);
  for (int64_t q = 0; q < n; q++) {
    int64_t i = t->perm[q];
    C.vx[q] = r->vx ? r->vx[i] : 0.0;
    C.vy[q] = r->vy ? r->vy[i] : 0.0;
    C.vz[q] = r->vz ? r->vz[i] : 0.0;
    C.gas[q] = i < r->n_gas;
    C.u[q] = (C.gas[q] && r->u) ? r->u[i] : 0.0;
  }
  C.h = calloc(n, sizeof(double)); C.nh = calloc(n, sizeof(double)); C.rho = calloc(n, sizeof(double));
  C.omega = calloc(n, sizeof(double)); C.zeta = calloc(n, sizeof(double)); C.divv = calloc(n, sizeof(double));
  C.divv_e = calloc(n, sizeof(double));
  C.eps = calloc(n, sizeof(double)); C.neps = calloc(n, sizeof(double)); C.ups = calloc(n, sizeof(double));
  C.xi = calloc(n, sizeof(double));
  C.ax = calloc(n, sizeof(double)); C.ay = calloc(n, sizeof(double)); C.az = calloc(n, sizeof(double));
  C.pot = calloc(n, sizeof(double)); C.dudt = calloc(n, sizeof(double)); C.maxmu = calloc(n, sizeof(double));
  C.P = calloc(n, sizeof(double)); C.cs = calloc(n, sizeof(double));
  C.fa = calloc(n, sizeof(double));
  for (int64_t q = 0; q < n; q++) C.fa[q] = 1.0;
  C.xsx = calloc(n, sizeof(double)); C.xsy = calloc(n, sizeof(double)); C.xsz = calloc(n, sizeof(double));
  C.vsig = calloc(n, sizeof(double));
  C.curl = calloc(3 * n, sizeof(double)); C.fbal = calloc(n, sizeof(double)); C.lapu = calloc(n, sizeof(double));
  C.alpha = calloc(n, sizeof(double)); C.alpha_u = calloc(n, sizeof(double));
  C.dalpha = calloc(n, sizeof(double)); C.dalpha_u = calloc(n, sizeof(double));
  for (int64_t q = 0; q < n; q++) {
    int64_t i = t->perm[q];
    C.alpha[q] = r->alpha_in ? r->alpha_in[i] : p->alpha;
    C.alpha_u[q] = r->alpha_u_in ? r->alpha_u_in[i] : 0.0;
  }
  C.cnt_node = calloc(n, sizeof(int64_t)); C.cnt_pair = calloc(n, sizeof(int64_t));
  C.cnt_sph = calloc(n, sizeof(int64_t));
  C.cnt_soft = calloc(n, sizeof(int64_t));
  C.iters = calloc(n, sizeof(int32_t));
  C.active = malloc(n);
  if (r->n_sinks > 0) {
    int64_t *inv = malloc(n * sizeof(int64_t));
    for (int64_t q = 0; q < n; q++) inv[t->perm[q]] = q;
    memset(C.active, 0, n);
    for (int64_t s = 0; s < r->n_sinks; s++)
      if (r->sinks[s] >= 0 && r->sinks[s] < n) C.active[inv[r->sinks[s]]] = 1;
    free(inv);
  } else {
    memset(C.active, 1, n);
  }
  C.epsmax = calloc(t->nnodes, sizeof(double));
  C.hmax = calloc(t->nnodes, sizeof(double));
  C.epsbar = calloc(t->nnodes, sizeof(double));
  C.xsum = calloc(t->nnodes, sizeof(double));
  C.ngas = calloc(t->nnodes, sizeof(int64_t));
  for (int64_t k = 0; k < t->nnodes; k++) {
    int64_t g = 0;
    for (int64_t q = t->first[k]; q < t->first[k] + t->count[k]; q++) g += C.gas[q];
    C.ngas[k] = g;
  }
  double t1 = wall_seconds();
  /* 1. densities and lengths (Sect. 3.1: first, gather, walk) */
  density_phase(&C, r->h_in, r->eps_in);
  node_maxima(&C);
  double t2 = wall_seconds();
  /* 2. gravity with the softened near field and its corrections */
  if (p->gravity) {
    if (p->walk_mode == ORC_WALK_DIRECT) gravity_direct(&C);
    else if (p->walk_mode == ORC_WALK_GROUP) gravity_group_walk(&C);
    else gravity_particle_walk(&C);
  }
  double t3 = wall_seconds();
  /* 3. SPH pressure, viscosity and heating (Sect. 3.1: second walk) */
  if (p->hydro) sph_phase(&C);
  double t4 = wall_seconds();
  r->t_phase[0] = t1 - t0;
  r->t_phase[1] = t2 - t1;
  r->t_phase[2] = t3 - t2;
  r->t_phase[3] = t4 - t3;
  r->n_noconv = C.noconv;
  /* scatter to caller order */
  for (int64_t q = 0; q < n; q++) {
    int64_t i = t->perm[q];
#define OUT(arr, src) if (r->arr) r->arr[i] = C.src[q]
    OUT(h, h); OUT(nh, nh); OUT(rho, rho); OUT(omega, omega); OUT(zeta, zeta); OUT(divv, divv); OUT(divv_eps, divv_e);
    OUT(eps, eps); OUT(neps, neps); OUT(ups, ups); OUT(xi, xi);
    OUT(ax, ax); OUT(ay, ay); OUT(az, az); OUT(pot, pot); OUT(dudt, dudt); OUT(maxmu, maxmu);
    OUT(cnt_node, cnt_node); OUT(cnt_pair, cnt_pair); OUT(cnt_sph, cnt_sph); OUT(iters, iters);
    OUT(cnt_soft, cnt_soft);
    OUT(xsph_x, xsx); OUT(xsph_y, xsy); OUT(xsph_z, xsz); OUT(vsig, vsig);
    OUT(fbal, fbal); OUT(lapu, lapu); OUT(dalpha, dalpha); OUT(dalpha_u, dalpha_u);
    if (r->curlx) { r->curlx[i] = C.curl[3 * q]; r->curly[i] = C.curl[3 * q + 1]; r->curlz[i] = C.curl[3 * q + 2]; }
#undef OUT
  }
  free(C.vx); free(C.vy); free(C.vz); free(C.u); free(C.gas);
  free(C.h); free(C.nh); free(C.rho); free(C.omega); free(C.zeta); free(C.divv); free(C.divv_e);
  free(C.eps); free(C.neps); free(C.ups); free(C.xi);
  free(C.ax); free(C.ay); free(C.az); free(C.pot); free(C.dudt); free(C.maxmu);
  free(C.P); free(C.cs); free(C.fa); free(C.xsx); free(C.xsy); free(C.xsz); free(C.vsig);
  free(C.curl); free(C.fbal); free(C.lapu); free(C.alpha); free(C.alpha_u); free(C.dalpha); free(C.dalpha_u); free(C.cnt_node); free(C.cnt_pair); free(C.cnt_sph); free(C.iters);
  free(C.cnt_soft); free(C.active);
  free(C.epsmax); free(C.hmax); free(C.ngas); free(C.epsbar); free(C.xsum);
  orc_tree_free(t);
  return 0;
}

/* ===================================================================== */
/* Neighbour sets                                                          */
/* ===================================================================== */

static int cmp_i64_int(const void *a, const void *b)
{
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  return (x > y) - (x < y);
}

int64_t orc_neighbours(int kind, int mode, int64_t n, int64_t n_gas, const double *x,
                       const double *y, const double *z, const double *len, int32_t leaf_size,
                       int64_t *offsets, int64_t *idx, int64_t cap, double period)
{
  /* The predicates are the symmetric ones of Sect. 3.1 and the correction
   * criterion of Sect. 2.1, evaluated on caller-order coordinates with
   * dx = x_j - x_i, r^2 = dx dx + dy dy + dz dz (left to right); in a
   * periodic box the positions are taken modulo the side and dx is the
   * nearest image. */
  const double L = period > 0.0 ? period : 0.0;
  double *wx = NULL, *wy = NULL, *wz = NULL;
  if (L > 0.0) {
    wx = malloc(n * sizeof(double));
    wy = malloc(n * sizeof(double));
    wz = malloc(n * sizeof(double));
    for (int64_t i = 0; i < n; i++) {
      wx[i] = x[i] - L * floor(x[i] / L);
      wy[i] = y[i] - L * floor(y[i] / L);
      wz[i] = z[i] - L * floor(z[i] / L);
    }
    x = wx;
    y = wy;
    z = wz;
  }
  int64_t *cnt = calloc(n, sizeof(int64_t));
  orc_tree *t = (mode == ORC_NBR_TREE) ? orc_tree_build(n, x, y, z, NULL, leaf_size) : NULL;
  double *lmax = NULL;
  if (t) {
    lmax = calloc(t->nnodes, sizeof(double));
    for (int64_t k = 0; k < t->nnodes; k++) {
      double mx = 0.0;
      for (int64_t q = t->first[k]; q < t->first[k] + t->count[k]; q++) {
        int64_t j = t->perm[q];
        if (kind != 2 && j >= n_gas) continue;
        if (len[j] > mx) mx = len[j];
      }
      lmax[k] = mx;
    }
  }
  for (int pass = 0; pass < 2; pass++) {
    int64_t total = 0;
    if (pass == 1) {
      offsets[0] = 0;
      for (int64_t i = 0; i < n; i++) offsets[i + 1] = offsets[i] + cnt[i];
      total = offsets[n];
      if (total > cap) { free(cnt); free(lmax); orc_tree_free(t); free(wx); free(wy); free(wz); return -1; }
    }
#pragma omp parallel
    {
      int64_t *stack = t ? malloc((8 * 22 * 8 + t->nnodes + 16) * sizeof(int64_t)) : NULL;
#pragma omp for schedule(dynamic, 16)
      for (int64_t i = 0; i < n; i++) {
        int sink = (kind == 2) || (i < n_gas);
        if (!sink) continue;
        int64_t c = 0, base = pass ? offsets[i] : 0;
        if (!t) {
          for (int64_t j = 0; j < n; j++) {
            if (kind != 2 && j >= n_gas) continue;
            if (kind != 0 && j == i) continue;
            double r2 = pair_r2(x[i], y[i], z[i], x[j], y[j], z[j], L);
            double Lj = (kind == 0) ? len[i] : (len[i] > len[j] ? len[i] : len[j]);
            double R = 2.0 * Lj;
            if (r2 < R * R) { if (pass) idx[base + c] = j; c++; }
          }
        } else {
          int64_t sp = 0;
          stack[sp++] = 0;
          while (sp > 0) {
            int64_t k = stack[--sp];
            double Lk = (kind == 0) ? len[i] : (len[i] > lmax[k] ? len[i] : lmax[k]);
            double R = 2.0 * Lk;
            if (!(box_point_d2(&t->bmin[3 * k], &t->bmax[3 * k], x[i], y[i], z[i], L) < R * R)) continue;
            if (t->nchild[k] == 0) {
              for (int64_t q = t->first[k]; q < t->first[k] + t->count[k]; q++) {
                int64_t j = t->perm[q];
                if (kind != 2 && j >= n_gas) continue;
                if (kind != 0 && j == i) continue;
                double r2 = pair_r2(x[i], y[i], z[i], x[j], y[j], z[j], L);
                double Lp = (kind == 0) ? len[i] : (len[i] > len[j] ? len[i] : len[j]);
                double Rp = 2.0 * Lp;
                if (r2 < Rp * Rp) { if (pass) idx[base + c] = j; c++; }
              }
            } else {
              for (int32_t b = t->nchild[k] - 1; b >= 0; b--) stack[sp++] = t->child[k] + b;
            }
          }
        }
        if (pass) qsort(idx + base, c, sizeof(int64_t), cmp_i64_int);
        else cnt[i] = c;
      }
      free(stack);
    }
    if (pass == 1) {
      free(cnt); free(lmax); orc_tree_free(t); free(wx); free(wy); free(wz);
      return total;
    }
  }
  return -1;
}

/* ===================================================================== */
/* Direct potential, integrator, time-step, diagnostics                    */
/* ===================================================================== */

/* Softened potential energy (Sect. 2.1, Eqs. Lagrangian, potential, Lgrav):
 * V = (G/2) sum_i sum_j m_i m_j phi(r_ij, eps_i), the j = i terms included.
 * phi is the negative kernel of Eq. (softphi), so V < 0 and L = T - V. */
double orc_potential_energy(int64_t n, const double *x, const double *y, const double *z,
                            const double *m, const double *eps, double G)
{
  double V = 0.0;
#pragma omp parallel for reduction(+ : V) schedule(static)
  for (int64_t i = 0; i < n; i++) {
    double s = 0.0;
    for (int64_t j = 0; j < n; j++) {
      double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
      s += m[j] * orc_phi(sqrt(dx * dx + dy * dy + dz * dz), eps[i]);
    }
    V += m[i] * s;
  }
  return 0.5 * G * V;
}

/* Kick-drift-kick leapfrog (Sect. 4.1).  phase 0: first half kick and drift,
 * plus the predicted end-of-step velocity v_n + a_n dt (and u_n + du_n dt)
 * used by the next force evaluation; phase 1: closing half kick. */
static double predict_factor(double dt, double divv)
{
  double f = 1.0 + (dt / 3.0) * divv;
  if (!(f >= 0.5)) f = 0.5;
  else if (f > 2.0) f = 2.0;
  return f;
}

void orc_kick_drift(int64_t n, int64_t n_gas, double dt, int32_t phase,
                    double *x, double *y, double *z, double *vx, double *vy, double *vz,
                    double *u, const double *ax, const double *ay, const double *az,
                    const double *dudt, double *vpx, double *vpy, double *vpz, double *up,
                    double *h, double *eps, const double *divv_h, const double *divv_e,
                    const double *xsx, const double *xsy, const double *xsz,
                    double *alpha, const double *dalpha, double alpha_min,
                    double *alpha_u, const double *dalpha_u, double alpha_u_min, double period)
{
  for (int64_t i = 0; i < n; i++) {
    if (phase == 0) {
      /* lengths along the drift: h n^(1/3) = eta with dn/dt = -n div v gives
       * dh/dt = (h/3) div v (Sect. 2.1); a starting value for the next solve */
      if (h && divv_h && i < n_gas && h[i] > 0.0) h[i] *= predict_factor(dt, divv_h[i]);
      if (eps && divv_e && eps[i] > 0.0) eps[i] *= predict_factor(dt, divv_e[i]);
      if (vpx) { vpx[i] = vx[i] + dt * ax[i]; vpy[i] = vy[i] + dt * ay[i]; vpz[i] = vz[i] + dt * az[i]; }
      vx[i] += 0.5 * dt * ax[i];
      vy[i] += 0.5 * dt * ay[i];
      vz[i] += 0.5 * dt * az[i];
      if (xsx && i < n_gas) {
        /* X-SPH (Sect. 3.5, Eq. xsph): the particle drifts with the smoothed
         * velocity v + dv of the last force evaluation */
        x[i] += dt * (vx[i] + xsx[i]);
        y[i] += dt * (vy[i] + xsy[i]);
        z[i] += dt * (vz[i] + xsz[i]);
      } else {
        x[i] += dt * vx[i];
        y[i] += dt * vy[i];
        z[i] += dt * vz[i];
      }
      if (period > 0.0) {
        /* back into the periodic box */
        x[i] -= period * floor(x[i] / period);
        y[i] -= period * floor(y[i] / period);
        z[i] -= period * floor(z[i] / period);
      }
      if (i < n_gas) {
        if (up) up[i] = u[i] + dt * dudt[i];
        u[i] += 0.5 * dt * dudt[i];
      }
    } else {
      vx[i] += 0.5 * dt * ax[i];
      vy[i] += 0.5 * dt * ay[i];
      vz[i] += 0.5 * dt * az[i];
      if (i < n_gas) u[i] += 0.5 * dt * dudt[i];
    }
    /* the dissipation coefficients follow the half kicks with the rates of
     * the last force evaluation, kept at or above their floors */
    if (i < n_gas && alpha && dalpha) {
      alpha[i] += 0.5 * dt * dalpha[i];
      if (!(alpha[i] >= alpha_min)) alpha[i] = alpha_min;
    }
    if (i < n_gas && alpha_u && dalpha_u) {
      alpha_u[i] += 0.5 * dt * dalpha_u[i];
      if (!(alpha_u[i] >= alpha_u_min)) alpha_u[i] = alpha_u_min;
    }
  }
}

/* Global time-step (Sect. 4.2): min over particles of the acceleration,
 * Courant and thermal-energy criteria, all with the same eta. */
double orc_timestep(const orc_params *p, int64_t n, int64_t n_gas, const double *vx,
                    const double *vy, const double *vz, const double *u, const double *h,
                    const double *eps, const double *ax, const double *ay, const double *az,
                    const double *dudt, const double *divv, const double *maxmu, double eta_dt,
                    const double *rho, const double *alpha)
{
  return orc_timestep_each(p, n, n_gas, vx, vy, vz, u, h, eps, ax, ay, az, dudt, divv, maxmu, eta_dt, rho, alpha,
                           NULL);
}

/* The same criteria per particle (dt_out[i], INFINITY when none applies);
 * returns their minimum. */
double orc_timestep_each(const orc_params *p, int64_t n, int64_t n_gas, const double *vx,
                         const double *vy, const double *vz, const double *u, const double *h,
                         const double *eps, const double *ax, const double *ay, const double *az,
                         const double *dudt, const double *divv, const double *maxmu, double eta_dt,
                         const double *rho, const double *alpha, double *dt_out)
{
  (void)vx; (void)vy; (void)vz;
  double dt_min = INFINITY;
  for (int64_t i = 0; i < n; i++) {
    double dt = INFINITY;
    double amag = sqrt(ax[i] * ax[i] + ay[i] * ay[i] + az[i] * az[i]);
    /* min(eps, h) over the lengths the particle has: a softening that is
     * not positive (no gravity) drops out */
    double len = (eps && eps[i] > 0.0) ? eps[i] : INFINITY;
    if (i < n_gas && h && h[i] < len) len = h[i];
    if (amag > 0.0 && len < INFINITY) {
      double t = eta_dt * sqrt(len / amag);
      if (t < dt) dt = t;
    }
    if (i < n_gas && p->hydro) {
      /* with the entropy variable A (Sect. 3.4): c^2 = gamma A rho^(gamma - 1),
       * and the last criterion bounds the change of A */
      double c = p->entropy ? sqrt(p->gamma * u[i] * pow(rho[i], p->gamma - 1.0))
                            : sqrt(p->gamma * (p->gamma - 1.0) * u[i]);
      double al = alpha ? alpha[i] : p->alpha;
      double den = h[i] * fabs(divv[i]) + c + 1.2 * (al * c + p->beta * maxmu[i]);
      if (den > 0.0) {
        double t = eta_dt * h[i] / den;
        if (t < dt) dt = t;
      }
      if (dudt[i] != 0.0) {
        double t = eta_dt * fabs(u[i] / dudt[i]);
        if (t < dt) dt = t;
      }
    }
    if (dt_out) dt_out[i] = dt;
    if (dt < dt_min) dt_min = dt;
  }
  return dt_min;
}

void orc_diagnostics(int64_t n, int64_t n_gas, const double *x, const double *y, const double *z,
                     const double *vx, const double *vy, const double *vz, const double *m,
                     const double *u, const double *pot, double *out,
                     const double *rho, double gamma, int32_t entropy)
{
  double ek = 0, eth = 0, V = 0, P[3] = {0, 0, 0}, L[3] = {0, 0, 0};
  for (int64_t i = 0; i < n; i++) {
    ek += 0.5 * m[i] * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]);
    /* u = A rho^(gamma - 1) / (gamma - 1) with the entropy variable (Sect. 3.4) */
    if (i < n_gas && u) eth += m[i] * (entropy ? u[i] * pow(rho[i], gamma - 1.0) / (gamma - 1.0) : u[i]);
    if (pot) V += 0.5 * m[i] * pot[i];
    P[0] += m[i] * vx[i];
    P[1] += m[i] * vy[i];
    P[2] += m[i] * vz[i];
    L[0] += m[i] * (y[i] * vz[i] - z[i] * vy[i]);
    L[1] += m[i] * (z[i] * vx[i] - x[i] * vz[i]);
    L[2] += m[i] * (x[i] * vy[i] - y[i] * vx[i]);
  }
  out[0] = ek; out[1] = eth; out[2] = V;
  out[3] = P[0]; out[4] = P[1]; out[5] = P[2];
  out[6] = L[0]; out[7] = L[1]; out[8] = L[2];
}

/* batch evaluation of the kernel functions for the tests:
 * which 0 W, 1 dW/dr, 2 dW/dh, 3 TC92 dW/dr, 4 phi, 5 dphi/dr, 6 dphi/deps */
void orc_eval_kernel(int which, int64_t n, const double *r, const double *h, double *out)
{
  for (int64_t i = 0; i < n; i++) {
    double v = 0.0;
    switch (which) {
      case 0: v = orc_W(r[i], h[i]); break;
      case 1: v = orc_dWdr(r[i], h[i]); break;
      case 2: v = orc_dWdh(r[i], h[i]); break;
      case 3: v = orc_dWdr_tc92(r[i], h[i]); break;
      case 4: v = orc_phi(r[i], h[i]); break;
      case 5: v = orc_dphidr(r[i], h[i]); break;
      case 6: v = orc_dphideps(r[i], h[i]); break;
      default: v = NAN;
    }
    out[i] = v;
  }
}

/* Field of a particle set at a point through its node expansion (monopole,
 * plus the quadrupole when asked) -- the far-field arm of the walk, exposed so
 * that its error order can be checked against the direct sum. */
void orc_multipole_field(int64_t n, const double *x, const double *y, const double *z,
                         const double *m, double px, double py, double pz, int32_t quadrupole,
                         double *acc, double *pot)
{
  orc_tree *t = orc_tree_build(n, x, y, z, m, 1 << 30);
  orc_params P;
  memset(&P, 0, sizeof(P));
  P.G = 1.0;
  P.quadrupole = quadrupole;
  ctx_t Cx;
  memset(&Cx, 0, sizeof(Cx));
  Cx.p = &P;
  Cx.t = t;
  double a[3] = {0, 0, 0}, ph = 0.0;
  far_node(&Cx, 0, px, py, pz, a, &ph);
  acc[0] = a[0]; acc[1] = a[1]; acc[2] = a[2];
  *pot = ph;
  orc_tree_free(t);
}
