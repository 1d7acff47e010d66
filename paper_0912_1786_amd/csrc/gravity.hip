// gravity.hip -- Barnes-Hut walk with quadrupoles, the symmetrised spline
// softening and the adaptive-softening correction terms.
//
// Merlin et al., arXiv:0912.1786: Sect. 2.1 (Eqs. softforce, softphi,
// dLgravdr, zeta), Sect. 2.2 (tree walk with monopole + quadrupole, Dubinski
// criterion Eq. opcrit), App. B.
//
// One wavefront per walk group.  The wave pops up to 64 nodes at a time from
// an LDS stack, tests each against the group's bounding box (opening radius
// l/theta + delta from the centre of mass, and no particle of the node within
// the softening reach 2 max(eps) of the group), and appends accepted nodes and
// opened leaves to LDS lists.  Full lists are flushed through an LDS tile:
// the lanes load 64 node (or particle) records at once with vector loads,
// then every lane (sink) evaluates every staged interaction from broadcast
// LDS reads.  Accepted nodes act unsoftened
// through their monopole and quadrupole; particles of opened leaves interact
// through
//   a_i -= G m_j 1/2 [phi'(r, eps_i) + phi'(r, eps_j)] r_hat
//   a_i -= G/2 [xi_i/Ups_i W'(r, eps_i) + (m_j/m_i) xi_j/Ups_j W'(r, eps_j)] r_hat
// (r_hat = (x_i - x_j)/r, xi carrying the neighbour masses).
#include <stdio.h>

#include <type_traits>

#include "tsph_internal.h"

namespace tsph {

constexpr int kGStackCap = 1024;
constexpr int kGListCap = 192;  // below a flush threshold (64) plus one round (128)
constexpr int kGCellFlush = 64;
constexpr int kGLeafFlush = 32;
constexpr int kGSplitFlush = 64;  // near entries collected before a hand-off
constexpr double kInvPiG = 0.31830988618379067154;

struct GravArgs {
  int64_t cap_n;
  const uint8_t *act;  // key order: evaluate chunks holding one of these only (NULL: all)
  const int32_t *groups;
  const int32_t *ngroups;
  const int2 *batches;
  const int32_t *nbatches;
  const int32_t *nngas;
  Members mem;
  const NodeTopo *topo;
  const NodeBox *nbox;
  const NodeFar *nfar;
  const GravRec *grec;
  const int32_t *perm;
  const int32_t *nnodes;
  double *acc;
  int32_t *cnt;
  int32_t *work;
  uint32_t *flags;
  int32_t *dbg;
  int32_t dbg_max;
  const double2 *nsoft;  // softened cells: per node sum of m eps, sum of m xi/Upsilon
  double G;
  int32_t quadrupole, corr, want_pot;
  int32_t lit;     // correction terms with the printed mass weighting
  int32_t soften;  // softened cells
  // near-field hand-off (0 split_particles: none)
  int32_t split_particles;
  int64_t split_cap;
  int2 *split_rng;
  SplitItem *split_item;
  double4 *split_part;
  int32_t *split_head;
  double L;           // periodic box side (0: open)
  const double *ewt;  // its Ewald correction table
  const float4 *ewt32;  // the table in single precision (FP32-bulk walks)
};

struct Sink {
  double x, y, z, m, im, eps, ieps, xiu;
  double s4;  // (2 eps)^2: the squared softening reach of a pair is the larger s4
  double ax, ay, az, pot;
  int p;
  bool act;
  int32_t *dbg;
  int ndbg;
};

// kernel variants: bit 0 quadrupoles, bit 1 correction terms, bit 2
// potential, bit 3 periodic box
constexpr int kQuad = 1, kCorr = 2, kPot = 4, kPer = 8;

// ---- periodic box (Sect. 4.3): the correction for the replicas of a mass,
// tabulated for omega = 2/L, |n|, |h| < 5 on [0, L/2]^3 with kEwaldGrid
// intervals per axis, interpolated trilinearly on |x_k|; the component takes
// the sign of x_k (odd in its own coordinate, even in the others).
__device__ __forceinline__ void ewald_corr(const double *__restrict__ T, double L, double x, double y, double z,
                                           double &ex, double &ey, double &ez) {
#pragma clang fp contract(off)
  constexpr int n1 = kEwaldGrid + 1;
  const double step = 0.5 * L / kEwaldGrid;
  const double a[3] = {fabs(x), fabs(y), fabs(z)};
  int i[3];
  double f[3];
#pragma unroll
  for (int d = 0; d < 3; d++) {
    const double u = a[d] / step;
    int k = (int)floor(u);
    k = k > kEwaldGrid - 1 ? kEwaldGrid - 1 : (k < 0 ? 0 : k);
    i[d] = k;
    f[d] = u - k;
  }
  double v0 = 0.0, v1 = 0.0, v2 = 0.0;
#pragma unroll
  for (int b = 0; b < 8; b++) {
    const int ox = b >> 2, oy = (b >> 1) & 1, oz = b & 1;
    const double w = (ox ? f[0] : 1.0 - f[0]) * (oy ? f[1] : 1.0 - f[1]) * (oz ? f[2] : 1.0 - f[2]);
    const double *t = T + 3 * (((int64_t)(i[0] + ox) * n1 + (i[1] + oy)) * n1 + (i[2] + oz));
    v0 = v0 + w * t[0];
    v1 = v1 + w * t[1];
    v2 = v2 + w * t[2];
  }
  ex = x < 0.0 ? -v0 : v0;
  ey = y < 0.0 ? -v1 : v1;
  ez = z < 0.0 ? -v2 : v2;
}

// the replicas of mass m at displacement (x_i - x_j) added to a sink's
// acceleration (times g: G in the FP64 form, 1 in the FP32 form's units)
template <class S>
__device__ __forceinline__ void ewald_add(const GravArgs &A, S &s, double g, double m, double dx, double dy,
                                          double dz) {
#pragma clang fp contract(off)
  double ex, ey, ez;
  ewald_corr(A.ewt, A.L, dx, dy, dz, ex, ey, ez);
  const double gm = g * m;
  s.ax = s.ax + gm * ex;
  s.ay = s.ay + gm * ey;
  s.az = s.az + gm * ez;
}

// The FP32-bulk form of ewald_add: the table in single precision, one
// 16-byte record per grid point (a third of the loads of the FP64 table),
// the interpolation in single precision, added to the sink's tile sums.
// Records of the table's corner (kEwaldNear points per axis from the
// origin) that the periodic FP32 walks keep in LDS: a wave whose lanes all
// interpolate inside it (near pairs, close nodes) reads them there instead
// of gathering from global memory; a wave whose lanes share one cell reads
// its eight records as scalars.  Same records, same arithmetic.
constexpr int kEwaldNear = 4;
constexpr int kEwaldNearRecs = kEwaldNear * kEwaldNear * kEwaldNear;

template <class S>
__device__ __forceinline__ void ewald_add32(const GravArgs &A, S &s, float m, float x, float y, float z) {
  constexpr int n1 = kEwaldGrid + 1;
  const float istep = (float)(kEwaldGrid / (0.5 * A.L));
  const float a[3] = {fabsf(x), fabsf(y), fabsf(z)};
  int i[3];
  float f[3];
#pragma unroll
  for (int d = 0; d < 3; d++) {
    const float u = a[d] * istep;
    int k = (int)floorf(u);
    k = k > kEwaldGrid - 1 ? kEwaldGrid - 1 : (k < 0 ? 0 : k);
    i[d] = k;
    f[d] = u - (float)k;
  }
  float v0 = 0.0f, v1 = 0.0f, v2 = 0.0f;
  // one cell for the whole wave (a node far from a compact batch): the
  // corner records are wave-uniform and come through the scalar cache
  const int c0 = __builtin_amdgcn_readfirstlane(i[0]), c1 = __builtin_amdgcn_readfirstlane(i[1]),
            c2 = __builtin_amdgcn_readfirstlane(i[2]);
  const bool corner = i[0] < kEwaldNear - 1 && i[1] < kEwaldNear - 1 && i[2] < kEwaldNear - 1;
  if (__all(i[0] == c0 && i[1] == c1 && i[2] == c2)) {
    const float4 *cell = A.ewt32 + (c0 * n1 + c1) * n1 + c2;
#pragma unroll
    for (int b = 0; b < 8; b++) {
      const int ox = b >> 2, oy = (b >> 1) & 1, oz = b & 1;
      const float w = (ox ? f[0] : 1.0f - f[0]) * (oy ? f[1] : 1.0f - f[1]) * (oz ? f[2] : 1.0f - f[2]);
      const float4 t = sload(cell + (ox * n1 + oy) * n1 + oz);
      v0 += w * t.x;
      v1 += w * t.y;
      v2 += w * t.z;
    }
  } else if (__all(corner)) {
#pragma unroll
    for (int b = 0; b < 8; b++) {
      const int ox = b >> 2, oy = (b >> 1) & 1, oz = b & 1;
      const float w = (ox ? f[0] : 1.0f - f[0]) * (oy ? f[1] : 1.0f - f[1]) * (oz ? f[2] : 1.0f - f[2]);
      const float4 t = s.ew[((i[0] + ox) * kEwaldNear + (i[1] + oy)) * kEwaldNear + (i[2] + oz)];
      v0 += w * t.x;
      v1 += w * t.y;
      v2 += w * t.z;
    }
  } else {
#pragma unroll
    for (int b = 0; b < 8; b++) {
      const int ox = b >> 2, oy = (b >> 1) & 1, oz = b & 1;
      const float w = (ox ? f[0] : 1.0f - f[0]) * (oy ? f[1] : 1.0f - f[1]) * (oz ? f[2] : 1.0f - f[2]);
      const float4 t = A.ewt32[((i[0] + ox) * n1 + (i[1] + oy)) * n1 + (i[2] + oz)];
      v0 += w * t.x;
      v1 += w * t.y;
      v2 += w * t.z;
    }
  }
  s.tax += m * (x < 0.0f ? -v0 : v0);
  s.tay += m * (y < 0.0f ? -v1 : v1);
  s.taz += m * (z < 0.0f ? -v2 : v2);
}

// The table's corner records into LDS (the whole wave; the caller's next
// barrier publishes them).
__device__ __forceinline__ void ewald_near_fill(const GravArgs &A, float4 *ew) {
  constexpr int n1 = kEwaldGrid + 1;
  for (int r = __lane_id(); r < kEwaldNearRecs; r += kWave) {
    const int a = r / (kEwaldNear * kEwaldNear), b = (r / kEwaldNear) % kEwaldNear, c = r % kEwaldNear;
    ew[r] = A.ewt32[(a * n1 + b) * n1 + c];
  }
}

// the single-precision copy of the table, (x, y, z, 0) per grid point
__global__ __launch_bounds__(256) void k_ewald_pack(const double *__restrict__ T, float4 *__restrict__ T32) {
  constexpr int n = (kEwaldGrid + 1) * (kEwaldGrid + 1) * (kEwaldGrid + 1);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) T32[i] = make_float4((float)T[3 * i], (float)T[3 * i + 1], (float)T[3 * i + 2], 0.0f);
}

// one thread per grid point: the Ewald sums (real space over |n| < 5 with
// erfc and the Gaussian, Fourier space over 0 < |h| < 5) less the direct
// term, the coordinate planes of each component set to zero by symmetry
__global__ __launch_bounds__(256) void k_ewald_table(double L, double *__restrict__ T) {
  constexpr int n1 = kEwaldGrid + 1;
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n1 * n1 * n1) return;
  const int i = a / (n1 * n1), j = (a / n1) % n1, k = a % n1;
  const double step = 0.5 * L / kEwaldGrid;
  const double x = i * step, y = j * step, z = k * step;
  double ax = 0.0, ay = 0.0, az = 0.0;
  if (a > 0) {
    const double w = 2.0 / L;
    const double r2 = x * x + y * y + z * z, r = sqrt(r2);
    ax = x / (r2 * r);
    ay = y / (r2 * r);
    az = z / (r2 * r);
    for (int nx = -4; nx <= 4; nx++)
      for (int ny = -4; ny <= 4; ny++)
        for (int nz = -4; nz <= 4; nz++) {
          if (nx * nx + ny * ny + nz * nz >= 25) continue;
          const double dx = x - nx * L, dy = y - ny * L, dz = z - nz * L;
          const double d2 = dx * dx + dy * dy + dz * dz, d = sqrt(d2);
          const double g = (erfc(w * d) + 2.0 * w * d * (1.0 / sqrt(M_PI)) * exp(-w * w * d2)) / (d2 * d);
          ax -= dx * g;
          ay -= dy * g;
          az -= dz * g;
        }
    for (int hx = -4; hx <= 4; hx++)
      for (int hy = -4; hy <= 4; hy++)
        for (int hz = -4; hz <= 4; hz++) {
          const int h2 = hx * hx + hy * hy + hz * hz;
          if (h2 == 0 || h2 >= 25) continue;
          const double c = 2.0 / (L * L) / h2 * exp(-M_PI * M_PI * h2 / (w * w * L * L)) *
                           sin(2.0 * M_PI / L * (hx * x + hy * y + hz * z));
          ax -= c * hx;
          ay -= c * hy;
          az -= c * hz;
        }
  }
  T[3 * a + 0] = i == 0 ? 0.0 : ax;
  T[3 * a + 1] = j == 0 ? 0.0 : ay;
  T[3 * a + 2] = k == 0 ? 0.0 : az;
}

template <int M>
__device__ __forceinline__ void far_field(const GravArgs &A, Sink &s, const NodeFar &f) {
  double dx = s.x - f.cx, dy = s.y - f.cy, dz = s.z - f.cz;
  if (M & kPer) {
    dx = wrap_d(dx, A.L);
    dy = wrap_d(dy, A.L);
    dz = wrap_d(dz, A.L);
    ewald_add(A, s, A.G, f.m, dx, dy, dz);
  }
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double ir = rsq64(r2);
  const double ir2 = ir * ir;
  const double ir3 = ir * ir2;
  if (M & kQuad) {
    const double qx = f.qxx * dx + f.qxy * dy + f.qxz * dz;
    const double qy = f.qxy * dx + f.qyy * dy + f.qyz * dz;
    const double qz = f.qxz * dx + f.qyz * dy + f.qzz * dz;
    const double rqr = dx * qx + dy * qy + dz * qz;
    const double ir5 = ir3 * ir2;
    const double t = rqr * (ir2 * ir2);  // r.Q.r / r^4
    // a = G [Q.r / r^5 - (m + 5/2 r.Q.r / r^4) r / r^3], as fused steps
    const double fm = ir3 * fma(2.5, t, f.m);
    s.ax = fma(A.G, fma(qx, ir5, -fm * dx), s.ax);
    s.ay = fma(A.G, fma(qy, ir5, -fm * dy), s.ay);
    s.az = fma(A.G, fma(qz, ir5, -fm * dz), s.az);
    if (M & kPot) s.pot -= A.G * (ir * fma(0.5, t, f.m));
  } else {
    const double fm = A.G * f.m * ir3;
    s.ax = fma(-fm, dx, s.ax);
    s.ay = fma(-fm, dy, s.ay);
    s.az = fma(-fm, dz, s.az);
    if (M & kPot) s.pot -= A.G * f.m * ir;
  }
}

template <int M>
__device__ __forceinline__ void near_pair(const GravArgs &A, Sink &s, const GravRec &b) {
  double dx = s.x - b.x, dy = s.y - b.y, dz = s.z - b.z;
  if (M & kPer) {
    dx = wrap_d(dx, A.L);
    dy = wrap_d(dy, A.L);
    dz = wrap_d(dz, A.L);
  }
  const double r2 = dx * dx + dy * dy + dz * dz;
  if (r2 >= fmax(s.s4, b.s4)) {
    const double ir = rsq64(r2);
    const double mr = b.m * ir;
    const double f = A.G * mr * ir * ir;
    s.ax -= f * dx;
    s.ay -= f * dy;
    s.az -= f * dz;
    if (M & kPot) s.pot -= A.G * mr;
    return;
  }
  if (r2 > 0.0) {
    const double ir = rsq64(r2);
    const double r = r2 * ir;
    const double qi = r * s.ieps, qj = r * b.ieps;
    double F = 0.5 * b.m * (soft_fr_q(qi, s.ieps, ir) + soft_fr_q(qj, b.ieps, ir));
    if (M & kCorr) {
      const double ii2 = s.ieps * s.ieps, ij2 = b.ieps * b.ieps;
      const double Wi = m4_dw(qi) * (ii2 * ii2) * kInvPiG;
      const double Wj = m4_dw(qj) * (ij2 * ij2) * kInvPiG;
      if (A.lit)
        F += 0.5 * b.m * (s.xiu * Wi + b.xiu * Wj);
      else
        F += 0.5 * (s.xiu * Wi + (b.m * s.im) * b.xiu * Wj);
    }
    const double fr = A.G * F * ir;
    s.ax -= fr * dx;
    s.ay -= fr * dy;
    s.az -= fr * dz;
    if (M & kPot) s.pot += A.G * b.m * 0.5 * (soft_ph_q(qi, s.ieps, ir) + soft_ph_q(qj, b.ieps, ir));
  } else if (M & kPot) {
    s.pot += A.G * b.m * 0.5 * (-1.4 * s.ieps - 1.4 * b.ieps);
  }
}

// Softened cell acting on a sink (Sect. 2.2): the node as one particle of
// mass M at its centre of mass, softened with the mass-weighted mean eps of
// its particles, through the symmetrised pair; the correction terms of its
// particles gathered there: the sink's term once per particle (N times; with
// the printed weighting, M times), theirs as X = sum m xi/Upsilon.  Staged
// as a GravRec (x, y, z, M, eps, 1/eps, X, N).  The opening test keeps the
// cell's centre of mass away from every sink of the batch (r > 0).
template <int M>
__device__ __forceinline__ void soft_cell(const GravArgs &A, Sink &s, const GravRec &b) {
  double dx = s.x - b.x, dy = s.y - b.y, dz = s.z - b.z;
  if (M & kPer) {
    dx = wrap_d(dx, A.L);
    dy = wrap_d(dy, A.L);
    dz = wrap_d(dz, A.L);
    ewald_add(A, s, A.G, b.m, dx, dy, dz);
  }
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double ir = rsq64(r2);
  const double r = r2 * ir;
  const double qi = r * s.ieps, qj = r * b.ieps;
  double F = 0.5 * b.m * (soft_fr_q(qi, s.ieps, ir) + soft_fr_q(qj, b.ieps, ir));
  if (M & kCorr) {
    const double ii2 = s.ieps * s.ieps, ij2 = b.ieps * b.ieps;
    const double Wi = m4_dw(qi) * (ii2 * ii2) * kInvPiG;
    const double Wj = m4_dw(qj) * (ij2 * ij2) * kInvPiG;
    F += 0.5 * ((A.lit ? b.m : b.s4) * s.xiu * Wi + (A.lit ? 1.0 : s.im) * b.xiu * Wj);
  }
  const double fr = A.G * F * ir;
  s.ax -= fr * dx;
  s.ay -= fr * dy;
  s.az -= fr * dz;
  if (M & kPot) s.pot += A.G * b.m * 0.5 * (soft_ph_q(qi, s.ieps, ir) + soft_ph_q(qj, b.ieps, ir));
}

template <int M>
__device__ __forceinline__ void debug_pair(const GravArgs &A, Sink &s, const GravRec &b, int q) {
  const double r2 = (M & kPer)
                        ? dist2_disp(wrap_d(s.x - b.x, A.L), wrap_d(s.y - b.y, A.L), wrap_d(s.z - b.z, A.L))
                        : dist2_pair(s.x, s.y, s.z, b.x, b.y, b.z);
  const double R = 2.0 * fmax(s.eps, b.eps);
  if (r2 < R * R) {
    if (s.ndbg < A.dbg_max) s.dbg[s.ndbg] = A.perm[q];
    s.ndbg++;
  }
}

// Evaluates the nt particle records staged in rec (indices in tq) on sink s.
// First every pair of the tile as a Newtonian pair, in tile order, with the
// pairs inside 2 max(eps) (and the self pair) given zero weight; each lane
// notes those in a mask and then evaluates only its own softened pairs, in
// tile order.  The wave thus does not run the softened formula for a pair
// that only some other lane needs.
template <int M>
__device__ __forceinline__ void near_tile(const GravArgs &A, Sink &s, const GravRec *rec, const int *tq, int nt) {
  uint64_t soft = tile_mask(nt, [&](int j) {
    const GravRec b = rec[j];
    double dx = s.x - b.x, dy = s.y - b.y, dz = s.z - b.z;
    if (M & kPer) {
      // every pair: the replicas (none for the sink itself, at x = 0)
      dx = wrap_d(dx, A.L);
      dy = wrap_d(dy, A.L);
      dz = wrap_d(dz, A.L);
      ewald_add(A, s, A.G, b.m, dx, dy, dz);
    }
    const double r2 = dx * dx + dy * dy + dz * dz;
    const bool near = r2 < fmax(s.s4, b.s4);
    const double ir = near ? 0.0 : rsq64(r2);
    const double mr = b.m * ir;
    const double f = A.G * mr * ir * ir;
    s.ax -= f * dx;
    s.ay -= f * dy;
    s.az -= f * dz;
    if (M & kPot) s.pot -= A.G * mr;
    if (s.dbg && tq[j] != s.p) debug_pair<M>(A, s, b, tq[j]);
    return near;
  });
  while (soft) {
    const int j = __builtin_ctzll(soft);
    soft &= soft - 1;
    if (tq[j] != s.p) near_pair<M>(A, s, rec[j]);
  }
}

// ---- FP32-bulk form: interactions in single precision on coordinates
// relative to the batch centre, partial sums per staged tile in single
// precision carried into double-precision totals after every tile.


// fmaxf of two non-negative floats, as the larger bit pattern (no NaN
// canonicalisation).  With s4 = (2 eps)^2 rounded, max(s4_i, s4_j) is the
// value 4 max(eps_i, eps_j)^2 rounds to: rounding the square is monotone,
// and both are the one rounding of the exact 4 max(eps)^2.
__device__ __forceinline__ float max_nonneg(float a, float b) {
  return __uint_as_float(max(__float_as_uint(a), __float_as_uint(b)));
}

// node record staged for the FP32 form (48 B): COM relative to the batch
// centre, mass, traceless quadrupole
struct alignas(16) NodeF32 {
  float cx, cy, cz, m;
  float qxx, qyy, qzz, qxy;
  float qxz, qyz, pad0, pad1;
};

// particle record staged for the FP32 form (32 B)
struct alignas(16) RecF32 {
  float x, y, z, m;
  float eps, ieps, xiu, s4;  // s4 = (2 eps)^2
};

// LDS staging tiles of the two forms
union Tile64 {
  NodeFar far[kWave];
  GravRec rec[kWave];
};
union Tile32 {
  NodeF32 far32[kWave];
  RecF32 rec32[kWave];
};

struct Sink32 {
  float x, y, z, m, im, eps, ieps, xiu;  // position relative to the batch centre
  float s4;                              // (2 eps)^2
  float tax, tay, taz, tpot;             // sums over the current tile
  double ax, ay, az, pot;                // totals (in units of G)
  const float4 *ew;                      // periodic box: the table's first kEwaldNear^3 records in LDS
  int p;
  bool act;
};

__device__ __forceinline__ void carry_tile(Sink32 &s) {
  s.ax += (double)s.tax;
  s.ay += (double)s.tay;
  s.az += (double)s.taz;
  s.pot += (double)s.tpot;
  s.tax = s.tay = s.taz = s.tpot = 0.0f;
}

// nearest image of an FP32 displacement (periodic box of side Lf)
__device__ __forceinline__ float wrap_f(float d, float Lf) { return d - Lf * rintf(d / Lf); }

template <int M>
__device__ __forceinline__ void far_field32(const GravArgs &A, Sink32 &s, const NodeF32 &f) {
  float dx = s.x - f.cx, dy = s.y - f.cy, dz = s.z - f.cz;
  if (M & kPer) {
    const float Lf = (float)A.L;
    dx = wrap_f(dx, Lf);
    dy = wrap_f(dy, Lf);
    dz = wrap_f(dz, Lf);
    ewald_add32(A, s, f.m, dx, dy, dz);
  }
  const float r2 = dx * dx + dy * dy + dz * dz;
  const float ir = rsq32(r2);
  const float ir2 = ir * ir;
  const float ir3 = ir * ir2;
  if (M & kQuad) {
    const float qx = f.qxx * dx + f.qxy * dy + f.qxz * dz;
    const float qy = f.qxy * dx + f.qyy * dy + f.qyz * dz;
    const float qz = f.qxz * dx + f.qyz * dy + f.qzz * dz;
    const float rqr = dx * qx + dy * qy + dz * qz;
    const float ir5 = ir3 * ir2;
    const float t = rqr * (ir2 * ir2);  // r.Q.r / r^4
    // a = Q.r / r^5 - (m + 5/2 r.Q.r / r^4) r / r^3, as fused steps
    const float fm = ir3 * fmaf(2.5f, t, f.m);
    s.tax = fmaf(qx, ir5, fmaf(-fm, dx, s.tax));
    s.tay = fmaf(qy, ir5, fmaf(-fm, dy, s.tay));
    s.taz = fmaf(qz, ir5, fmaf(-fm, dz, s.taz));
    if (M & kPot) s.tpot -= ir * fmaf(0.5f, t, f.m);
  } else {
    const float fm = f.m * ir3;
    s.tax = fmaf(-fm, dx, s.tax);
    s.tay = fmaf(-fm, dy, s.tay);
    s.taz = fmaf(-fm, dz, s.taz);
    if (M & kPot) s.tpot -= f.m * ir;
  }
}

template <int M>
__device__ __forceinline__ void newton_pair32(Sink32 &s, const RecF32 &b, float dx, float dy, float dz) {
  const float r2 = dx * dx + dy * dy + dz * dz;
  const float ir = rsq32(r2);
  const float mr = b.m * ir;
  const float f = mr * ir * ir;
  s.tax -= f * dx;
  s.tay -= f * dy;
  s.taz -= f * dz;
  if (M & kPot) s.tpot -= mr;
}

template <int M>
__device__ __forceinline__ void near_pair32(const GravArgs &A, Sink32 &s, const RecF32 &b, bool lit) {
  float dx = s.x - b.x, dy = s.y - b.y, dz = s.z - b.z;
  if (M & kPer) {
    const float Lf = (float)A.L;
    dx = wrap_f(dx, Lf);
    dy = wrap_f(dy, Lf);
    dz = wrap_f(dz, Lf);
  }
  const float r2 = dx * dx + dy * dy + dz * dz;
  if (r2 >= max_nonneg(s.s4, b.s4)) {
    newton_pair32<M>(s, b, dx, dy, dz);
    return;
  }
  if (r2 > 0.0f) {
    const float ir = rsq32(r2);
    const float r = r2 * ir;
    const float qi = r * s.ieps, qj = r * b.ieps;
    float F = 0.5f * b.m * (soft_fr_q(qi, s.ieps, ir) + soft_fr_q(qj, b.ieps, ir));
    if (M & kCorr) {
      const float ii2 = s.ieps * s.ieps, ij2 = b.ieps * b.ieps;
      const float Wi = m4_dw(qi) * (ii2 * ii2) * (float)kInvPiG;
      const float Wj = m4_dw(qj) * (ij2 * ij2) * (float)kInvPiG;
      if (lit)
        F += 0.5f * b.m * (s.xiu * Wi + b.xiu * Wj);
      else
        F += 0.5f * (s.xiu * Wi + (b.m * s.im) * b.xiu * Wj);
    }
    const float fr = F * ir;
    s.tax -= fr * dx;
    s.tay -= fr * dy;
    s.taz -= fr * dz;
    if (M & kPot) s.tpot += b.m * 0.5f * (soft_ph_q(qi, s.ieps, ir) + soft_ph_q(qj, b.ieps, ir));
  } else if (M & kPot) {
    s.tpot += b.m * 0.5f * (-1.4f * s.ieps - 1.4f * b.ieps);
  }
}

// soft_cell in the FP32 form (RecF32: x, y, z, M, eps, 1/eps, X, N)
template <int M>
__device__ __forceinline__ void soft_cell32(const GravArgs &A, Sink32 &s, const RecF32 &b, bool lit) {
  float dx = s.x - b.x, dy = s.y - b.y, dz = s.z - b.z;
  if (M & kPer) {
    const float Lf = (float)A.L;
    dx = wrap_f(dx, Lf);
    dy = wrap_f(dy, Lf);
    dz = wrap_f(dz, Lf);
    ewald_add32(A, s, b.m, dx, dy, dz);
  }
  const float r2 = dx * dx + dy * dy + dz * dz;
  const float ir = rsq32(r2);
  const float r = r2 * ir;
  const float qi = r * s.ieps, qj = r * b.ieps;
  float F = 0.5f * b.m * (soft_fr_q(qi, s.ieps, ir) + soft_fr_q(qj, b.ieps, ir));
  if (M & kCorr) {
    const float ii2 = s.ieps * s.ieps, ij2 = b.ieps * b.ieps;
    const float Wi = m4_dw(qi) * (ii2 * ii2) * (float)kInvPiG;
    const float Wj = m4_dw(qj) * (ij2 * ij2) * (float)kInvPiG;
    F += 0.5f * ((lit ? b.m : b.s4) * s.xiu * Wi + (lit ? 1.0f : s.im) * b.xiu * Wj);
  }
  const float fr = F * ir;
  s.tax -= fr * dx;
  s.tay -= fr * dy;
  s.taz -= fr * dz;
  if (M & kPot) s.tpot += b.m * 0.5f * (soft_ph_q(qi, s.ieps, ir) + soft_ph_q(qj, b.ieps, ir));
}

// As near_tile: Newtonian pass over the tile, then each lane's own
// softened pairs.
template <int M>
__device__ __forceinline__ void near_tile32(const GravArgs &A, Sink32 &s, const RecF32 *rec, const int *tq, int nt,
                                            bool lit) {
  uint64_t soft = tile_mask(nt, [&](int j) {
    const RecF32 b = rec[j];
    float dx = s.x - b.x, dy = s.y - b.y, dz = s.z - b.z;
    if (M & kPer) {
      // every pair: the replicas (none for the sink itself, at x = 0)
      const float Lf = (float)A.L;
      dx = wrap_f(dx, Lf);
      dy = wrap_f(dy, Lf);
      dz = wrap_f(dz, Lf);
      ewald_add32(A, s, b.m, dx, dy, dz);
    }
    const float r2 = dx * dx + dy * dy + dz * dz;
    const bool near = r2 < max_nonneg(s.s4, b.s4);
    const float ir = near ? 0.0f : rsq32(r2);
    const float mr = b.m * ir;
    const float f = mr * ir * ir;
    s.tax -= f * dx;
    s.tay -= f * dy;
    s.taz -= f * dz;
    if (M & kPot) s.tpot -= mr;
    return near;
  });
  while (soft) {
    const int j = __builtin_ctzll(soft);
    soft &= soft - 1;
    if (tq[j] != s.p) near_pair32<M>(A, s, rec[j], lit);
  }
}

// LDS staging tiles of the two forms
template <bool F32>
using TileT = typename std::conditional<F32, Tile32, Tile64>::type;
template <bool F32>
using SinkT = typename std::conditional<F32, Sink32, Sink>::type;

// Near-field entries: particle ranges (first, count), given as tree nodes
// (their particle range) or as explicit ranges.
struct NodeSrc {
  const NodeTopo *topo;
  const int *node;
  __device__ int2 operator()(int i) const {
    const NodeTopo t = topo[node[i]];
    return make_int2(t.first, t.count);
  }
};
struct RangeSrc {
  const int2 *rng;
  __device__ int2 operator()(int i) const { return rng[i]; }
};

// Near field of the entries [0, n) on sink s: their particles are packed 64
// to a tile while the entries are scanned in order (each lane noting the
// particle of its slot), loaded with one vector load per lane and evaluated
// by every lane.  Returns the number of particles visited.
template <int M, bool F32, class Src>
__device__ __forceinline__ int near_entries(const GravArgs &A, SinkT<F32> &s, const Src &src, int n, TileT<F32> &T,
                                            int *tq, double cx, double cy, double cz) {
  const int ln = lane();
  int fill = 0, rq = -1, visited = 0;
  auto flush = [&](int nt) {
    if (ln < nt) {
      const GravRec r = A.grec[rq];
      if constexpr (F32) {
        RecF32 h;
        h.x = (float)((M & kPer) ? wrap_d(r.x - cx, A.L) : r.x - cx); h.y = (float)((M & kPer) ? wrap_d(r.y - cy, A.L) : r.y - cy); h.z = (float)((M & kPer) ? wrap_d(r.z - cz, A.L) : r.z - cz);
        h.m = (float)r.m; h.eps = (float)r.eps; h.ieps = (float)r.ieps; h.xiu = (float)r.xiu;
        h.s4 = (2.0f * h.eps) * (2.0f * h.eps);
        T.rec32[ln] = h;
      } else {
        T.rec[ln] = r;
      }
      tq[ln] = rq;
    }
    __syncthreads();
    if constexpr (F32) {
      near_tile32<M>(A, s, T.rec32, tq, nt, A.lit != 0);
      carry_tile(s);
    } else {
      near_tile<M>(A, s, T.rec, tq, nt);
    }
    __syncthreads();
  };
  for (int c1 = 0; c1 < n; c1 += kWave) {
    const int nc = min(kWave, n - c1);
    const int2 my = ln < nc ? src(c1 + ln) : make_int2(0, 0);
    for (int j = 0; j < nc; j++) {
      const int first = __builtin_amdgcn_readlane(my.x, j);
      const int count = __builtin_amdgcn_readlane(my.y, j);
      visited += count;
      for (int off = 0; off < count;) {
        const int tk = min(count - off, kWave - fill);
        if (ln >= fill && ln < fill + tk) rq = first + off + (ln - fill);
        fill += tk;
        off += tk;
        if (fill == kWave) {
          flush(kWave);
          fill = 0;
        }
      }
    }
  }
  if (fill > 0) flush(fill);
  return visited;
}

// Every point of box b within distance r of box a (farthest-point test).
// A node passing it can only end as near pairs: each descendant's box gap
// to a is at most this distance, below 2 max(eps) of the softening test.
__device__ __forceinline__ bool box_within(const NodeBox &a, const NodeBox &b, double r) {
#pragma clang fp contract(off)
  const double ex = fmax(0.0, fmax(b.hix - a.hix, a.lox - b.lox));
  const double ey = fmax(0.0, fmax(b.hiy - a.hiy, a.loy - b.loy));
  const double ez = fmax(0.0, fmax(b.hiz - a.hiz, a.loz - b.loz));
  double d = ex * ex;
  d = d + ey * ey;
  d = d + ez * ez;
  return d < r * r;
}

// Loads sink chunk c0 of a batch (coordinates relative to the batch centre
// in the FP32 form).
template <bool F32>
__device__ __forceinline__ void load_sink(const GravArgs &A, SinkT<F32> &s, const NodeTopo &gnd, int c0, double cx,
                                          double cy, double cz, bool dbg) {
  const int ln = lane();
  s.act = c0 + ln < gnd.count;
  s.p = gnd.first + c0 + (s.act ? ln : 0);
  const GravRec r = A.grec[s.p];
  if constexpr (F32) {
    s.x = (float)(r.x - cx); s.y = (float)(r.y - cy); s.z = (float)(r.z - cz);
    s.m = (float)r.m; s.im = (float)(1.0 / r.m);
    s.eps = (float)r.eps; s.ieps = (float)r.ieps; s.xiu = (float)r.xiu;
    s.s4 = (2.0f * s.eps) * (2.0f * s.eps);
    s.tax = s.tay = s.taz = s.tpot = 0.0f;
  } else {
    s.x = r.x; s.y = r.y; s.z = r.z; s.m = r.m; s.im = 1.0 / r.m;
    s.eps = r.eps; s.ieps = r.ieps; s.xiu = r.xiu; s.s4 = r.s4;
    s.dbg = (dbg && A.dbg && s.act) ? A.dbg + ((int64_t)2 * A.cap_n + A.perm[s.p]) * A.dbg_max : nullptr;
    s.ndbg = 0;
  }
  s.ax = s.ay = s.az = s.pot = 0.0;
}

// Walk decision for node k (k < 0: none) of the batch with box gb: accepted
// as a far node (Dubinski radius cleared and the softening reach of batch and
// node apart), taken whole as near particles (a leaf, or a node lying within
// the softening reach of the batch), or opened.
struct GClass {
  bool acc, leaf, open, scell;
  int child, nchild;
};

template <int M>
__device__ __forceinline__ GClass classify(const GravArgs &A, const NodeBox &gb, double gemax, int k) {
  const double L = (M & kPer) ? A.L : 0.0;  // periodic box (folded away in the open kernels)
  GClass c{false, false, false, false, -1, 0};
  if (k < 0) return c;
  // all three records in one round trip (the topology is used only when the
  // node is not accepted)
  const NodeFar f = A.nfar[k];
  const NodeBox b = A.nbox[k];
  const NodeTopo nd = A.topo[k];
  double d2 = axis_gap_point_p(gb.lox, gb.hix, f.cx, L);
  d2 = d2 + axis_gap_point_p(gb.loy, gb.hiy, f.cy, L);
  d2 = d2 + axis_gap_point_p(gb.loz, gb.hiz, f.cz, L);
  if (d2 > f.rmac * f.rmac) {
    double c2 = axis_gap_box_p(gb.lox, gb.hix, b.lox, b.hix, L);
    c2 = c2 + axis_gap_box_p(gb.loy, gb.hiy, b.loy, b.hiy, L);
    c2 = c2 + axis_gap_box_p(gb.loz, gb.hiz, b.loz, b.hiz, L);
    const double sr = 2.0 * fmax(gemax, b.epsmax);
    c.acc = c2 >= sr * sr;
    // with softened cells, a node that passes the opening test inside the
    // softening reach acts as one softened particle
    c.scell = A.soften && !c.acc;
  }
  if (!c.acc && !c.scell) {
    // a node wholly inside the softening reach of the batch is taken whole:
    // all its particles are near pairs (unless a descendant may become a
    // softened cell)
    c.leaf = nd.nchild == 0 || (!A.soften && !(M & kPer) && box_within(gb, b, 2.0 * gemax));
    c.open = !c.leaf;
    c.child = nd.child;
    c.nchild = nd.nchild;
  }
  return c;
}

template <int M, bool F32>
__global__ __launch_bounds__(64, 3) void k_gravity(GravArgs A) {
  __shared__ int s_stack[kGStackCap];
  __shared__ int s_cell[kGListCap];
  __shared__ int s_leaf[kGListCap];
  __shared__ int s_scell[kGListCap];  // softened cells
  // staging tile: 64 node records (far flush) or 64 particle records (near
  // flush), filled with one vector load per lane and read back as broadcasts
  __shared__ TileT<F32> s_t;
  __shared__ int s_tq[kWave];
  __shared__ int s_g;
  __shared__ float4 s_ew[(F32 && (M & kPer)) ? kEwaldNearRecs : 1];
  const int ln = lane();
  const int ng = *A.nbatches;
  if constexpr (F32 && (M & kPer)) ewald_near_fill(A, s_ew);
  for (;;) {
    if (ln == 0) s_g = xcd_next(A.work + 16, ng);
    __syncthreads();
    const int g = s_g;
    __syncthreads();
    if (g < 0) break;
    const Batch bt = load_batch(A.batches, A.groups, A.topo, A.nbox, A.nngas, A.mem, g);
    const NodeTopo gnd{bt.first, bt.count, -1, 0};
    const NodeBox gb = bt.box;
    const double gemax = gb.epsmax;
    // batch centre: origin of the single-precision coordinates
    const double cx = 0.5 * (gb.lox + gb.hix), cy = 0.5 * (gb.loy + gb.hiy), cz = 0.5 * (gb.loz + gb.hiz);
    int prev_item = -1;  // last handed-off item of this batch
    for (int c0 = 0; c0 < gnd.count; c0 += kWave) {
      // individual time-steps: a chunk without an active sink is skipped
      if (A.act && ballot(c0 + ln < gnd.count && A.act[gnd.first + c0 + ln]) == 0) continue;
      SinkT<F32> s;
      load_sink<F32>(A, s, gnd, c0, cx, cy, cz, true);
      if constexpr (F32) s.ew = s_ew;
      int near_done = 0;  // near-field particles evaluated by this wave
      int nfar = 0, npair = 0;
      int sp = 1, ncell = 0, nleaf = 0, nscell = 0;
      bool overflow = false;
      int rounds = 0;
      const int guard = *A.nnodes + 2;
      if (ln == 0) s_stack[0] = bt.root;
      __syncthreads();

      for (;;) {
        if (sp > 0 && ++rounds > guard) {
          atomicOr(A.flags, TSPH_FLAG_INTERNAL);
          overflow = true;
        }
        if (sp > 0 && !overflow) {
          // up to two nodes per lane: the loads of both are in flight together
          const int take = walk_take(sp, kGStackCap, 2 * kWave);
          const int k0 = ln < take ? s_stack[sp - take + ln] : -1;
          const int k1 = ln + kWave < take ? s_stack[sp - take + kWave + ln] : -1;
          sp -= take;
          __syncthreads();
          const GClass c0 = classify<M>(A, gb, gemax, k0);
          const GClass c1 = classify<M>(A, gb, gemax, k1);
          uint64_t m = ballot(c0.acc);
          if (c0.acc) s_cell[ncell + mbcnt(m)] = k0;
          ncell += __popcll(m);
          m = ballot(c1.acc);
          if (c1.acc) s_cell[ncell + mbcnt(m)] = k1;
          ncell += __popcll(m);
          m = ballot(c0.scell);
          if (c0.scell) s_scell[nscell + mbcnt(m)] = k0;
          nscell += __popcll(m);
          m = ballot(c1.scell);
          if (c1.scell) s_scell[nscell + mbcnt(m)] = k1;
          nscell += __popcll(m);
          m = ballot(c0.leaf);
          if (c0.leaf) s_leaf[nleaf + mbcnt(m)] = k0;
          nleaf += __popcll(m);
          m = ballot(c1.leaf);
          if (c1.leaf) s_leaf[nleaf + mbcnt(m)] = k1;
          nleaf += __popcll(m);
          const int n0 = c0.open ? c0.nchild : 0, n1 = c1.open ? c1.nchild : 0;
          const int incl = wave_incl_scan(n0 + n1);
          const int tot = __shfl(incl, kWave - 1, kWave);
          if (sp + tot > kGStackCap) {
            overflow = true;
          } else {
            const int base = sp + incl - n0 - n1;
            for (int a = 0; a < n0; a++) s_stack[base + a] = c0.child + a;
            for (int a = 0; a < n1; a++) s_stack[base + n0 + a] = c1.child + a;
            sp += tot;
          }
          __syncthreads();
        }
        const bool last = (sp == 0) || overflow;
        if (ncell >= kGCellFlush || (last && ncell > 0)) {
          // accepted nodes, 64 per tile
          for (int t0 = 0; t0 < ncell; t0 += kWave) {
            const int nt = uniform(min(kWave, ncell - t0));
            if (ln < nt) {
              const NodeFar f = A.nfar[s_cell[t0 + ln]];
              if constexpr (F32) {
                NodeF32 h;
                h.cx = (float)((M & kPer) ? wrap_d(f.cx - cx, A.L) : f.cx - cx);
                h.cy = (float)((M & kPer) ? wrap_d(f.cy - cy, A.L) : f.cy - cy);
                h.cz = (float)((M & kPer) ? wrap_d(f.cz - cz, A.L) : f.cz - cz);
                h.m = (float)f.m;
                h.qxx = (float)f.qxx; h.qyy = (float)f.qyy; h.qzz = (float)f.qzz;
                h.qxy = (float)f.qxy; h.qxz = (float)f.qxz; h.qyz = (float)f.qyz;
                h.pad0 = h.pad1 = 0.0f;
                s_t.far32[ln] = h;
              } else {
                s_t.far[ln] = f;
              }
            }
            __syncthreads();
            if constexpr (F32) {
#pragma unroll 2
              for (int j = 0; j < nt; j++) far_field32<M>(A, s, s_t.far32[j]);
              carry_tile(s);
            } else {
              for (int j = 0; j < nt; j++) far_field<M>(A, s, s_t.far[j]);
            }
            __syncthreads();
          }
          nfar += ncell;
          ncell = 0;
        }
        if (nscell >= kGCellFlush || (last && nscell > 0)) {
          // softened cells, 64 per tile, staged as particle records
          for (int t0 = 0; t0 < nscell; t0 += kWave) {
            const int nt = uniform(min(kWave, nscell - t0));
            if (ln < nt) {
              const int k = s_scell[t0 + ln];
              const NodeFar f = A.nfar[k];
              const double2 ns = A.nsoft[k];
              const double e = ns.x / f.m;
              const double cntk = (double)A.topo[k].count;
              if constexpr (F32) {
                RecF32 h;
                h.x = (float)((M & kPer) ? wrap_d(f.cx - cx, A.L) : f.cx - cx);
                h.y = (float)((M & kPer) ? wrap_d(f.cy - cy, A.L) : f.cy - cy);
                h.z = (float)((M & kPer) ? wrap_d(f.cz - cz, A.L) : f.cz - cz);
                h.m = (float)f.m; h.eps = (float)e; h.ieps = (float)(1.0 / e); h.xiu = (float)ns.y;
                h.s4 = (float)cntk;
                s_t.rec32[ln] = h;
              } else {
                s_t.rec[ln] = GravRec{f.cx, f.cy, f.cz, f.m, e, 1.0 / e, ns.y, cntk};
              }
            }
            __syncthreads();
            if constexpr (F32) {
              for (int j = 0; j < nt; j++) soft_cell32<M>(A, s, s_t.rec32[j], A.lit != 0);
              carry_tile(s);
            } else {
              for (int j = 0; j < nt; j++) soft_cell<M>(A, s, s_t.rec[j]);
            }
            __syncthreads();
          }
          nfar += nscell;
          nscell = 0;
        }
        const bool splitting = A.split_particles > 0 && near_done >= A.split_particles;
        if (nleaf >= (splitting ? kGSplitFlush : kGLeafFlush) || (last && nleaf > 0)) {
          bool handed = false;
          int tot = 0;
          if (A.split_particles > 0) {
            for (int a = ln; a < nleaf; a += kWave) tot += A.topo[s_leaf[a]].count;
            tot = __shfl(wave_incl_scan(tot), kWave - 1, kWave);
          }
          if (A.split_particles > 0 && near_done + tot > A.split_particles) {
            // hand the entries to other wavefronts as items of at most
            // kSplitItemRanges ranges and kSplitItemParticles particles;
            // ranges and items for the worst case are reserved up front
            // an item closes at kSplitItemRanges ranges or kSplitItemParticles
            // particles, and ranges are cut only at the latter
            const int rmax = nleaf + tot / kSplitItemParticles + 1;
            const int imax = (rmax + kSplitItemRanges - 1) / kSplitItemRanges + tot / kSplitItemParticles + 1;
            int rbase = 0, ibase = 0;
            if (ln == 0) {
              rbase = atomicAdd(&A.work[3], rmax);
              ibase = rbase + rmax <= A.split_cap * kSplitItemRanges ? atomicAdd(&A.work[4], imax) : INT32_MAX;
            }
            rbase = __shfl(rbase, 0, kWave);
            ibase = __shfl(ibase, 0, kWave);
            if (ibase > A.split_cap - imax) {
              // capacity exhausted: the batch keeps these entries.  Item slots
              // reserved below the capacity are marked unused, since
              // k_gravity_split reads every slot up to the capacity.
              for (int64_t a = (int64_t)ibase + ln; a < A.split_cap; a += kWave)
                A.split_item[a] = SplitItem{-1, 0, 0, 0, -1, 0, 0, 0};
              if (ln == 0) atomicOr(A.flags, TSPH_FLAG_HANDOFF_CAPACITY);
            } else {
              handed = true;
              near_done += tot;
              npair += tot;
              int nr = 0, parts = 0, ri = 0, ii = 0;  // ranges of the open item, totals used
              for (int c1 = 0; c1 < nleaf; c1 += kWave) {
                const int nc = min(kWave, nleaf - c1);
                const NodeTopo my = ln < nc ? A.topo[s_leaf[c1 + ln]] : NodeTopo{0, 0, -1, 0};
                for (int j = 0; j < nc; j++) {
                  const int first = __builtin_amdgcn_readlane(my.first, j);
                  const int count = __builtin_amdgcn_readlane(my.count, j);
                  for (int off = 0; off < count;) {
                    const int tk = min(count - off, kSplitItemParticles - parts);
                    if (ln == 0) A.split_rng[rbase + ri + nr] = make_int2(first + off, tk);
                    nr++;
                    parts += tk;
                    off += tk;
                    if (nr == kSplitItemRanges || parts == kSplitItemParticles) {
                      const int it = ibase + ii;
                      if (ln == 0) {
                        A.split_item[it] = SplitItem{g, c0, rbase + ri, nr, -1, 0, 0, 0};
                        if (prev_item >= 0) A.split_item[prev_item].next = it;
                        else A.split_head[g] = it;
                      }
                      prev_item = it;
                      ri += nr;
                      ii++;
                      nr = 0;
                      parts = 0;
                    }
                  }
                }
              }
              if (nr > 0) {
                const int it = ibase + ii;
                if (ln == 0) {
                  A.split_item[it] = SplitItem{g, c0, rbase + ri, nr, -1, 0, 0, 0};
                  if (prev_item >= 0) A.split_item[prev_item].next = it;
                  else A.split_head[g] = it;
                }
                prev_item = it;
                ii++;
              }
              // reserved items left over stay empty
              for (int a = ii + ln; a < imax; a += kWave)
                A.split_item[ibase + a] = SplitItem{-1, 0, 0, 0, -1, 0, 0, 0};
            }
          }
          if (!handed) {
            const int v = near_entries<M, F32>(A, s, NodeSrc{A.topo, s_leaf}, nleaf, s_t, s_tq, cx, cy, cz);
            near_done += v;
            npair += v;
          }
          nleaf = 0;
        }
        __syncthreads();
        if (last) break;
      }
      if (overflow) atomicOr(A.flags, TSPH_FLAG_STACK_OVERFLOW);
      if constexpr (!F32) {
        if (s.dbg && s.ndbg > A.dbg_max) atomicOr(A.flags, TSPH_FLAG_LIST_OVERFLOW);
      }
      if (s.act) {
        double ax = s.ax, ay = s.ay, az = s.az, pot = s.pot;
        if constexpr (F32) {
          ax *= A.G;
          ay *= A.G;
          az *= A.G;
          pot *= A.G;
        }
        if (M & kPot) pot += A.G * (double)s.m * (-1.4 * (double)s.ieps);  // self term phi(0, eps_i)
        A.acc[0 * A.cap_n + s.p] = ax;
        A.acc[1 * A.cap_n + s.p] = ay;
        A.acc[2 * A.cap_n + s.p] = az;
        A.acc[3 * A.cap_n + s.p] = pot;
        const int ci = A.perm[s.p];
        A.cnt[0 * A.cap_n + ci] = nfar;
        A.cnt[1 * A.cap_n + ci] = npair - 1;
      }
    }
  }
}

// Handed-off near fields: one work item (a chunk of a batch's opened leaves)
// per wavefront; its partial acceleration and potential of the batch's sinks
// go to split_part, to be added in item order by k_split_reduce.
template <int M, bool F32>
__global__ __launch_bounds__(64) void k_gravity_split(GravArgs A) {
  __shared__ int2 s_rng[kSplitItemRanges];
  __shared__ TileT<F32> s_t;
  __shared__ int s_tq[kWave];
  __shared__ int s_g;
  __shared__ float4 s_ew[(F32 && (M & kPer)) ? kEwaldNearRecs : 1];
  const int ln = lane();
  const int nitems = min((int64_t)A.work[4], A.split_cap);
  if constexpr (F32 && (M & kPer)) ewald_near_fill(A, s_ew);
  for (;;) {
    if (ln == 0) s_g = atomicAdd(&A.work[5], 1);
    __syncthreads();
    const int it = s_g;
    __syncthreads();
    if (it >= nitems) break;
    const SplitItem I = A.split_item[it];
    if (I.g < 0) continue;  // reserved but unused
    const Batch bt = load_batch(A.batches, A.groups, A.topo, A.nbox, A.nngas, A.mem, I.g);
    const NodeTopo gnd{bt.first, bt.count, -1, 0};
    const NodeBox gb = bt.box;
    const double cx = 0.5 * (gb.lox + gb.hix), cy = 0.5 * (gb.loy + gb.hiy), cz = 0.5 * (gb.loz + gb.hiz);
    SinkT<F32> s;
    load_sink<F32>(A, s, gnd, I.c0, cx, cy, cz, false);
    if constexpr (F32) s.ew = s_ew;
    for (int a = ln; a < I.count; a += kWave) s_rng[a] = A.split_rng[I.start + a];
    __syncthreads();
    near_entries<M, F32>(A, s, RangeSrc{s_rng}, I.count, s_t, s_tq, cx, cy, cz);
    double4 part = make_double4(s.ax, s.ay, s.az, s.pot);
    if constexpr (F32) {
      part.x *= A.G;
      part.y *= A.G;
      part.z *= A.G;
      part.w *= A.G;
    }
    A.split_part[(int64_t)it * kWave + ln] = part;
  }
}

// Adds the handed-off partial sums to each batch's sinks, walking the batch's
// item chain in creation order (a fixed summation order).
__global__ __launch_bounds__(64) void k_split_reduce(GravArgs A) {
  const int ln = lane();
  const int ng = *A.nbatches;
  for (int g = blockIdx.x; g < ng; g += gridDim.x) {
    int it = A.split_head[g];
    if (it < 0) continue;
    const Batch bt = load_batch(A.batches, A.groups, A.topo, A.nbox, A.nngas, A.mem, g);
    int guard = 0;
    while (it >= 0 && it < A.split_cap && ++guard <= A.split_cap) {
      const SplitItem I = A.split_item[it];
      if (I.c0 + ln < bt.count) {
        const int64_t p = bt.first + I.c0 + ln;
        const double4 v = A.split_part[(int64_t)it * kWave + ln];
        A.acc[0 * A.cap_n + p] += v.x;
        A.acc[1 * A.cap_n + p] += v.y;
        A.acc[2 * A.cap_n + p] += v.z;
        A.acc[3 * A.cap_n + p] += v.w;
      }
      it = I.next;
    }
  }
}

__global__ __launch_bounds__(256) void k_zero_acc(int64_t n, int64_t cap_n, double *__restrict__ acc,
                                                  int32_t *__restrict__ cnt, const int32_t *__restrict__ perm) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    for (int k = 0; k < 4; k++) acc[k * cap_n + p] = 0.0;
    cnt[perm[p]] = 0;
    cnt[cap_n + perm[p]] = 0;
  }
}

}  // namespace tsph

using namespace tsph;

tsph_status tsph_impl_gravity(Ctx *c, bool want_pot, hipStream_t st) {
  if (!c->p.gravity) {
    hipLaunchKernelGGL(k_zero_acc, dim3(blocks_for(c->n, 256, 8192)), dim3(256), 0, st, c->n, c->cap_n, c->acc,
                       c->cnt, c->perm);
    TSPH_HIP_CHECK(c, hipGetLastError());
    return TSPH_OK;
  }
  GravArgs A;
  A.cap_n = c->cap_n;
  A.groups = c->groups;
  A.ngroups = c->ngroups;
  A.batches = c->batches;
  A.nbatches = c->nbatches;
  A.nngas = c->nngas;
  A.mem = members_of(c, c->n, c->n_gas);
  A.topo = c->topo;
  A.nbox = c->nbox;
  A.nfar = c->nfar;
  A.grec = c->grec;
  A.perm = c->perm;
  A.nnodes = c->lvl + 46;
  A.acc = c->acc;
  A.cnt = c->cnt;
  A.work = c->work;
  A.flags = c->flags;
  A.dbg = c->dbg_nbr;
  A.dbg_max = c->dbg_max;
  A.G = c->p.G;
  A.quadrupole = c->p.quadrupole;
  A.corr = c->p.soft_mode == TSPH_SOFT_ADAPTIVE ? 1 : 0;
  A.lit = c->p.grav_corr_literal;
  A.soften = c->p.soften_cells;
  A.act = c->blk_on ? c->bact_s : nullptr;
  A.nsoft = c->nsoft;
  A.want_pot = want_pot ? 1 : 0;
  // debug lists are written by the batch's own wave
  A.split_particles = c->dbg_nbr ? 0 : c->p.split_leaves * c->p.leaf_size;
  A.split_cap = split_cap_used(c);
  A.split_rng = c->split_rng;
  A.split_item = c->split_item;
  A.split_part = c->split_part;
  A.split_head = c->split_head;
  A.L = c->p.period;
  A.ewt = c->ewt;
  A.ewt32 = c->ewt32;
  if (A.L > 0.0 && c->ew_L != A.L) {
    snprintf(c->err, sizeof(c->err), "the Ewald table of the periodic box was not built");
    return TSPH_EINVAL;
  }
  const int mode =
      (A.quadrupole ? kQuad : 0) | (A.corr ? kCorr : 0) | (A.want_pot ? kPot : 0) | (A.L > 0.0 ? kPer : 0);
#define TSPH_G16(K, F)                                                                                   \
  {K<0, F>, K<1, F>, K<2, F>, K<3, F>, K<4, F>, K<5, F>, K<6, F>, K<7, F>, K<8, F>, K<9, F>, K<10, F>, \
   K<11, F>, K<12, F>, K<13, F>, K<14, F>, K<15, F>}
  void (*const k64[16])(GravArgs) = TSPH_G16(k_gravity, false);
  void (*const k32[16])(GravArgs) = TSPH_G16(k_gravity, true);
  void (*const s64[16])(GravArgs) = TSPH_G16(k_gravity_split, false);
  void (*const s32[16])(GravArgs) = TSPH_G16(k_gravity_split, true);
#undef TSPH_G16
  const bool f32 = c->p.precision == TSPH_FP32_BULK;
  void (*kern)(GravArgs) = f32 ? k32[mode] : k64[mode];
  void (*skern)(GravArgs) = f32 ? s32[mode] : s64[mode];
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(c->cap_nodes, 256, 4096)), dim3(256), 0, st, c->cap_nodes,
                     c->split_head, -1);
  hipLaunchKernelGGL(kern, dim3(persistent_blocks(c, (const void *)kern)), dim3(64), 0, st, A);
  if (A.split_particles > 0) {
    hipLaunchKernelGGL(skern, dim3(persistent_blocks(c, (const void *)skern)), dim3(64), 0, st, A);
    hipLaunchKernelGGL(k_split_reduce, dim3(4096), dim3(64), 0, st, A);
  }
  TSPH_HIP_CHECK(c, hipGetLastError());
  return TSPH_OK;
}

// The Ewald correction table of the context's periodic box (built when the
// box side changes; synchronous).
tsph_status tsph_impl_ewald(Ctx *c) {
  const double L = c->p.period;
  if (!(L > 0.0) || c->ew_L == L) return TSPH_OK;
  constexpr int n1 = kEwaldGrid + 1;
  hipLaunchKernelGGL(k_ewald_table, dim3((n1 * n1 * n1 + 255) / 256), dim3(256), 0, 0, L, c->ewt);
  hipLaunchKernelGGL(k_ewald_pack, dim3((n1 * n1 * n1 + 255) / 256), dim3(256), 0, 0, c->ewt, c->ewt32);
  TSPH_HIP_CHECK(c, hipGetLastError());
  TSPH_HIP_CHECK(c, hipDeviceSynchronize());
  c->ew_L = L;
  return TSPH_OK;
}
