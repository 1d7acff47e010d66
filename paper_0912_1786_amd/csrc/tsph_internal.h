// tsph_internal.h -- context layout, node records, wave primitives and the
// spline kernel functions of the HIP path (gfx950, wave64).
//
// Formulas: Merlin et al., arXiv:0912.1786 -- Sect. 2.1 (Eqs. spline,
// softforce, softphi, dphidh), Sect. 3 (TC92 gradient), App. B.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "tsph.h"

namespace tsph {

constexpr int kMaxLevel = 21;        // 3 x 21 key bits
constexpr int kWave = 64;            // CDNA wavefront
constexpr int kSortBits = 8;         // radix digit
constexpr int kSortBins = 1 << kSortBits;
constexpr int kSortTile = 4096;      // keys per sort block (256 threads x 16)
constexpr int kScanTile = 2048;      // elements per scan block (256 threads x 8)

// Far-field record of a node (96 B): centre of mass, mass, traceless
// quadrupole about the centre of mass (xx, yy, zz, xy, xz, yz), and the
// opening radius l/theta + delta of the Dubinski criterion.
struct NodeFar {
  double cx, cy, cz, m;
  double qxx, qyy, qzz, qxy;
  double qxz, qyz, rmac, pad;
};

// Neighbour-search record of a node (64 B): tight bounding box of its
// particles, the largest eps (all species) and the largest h (gas).
struct NodeBox {
  double lox, loy, loz, epsmax;
  double hix, hiy, hiz, hmax;
};

// Topology of a node in level order; children of a node are contiguous.
struct NodeTopo {
  int32_t first, count, child, nchild;
};

// Source record of a particle for the gravity walk (64 B, one scalar load).
struct GravRec {
  double x, y, z, m;
  double eps, ieps, xiu, s4;  // eps, 1/eps, xi~ / Upsilon, (2 eps)^2
};

// Source record of a gas particle for the SPH pairs (128 B); position and
// h lead, the part the candidate tiles stage.
struct SphRec {
  double x, y, z, h;
  double vx, vy, vz, m;        // predicted velocity, mass
  double im, ih, rho, c;       // 1/m, 1/h, density, sound speed
  double pr2, zo, fa, pad1;    // P / rho^2, zeta / Omega*, grad-h factor f_ij = fa + zo / m_j
};

// The partner fields of an SPH pair in single precision (the FP32-bulk
// form's force pass; positions stay in the double-precision record)
struct alignas(16) SphRec32 {
  float vx, vy, vz, m;   // predicted velocity, mass
  float ih, rho, c, pr2;
  float zo, fa, im, h;
};

// The simulations a context holds (a forest of independent trees).  Member
// m owns particles [off[m], off[m+1]) in caller order and, because the sort
// is segmented by member, the same range in key order; its first ngas[m]
// particles are gas.  Node m of level 0 is its root, and no walk, sum or
// time-step crosses members.  count == 1: a single system of n particles
// whose first n_gas are gas; the tables are then not read.
struct Members {
  const int64_t *off;   // count + 1 entries
  const int64_t *ngas;  // count entries
  int32_t count;
  int64_t n, n_gas;
};

constexpr int kMemberBlocks = 16;  // blocks per member of the per-member reductions

__device__ __forceinline__ int member_of(const Members &M, int64_t i) {
  if (M.count <= 1) return 0;
  int lo = 0, hi = M.count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (M.off[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int64_t member_begin(const Members &M, int m) { return M.count <= 1 ? 0 : M.off[m]; }

__device__ __forceinline__ int64_t member_end(const Members &M, int m) { return M.count <= 1 ? M.n : M.off[m + 1]; }

// is particle i (caller order) of member m gas?
__device__ __forceinline__ bool member_gas(const Members &M, int m, int64_t i) {
  return M.count <= 1 ? i < M.n_gas : i - M.off[m] < M.ngas[m];
}

struct DevRoot {
  double x0, y0, z0, side;  // power-of-two root cube
  double scale;             // 2^(21 - e): key = floor((x - x0) * scale)
  int32_t e, pad;
};

// Per-particle solve outputs kept for export (sorted order).
// A piece of a walk batch's near field evaluated by another wavefront: the
// particle ranges split_rng[start, start + count) = (first, count) acting on
// sink chunk c0 of batch g; next chains the items of one batch in creation
// order.
struct SplitItem {
  int32_t g, c0, start, count, next, pad0, pad1, pad2;
};
constexpr int kSplitItemRanges = 128;      // ranges per item
constexpr int kSplitItemParticles = 2048;  // particles per item; longer ranges are cut
// capacity in split items of a context with cap_nodes nodes.  Past it,
// batches evaluate their whole near field themselves (correct, but the
// summation order then depends on which batches got items first).
inline int64_t split_item_cap(int64_t cap_nodes) {
  const int64_t v = cap_nodes / 4;
  return v < 4096 ? 4096 : (v > 262144 ? 262144 : v);
}

// capacity of the list of density batches solved one sink per wavefront
inline int64_t heavy_batch_cap(int64_t cap_nodes) { return cap_nodes < 4096 ? 4096 : cap_nodes; }

// per-particle outputs of the force pass kept in key order: the solves'
// sums and factors, and the SPH pass's largest |mu|, largest signal
// velocity, viscous heating and X-SPH sum
// rows of the carry from one force pass to the next step (caller order):
// div v (h kernel), div v (eps kernel), X-SPH correction (3), the rates of
// alpha and alpha_u, the largest |mu_ij| (for the Courant criterion)
constexpr int kCarryRows = 8;

// intervals per axis of the Ewald correction table over [0, L/2]
constexpr int kEwaldGrid = 32;
constexpr int64_t kEwaldValues = 3 * (int64_t)(kEwaldGrid + 1) * (kEwaldGrid + 1) * (kEwaldGrid + 1);

enum SolveField { kNh = 0, kOmega, kZeta, kDivv, kNeps, kUps, kXi, kMaxmu, kDivvE, kVsig, kDuv, kXsx, kXsy, kXsz,
                  kCurlx, kCurly, kCurlz, kFbal, kLapu, kNumSolve };

struct Ctx {
  int device;
  tsph_params p;
  int64_t cap_n, cap_nodes;
  int64_t n, n_gas;       // of the last tree build
  void *arena;
  size_t arena_bytes;
  hipStream_t last_stream;
  char err[512];

  // ---- particles, sorted order (capacity cap_n) ----
  uint64_t *key[2];
  int32_t *idx[2];
  int32_t *perm;          // = idx[final]: sorted -> caller
  double4 *pm;            // x, y, z, m
  double4 *vu;            // predicted vx, vy, vz, u
  double *hs, *es;        // h, eps (guess in, solution out)
  uint8_t *gas;
  int32_t *leaf_of;
  double4 *sph;           // h, rho, c, P/rho^2
  double *zo;             // zeta / Omega*
  double2 *soft;          // eps, xi / Upsilon
  GravRec *grec;          // gravity source records
  SphRec *srec;           // SPH source records (gas entries)
  SphRec32 *srec32;       // their single-precision partner fields (FP32-bulk form)
  double4 *srec2;         // dissipation switches: alpha, alpha_u, Balsara factor, u (gas entries)
  double2 *av;            // alpha, alpha_u gathered into key order
  const double *alpha_state, *alpha_u_state;  // the state's arrays of the current force pass (caller order)
  double *solve;          // kNumSolve x cap_n
  double *pdiv;           // kCarryRows x cap_n, caller order: div v with the h kernel (gas) and the eps
                          // kernel, the X-SPH velocity correction (3 rows)
  int64_t pdiv_n;         // particle count the divergences belong to (0: none yet)
  double *acc;            // 6 x cap_n: ax, ay, az, pot, dudt (key order); per-particle time-steps
                          // (caller order)
  int32_t *cnt;           // 3 x cap_n: far nodes, near pairs, SPH pairs

  // ---- nodes, level order (capacity cap_nodes) ----
  NodeTopo *topo;
  int32_t *nlevel, *nparent, *nngas;
  NodeFar *nfar;
  NodeBox *nbox;
  double2 *nsoft;         // softened cells: sum of m eps and of m xi/Upsilon over the node
  int2 *ctmp;             // 8 x cap_nodes child (first, count) scratch
  int32_t *ctmpn;         // cap_nodes child counts of a level
  int32_t *cscan;         // cap_nodes exclusive scan of ctmpn
  int32_t *groups;        // cap_nodes group nodes
  int2 *batches;          // cap_nodes walk batches: group ranges [g0, g1)
  int32_t *nbatches;
  int2 *sbatches;         // cap_nodes SPH walk batches (packed by gas count)
  int32_t *nsbatches;
  int32_t *gflag;         // cap_n group start flags / scan

  // ---- members (tsph_set_members) ----
  int32_t nmem, cap_mem;  // members held (1: a single system), capacity
  int64_t *moff, *mgas;   // device tables: cap_mem + 1 offsets, cap_mem gas counts
  int32_t *mtile;         // device: cap_mem + 1 prefix of the members' sort tiles
  int64_t *h_moff, *h_mgas;  // host copies
  int32_t sort_tiles;     // sum of the members' sort tiles

  // ---- small device state ----
  DevRoot *root;          // cap_mem root cubes
  double *bbox_part;      // partial bbox (6 x max blocks)
  int32_t *lvl;           // [0..23): level begin, [23..46): level count, [46]: total nodes
  int32_t *ngroups;
  uint32_t *hist;         // radix histograms kSortBins x sort blocks
  int32_t *scan_part;     // scan block sums
  int32_t *work;          // kWorkCounters work-queue counters: 3 split leaves, 4 split items, 5 split walk,
                          // 6 handed-off density batches, 7 their sinks, 8/16/24 the XCD queues of the
                          // density, gravity and SPH walks (8 each), 34/35/36 SPH hand-off ranges, items, split walk
  int2 *split_rng;        // split_cap x kSplitItemRanges particle ranges handed from batches' near fields
  SplitItem *split_item;  // split_cap work items over split_rng
  double4 *split_part;    // split_cap x 64 partial (ax, ay, az, pot) of the items
  int64_t split_cap;
  int64_t split_cap_limit; // > 0: hand-off items used at most (tsph_debug_handoff_cap)
  int32_t *split_head;    // cap_nodes: first item of each batch (-1: none), items chained in order
  int32_t *heavy;         // heavy_cap batches whose length solves run one sink per wavefront,
                          // then heavy_cap sort keys, then heavy_cap batches in processing order
  int64_t heavy_cap;
  uint32_t *flags;        // device flag word
  int32_t *noconv;        // unconverged solves
  double *red;            // reduction scratch
  double *dt;             // cap_mem time-steps of the last tsph_timestep (one per member)

  // ---- individual time-steps (tsph_block_*) ----
  uint8_t *bact;          // cap_n active flags, caller order
  uint8_t *bact_s;        // cap_n active flags, key order (force passes with blk_on)
  int32_t *bcur;          // cap_n current step lengths in ticks (criterion step of the active), caller order
  int32_t *bcur_s;        // cap_n the same in key order
  int32_t *bm, *bw;       // cap_n: shortest current step around each gas particle, shortest criterion
                          // step of its active neighbours (caller order; INT32_MAX: none)
  int32_t *bnext;         // [0] next system time, [1] active count, [2] woken count
  int32_t blk_on;         // the force pass evaluates the active sinks only

  // ---- periodic box ----
  double *ewt;            // Ewald correction table, 3 x (kEwaldGrid + 1)^3
  float4 *ewt32;          // the same table in single precision, (x, y, z, 0) per grid point
  double ew_L;            // box side the table was built for (0: none)

  // ---- phase timing (ring of event sets) ----
  int32_t timing;
  int64_t t_calls, t_done;
  hipEvent_t (*tev)[6];
  double t_ms[5];

  // ---- launch shapes ----
  int32_t n_cu;
  const void *occ_kernel[16];
  int32_t occ_blocks[16];

  // ---- debug ----
  int32_t dbg_max;
  int32_t *dbg_nbr;       // 3 x cap_n x dbg_max (caller index), or null
  uint32_t *h_flags;      // pinned host copy
  int32_t *h_noconv;
};

// hand-off items a force pass may use
inline int64_t split_cap_used(const Ctx *c) {
  return c->split_cap_limit > 0 && c->split_cap_limit < c->split_cap ? c->split_cap_limit : c->split_cap;
}

inline Members members_of(const Ctx *c, int64_t n, int64_t n_gas) {
  return Members{c->moff, c->mgas, c->nmem, n, n_gas};
}

// ---------------------------------------------------------------------------
// wave primitives (wave64)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// 1/sqrt(x) in FP64 for positive, finite, normal x: the hardware estimate y
// refined by one second-order step, y (1 + e/2 + 3 e^2/8) with
// e = 1 - x y^2 (the Taylor series of (1 - e)^(-1/2)), written as
// y + (y e)(1/2 + 3e/8).  Zero, infinity and NaN are not special-cased: the
// callers pass positive squared distances, or discard the result.
__device__ __forceinline__ double rsq64(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(y * -x, y, 1.0);
  const double u = y * e;
  return fma(u, fma(e, 0.375, 0.5), y);
}

// Single-precision hardware 1/sqrt(x) and 1/x (about one ulp).  For normal x
// rsq32 is what rsqrtf returns; rsqrtf's extra scaling of denormal arguments
// is left out (the callers' squared distances never lie in that range, and
// zero gives +inf either way).
__device__ __forceinline__ float rsq32(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float rcp32(float x) { return __builtin_amdgcn_rcpf(x); }

// Per-lane mask of the tile entries j < nt (nt <= 64) for which f(j) holds,
// f called for j = 0, 1, ... in order.  Built as two 32-bit halves, so that
// the bit of entry j is a wave-uniform constant.
template <class F>
__device__ __forceinline__ uint64_t tile_mask(int nt, F &&f) {
  uint32_t lo = 0, hi = 0;
  const int n0 = nt < 32 ? nt : 32;
  for (int j = 0; j < n0; j++) lo |= f(j) ? 1u << j : 0u;
  for (int j = 32; j < nt; j++) hi |= f(j) ? 1u << (j - 32) : 0u;
  return (uint64_t)hi << 32 | lo;
}

// number of set bits of m below this lane
__device__ __forceinline__ int mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Load through the constant address space: with a wave-uniform address the
// backend emits scalar (SMEM) loads into SGPRs, one per wave instead of one
// per lane.  Only for data no kernel of the same launch writes.
typedef const __attribute__((address_space(4))) uint32_t *cdword_ptr;

template <class T>
__device__ __forceinline__ T sload(const T *p) {
  static_assert(sizeof(T) % 4 == 0, "records are whole dwords");
  T v;
  cdword_ptr src = (cdword_ptr)(p);
  uint32_t *dst = reinterpret_cast<uint32_t *>(&v);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); i++) dst[i] = src[i];
  return v;
}

// byte variant: reads the aligned dword holding the byte (arena buffers are
// padded to 256 bytes, so the dword never leaves the allocation)
__device__ __forceinline__ uint32_t sload_u8(const uint8_t *p) {
  const uintptr_t a = (uintptr_t)p;
  cdword_ptr w = (cdword_ptr)(a & ~(uintptr_t)3);
  return (*w >> (8 * (a & 3))) & 0xffu;
}

__device__ __forceinline__ int wave_incl_scan(int v) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int t = __shfl_up(v, o, kWave);
    if (lane() >= o) v += t;
  }
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}

__device__ __forceinline__ int wave_or(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, kWave);
  return v;
}

// ---------------------------------------------------------------------------
// spline kernel family (M4 cubic spline, support 2h)
// q = r / h.  w(q) = 1 - 3/2 q^2 + 3/4 q^3 (q < 1), 1/4 (2 - q)^3 (q < 2).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void m4(double q, double &w, double &dw) {
  if (q < 1.0) {
    w = 1.0 + q * q * (-1.5 + 0.75 * q);
    dw = q * (-3.0 + 2.25 * q);
  } else if (q < 2.0) {
    double t = 2.0 - q;
    w = 0.25 * t * t * t;
    dw = -0.75 * t * t;
  } else {
    w = 0.0;
    dw = 0.0;
  }
}

// derivative of the M4 kernel used in the SPH pairs: the plain dw/dq or the
// Thomas & Couchman (1992) form, constant inside q < 2/3 (Sect. 3).
template <class T>
__device__ __forceinline__ T m4_grad(T q, bool tc92) {
  if (q < T(1)) {
    if (tc92 && q < T(2.0 / 3.0)) return T(-1);
    return q * (T(-3) + T(2.25) * q);
  }
  if (q < T(2)) {
    const T t = T(2) - q;
    return T(-0.75) * t * t;
  }
  return T(0);
}

// m4 in either precision
template <class T>
__device__ __forceinline__ void m4_t(T q, T &w, T &dw) {
  if (q < T(1)) {
    w = T(1) + q * q * (T(-1.5) + T(0.75) * q);
    dw = q * (T(-3) + T(2.25) * q);
  } else if (q < T(2)) {
    const T t = T(2) - q;
    w = T(0.25) * t * t * t;
    dw = T(-0.75) * t * t;
  } else {
    w = T(0);
    dw = T(0);
  }
}

// Softened gravity of a unit mass smoothed by the spline (Sect. 2.1):
//   fr(r, e) = d phi / d r  (1/r^2 outside 2e)
//   ph(r, e) = phi          (-1/r outside 2e)
//   pe(r, e) = d phi / d e  (0 outside 2e)
// Polynomials in q = r/e; for the outer branch the e-derivative is
// -(f + q f')/e^2 with phi = f(q)/e.
__device__ __forceinline__ double soft_fr(double r, double e) {
  double q = r / e;
  if (q >= 2.0) return 1.0 / (r * r);
  double q2 = q * q, ie2 = 1.0 / (e * e);
  if (q < 1.0) return ie2 * q * ((4.0 / 3.0) + q2 * (-1.2 + 0.5 * q));
  return ie2 * (q * ((8.0 / 3.0) + q * (-3.0 + q * (1.2 - q / 6.0))) - 1.0 / (15.0 * q2));
}

__device__ __forceinline__ double soft_ph(double r, double e) {
  double q = r / e;
  if (q >= 2.0) return -1.0 / r;
  double q2 = q * q;
  if (q < 1.0) return (q2 * ((2.0 / 3.0) + q2 * (-0.3 + 0.1 * q)) - 1.4) / e;
  return (q2 * ((4.0 / 3.0) + q * (-1.0 + q * (0.3 - q / 30.0))) - 1.6 + 1.0 / (15.0 * q)) / e;
}

__device__ __forceinline__ double soft_pe(double r, double e) {
  double q = r / e;
  if (q >= 2.0) return 0.0;
  double q2 = q * q;
  if (q < 1.0) return (1.4 + q2 * (-2.0 + q2 * (1.5 - 0.6 * q))) / (e * e);
  return (1.6 + q2 * (-4.0 + q * (4.0 + q * (-1.5 + 0.2 * q)))) / (e * e);
}

// The same softened kernels in division-free form for the inner loops, in
// either precision: q = r / e with ie = 1/e and ir = 1/r given
// (1/(15 q^2 e^2) = ir^2 / 15).
template <class T>
__device__ __forceinline__ T soft_fr_q(T q, T ie, T ir) {
  if (q >= T(2)) return ir * ir;
  const T q2 = q * q, ie2 = ie * ie;
  if (q < T(1)) return ie2 * q * (T(4.0 / 3.0) + q2 * (T(-1.2) + T(0.5) * q));
  return ie2 * (q * (T(8.0 / 3.0) + q * (T(-3) + q * (T(1.2) - q * T(1.0 / 6.0))))) - ir * ir * T(1.0 / 15.0);
}

template <class T>
__device__ __forceinline__ T soft_ph_q(T q, T ie, T ir) {
  if (q >= T(2)) return -ir;
  const T q2 = q * q;
  if (q < T(1)) return ie * (q2 * (T(2.0 / 3.0) + q2 * (T(-0.3) + T(0.1) * q)) - T(1.4));
  return ie * (q2 * (T(4.0 / 3.0) + q * (T(-1) + q * (T(0.3) - q * T(1.0 / 30.0)))) - T(1.6)) + ir * T(1.0 / 15.0);
}

template <class T>
__device__ __forceinline__ T soft_pe_q(T q, T ie) {
  if (q >= T(2)) return T(0);
  const T q2 = q * q;
  if (q < T(1)) return (T(1.4) + q2 * (T(-2) + q2 * (T(1.5) - T(0.6) * q))) * (ie * ie);
  return (T(1.6) + q2 * (T(-4) + q * (T(4) + q * (T(-1.5) + T(0.2) * q)))) * (ie * ie);
}

template <class T>
__device__ __forceinline__ T m4_dw(T q) {
  if (q < T(1)) return q * (T(-3) + T(2.25) * q);
  if (q < T(2)) {
    const T t = T(2) - q;
    return T(-0.75) * t * t;
  }
  return T(0);
}

// ---------------------------------------------------------------------------
// exact geometric predicates (one rounding per operation, fixed order)
// ---------------------------------------------------------------------------
// For boxes with lo <= hi the gap is the larger of the two differences and
// zero: lo - p when p < lo, p - hi when p > hi, else both are <= 0 -- the
// same rounded values as the case-by-case form, in fewer instructions.
__device__ __forceinline__ double axis_gap_point(double lo, double hi, double p) {
#pragma clang fp contract(off)
  const double d = fmax(fmax(lo - p, p - hi), 0.0);
  return d * d;
}

__device__ __forceinline__ double axis_gap_box(double lo1, double hi1, double lo2, double hi2) {
#pragma clang fp contract(off)
  const double d = fmax(fmax(lo2 - hi1, lo1 - hi2), 0.0);
  return d * d;
}

// squared length of a displacement, in the order of dist2_pair
__device__ __forceinline__ double dist2_disp(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  double s = dx * dx;
  s = s + dy * dy;
  s = s + dz * dz;
  return s;
}

// ---- periodic box (Sect. 4.3): nearest images, side L (0: open) ----
// nearest-image component of a displacement
__device__ __forceinline__ double wrap_d(double d, double L) {
#pragma clang fp contract(off)
  return L > 0.0 ? d - L * rint(d / L) : d;
}
// squared gaps on a circle of circumference L: the nearest-image distance of
// the centres less the half-widths (the open forms when L = 0)
__device__ __forceinline__ double axis_gap_point_p(double lo, double hi, double p, double L) {
#pragma clang fp contract(off)
  if (!(L > 0.0)) return axis_gap_point(lo, hi, p);
  const double c = 0.5 * (lo + hi), w = 0.5 * (hi - lo);
  const double t = fabs(wrap_d(p - c, L));
  const double d = t > w ? t - w : 0.0;
  return d * d;
}
__device__ __forceinline__ double axis_gap_box_p(double lo1, double hi1, double lo2, double hi2, double L) {
#pragma clang fp contract(off)
  if (!(L > 0.0)) return axis_gap_box(lo1, hi1, lo2, hi2);
  const double c1 = 0.5 * (lo1 + hi1), w1 = 0.5 * (hi1 - lo1);
  const double c2 = 0.5 * (lo2 + hi2), w2 = 0.5 * (hi2 - lo2);
  double d = fabs(wrap_d(c2 - c1, L)) - w1 - w2;
  if (!(d > 0.0)) d = 0.0;
  return d * d;
}
// a coordinate taken into the periodic box [0, L)
__device__ __forceinline__ double in_box(double x, double L) {
#pragma clang fp contract(off)
  return L > 0.0 ? x - L * floor(x / L) : x;
}

__device__ __forceinline__ double dist2_pair(double xi, double yi, double zi, double xj, double yj,
                                             double zj) {
#pragma clang fp contract(off)
  double dx = xj - xi, dy = yj - yi, dz = zj - zi;
  double s = dx * dx;
  s = s + dy * dy;
  s = s + dz * dz;
  return s;
}

// Sink balls staged in LDS for the walk pruning: snk[s] = (x, y, z, R_s) for
// lane s (R_s <= 0: no ball), then one pair of records per group of
// kBallGroupSize consecutive lanes, snk[kWave + 2g] = (lowest x, y, z, largest R_s) and
// snk[kWave + 2g + 1] = (highest x, y, z, 0) over the group's balls (a group
// without a ball has largest radius -1).
constexpr int kBallGroupSize = 8;
constexpr int kBallGroups = kWave / kBallGroupSize;
constexpr int kSnkRecs = kWave + 2 * kBallGroups;

// Writes the group records from each lane's own ball b.  The whole wave
// calls it; the records are read after the caller's next barrier.
__device__ __forceinline__ void stage_ball_groups(double4 *snk, const double4 &b) {
  const bool on = b.w > 0.0;
  double lx = on ? b.x : INFINITY, ly = on ? b.y : INFINITY, lz = on ? b.z : INFINITY;
  double hx = on ? b.x : -INFINITY, hy = on ? b.y : -INFINITY, hz = on ? b.z : -INFINITY;
  double w = on ? b.w : -1.0;
  for (int o = 1; o < kBallGroupSize; o <<= 1) {
    lx = fmin(lx, __shfl_xor(lx, o, kWave));
    ly = fmin(ly, __shfl_xor(ly, o, kWave));
    lz = fmin(lz, __shfl_xor(lz, o, kWave));
    hx = fmax(hx, __shfl_xor(hx, o, kWave));
    hy = fmax(hy, __shfl_xor(hy, o, kWave));
    hz = fmax(hz, __shfl_xor(hz, o, kWave));
    w = fmax(w, __shfl_xor(w, o, kWave));
  }
  const int ln = __lane_id();
  if (ln % kBallGroupSize == 0) {
    snk[kWave + 2 * (ln / kBallGroupSize)] = make_double4(lx, ly, lz, w);
    snk[kWave + 2 * (ln / kBallGroupSize) + 1] = make_double4(hx, hy, hz, 0.0);
  }
}

// The periodic form: each group's centres are unwrapped around its first
// lane's position (nearest images), so its box may reach past the cell; a
// group spread over a quarter of the box or more keeps an infinite radius
// (its members are always tested).
__device__ __forceinline__ void stage_ball_groups_p(double4 *snk, const double4 &b, double L) {
  const int ln = __lane_id();
  const int first = ln & ~(kBallGroupSize - 1);
  const double rx = __shfl(b.x, first, kWave), ry = __shfl(b.y, first, kWave), rz = __shfl(b.z, first, kWave);
  const bool on = b.w > 0.0;
  const double ux = rx + wrap_d(b.x - rx, L), uy = ry + wrap_d(b.y - ry, L), uz = rz + wrap_d(b.z - rz, L);
  double lx = on ? ux : INFINITY, ly = on ? uy : INFINITY, lz = on ? uz : INFINITY;
  double hx = on ? ux : -INFINITY, hy = on ? uy : -INFINITY, hz = on ? uz : -INFINITY;
  double w = on ? b.w : -1.0;
  for (int o = 1; o < kBallGroupSize; o <<= 1) {
    lx = fmin(lx, __shfl_xor(lx, o, kWave));
    ly = fmin(ly, __shfl_xor(ly, o, kWave));
    lz = fmin(lz, __shfl_xor(lz, o, kWave));
    hx = fmax(hx, __shfl_xor(hx, o, kWave));
    hy = fmax(hy, __shfl_xor(hy, o, kWave));
    hz = fmax(hz, __shfl_xor(hz, o, kWave));
    w = fmax(w, __shfl_xor(w, o, kWave));
  }
  if (w > 0.0 && (hx - lx >= 0.25 * L || hy - ly >= 0.25 * L || hz - lz >= 0.25 * L)) w = INFINITY;
  if (ln % kBallGroupSize == 0) {
    snk[kWave + 2 * (ln / kBallGroupSize)] = make_double4(lx, ly, lz, w);
    snk[kWave + 2 * (ln / kBallGroupSize) + 1] = make_double4(hx, hy, hz, 0.0);
  }
}

// Periodic gap along one axis between a box and a group's box, lowered by
// 1e-12 L, far more than the rounding of either gap: never more than the
// nearest-image gap of any member inside the group's box.
__device__ __forceinline__ double group_gap_p(double lo, double hi, double glo, double ghi, double L) {
  const double c1 = 0.5 * (lo + hi), w1 = 0.5 * (hi - lo);
  const double c2 = 0.5 * (glo + ghi), w2 = 0.5 * (ghi - glo);
  const double d = fabs(wrap_d(c2 - c1, L)) - w1 - w2 - 1e-12 * L;
  return d > 0.0 ? d : 0.0;
}

// Does some sink ball of the wave reach the box?  The ball radius used for
// sink s is max(R_s, r_node).  Every lane tests its own box against the
// staged sinks (broadcast reads); the loop stops once every lane that still
// needs an answer has one.  The test only prunes candidates (the pair tests
// decide), so it may keep more than the exact one and never less: in the
// open box the gaps are max(lo - p, p - hi, 0) with fused squares, against
// a radius widened by 1e-14 relative, which covers their rounding.  A group
// of balls is tested first, as the gap from the box to the box of the
// group's centres against the group's largest radius: that gap is at most
// each member's (in the open box because rounding is monotone, in the
// periodic box because the periodic distance is a metric and group_gap_p
// keeps a margin), the radius at least each member's, so a group that fails
// holds no ball that reaches, and the result equals the test of every ball.
__device__ __forceinline__ bool balls_reach_box(const double4 *snk, double lox, double loy, double loz,
                                                double hix, double hiy, double hiz, double r_node, bool want,
                                                double L = 0.0) {
  bool hit = false;
  if (L > 0.0) {
    for (int g = 0; g < kBallGroups; g++) {
      if (!__any(want && !hit)) break;
      const double4 glo = snk[kWave + 2 * g], ghi = snk[kWave + 2 * g + 1];
      bool need = false;
      if (want && !hit && glo.w > 0.0) {
        const double Rg = fmax(glo.w, r_node);
        const double gx = group_gap_p(lox, hix, glo.x, ghi.x, L);
        const double gy = group_gap_p(loy, hiy, glo.y, ghi.y, L);
        const double gz = group_gap_p(loz, hiz, glo.z, ghi.z, L);
        need = gx * gx + gy * gy + gz * gz < (Rg * Rg) * (1.0 + 1e-12);
      }
      if (!__any(need)) continue;
      for (int s = kBallGroupSize * g; s < kBallGroupSize * (g + 1); s++) {
        const double4 q = snk[s];
        if (need && q.w > 0.0) {
          const double R = fmax(q.w, r_node);
          double d2 = axis_gap_point_p(lox, hix, q.x, L);
          d2 = d2 + axis_gap_point_p(loy, hiy, q.y, L);
          d2 = d2 + axis_gap_point_p(loz, hiz, q.z, L);
          hit = hit || (d2 < R * R);
        }
      }
    }
    return hit;
  }
  for (int g = 0; g < kBallGroups; g++) {
    if (!__any(want && !hit)) break;
    const double4 glo = snk[kWave + 2 * g], ghi = snk[kWave + 2 * g + 1];
    const double Rg = fmax(glo.w, r_node);
    const double R2g = glo.w > 0.0 ? (Rg * Rg) * (1.0 + 1e-14) : -1.0;
    const double gx = fmax(fmax(lox - ghi.x, glo.x - hix), 0.0);
    const double gy = fmax(fmax(loy - ghi.y, glo.y - hiy), 0.0);
    const double gz = fmax(fmax(loz - ghi.z, glo.z - hiz), 0.0);
    const bool need = want && !hit && fma(gz, gz, fma(gy, gy, gx * gx)) < R2g;
    if (!__any(need)) continue;
    for (int s = kBallGroupSize * g; s < kBallGroupSize * (g + 1); s++) {
      const double4 q = snk[s];
      const double R = fmax(q.w, r_node);
      const double R2 = q.w > 0.0 ? (R * R) * (1.0 + 1e-14) : -1.0;
      const double dx = fmax(fmax(lox - q.x, q.x - hix), 0.0);
      const double dy = fmax(fmax(loy - q.y, q.y - hiy), 0.0);
      const double dz = fmax(fmax(loz - q.z, q.z - hiz), 0.0);
      hit = hit || (need && fma(dz, dz, fma(dy, dy, dx * dx)) < R2);
    }
  }
  return hit;
}

// Nodes popped per walk round (at most `most`) from an LDS stack of capacity
// cap holding sp entries.  Each popped node pushes at most 8 children, so
// popping t nodes grows the stack by at most 7 t.  Full rounds run while that fits
// above a reserve of 160 entries; inside the reserve a single node is popped,
// i.e. the walk continues depth first from the top, which needs at most
// 7 x 21 more entries.  The stack therefore never exceeds cap.
__device__ __forceinline__ int walk_take(int sp, int cap, int most = kWave) {
  const int room = cap - sp - 160;
  int t = room >= 7 * most ? most : room / 7;
  t = t < 1 ? 1 : t;
  return t < sp ? t : sp;
}

// Work queues of the persistent walk kernels.  The batch list (Morton order)
// is cut into one contiguous segment per XCD; a workgroup takes batches from
// the segment of its XCD (workgroups are dispatched to the 8 XCDs round
// robin), so that batches in flight on one XCD share nodes and particles in
// that XCD's L2, and steals from the other segments once its own is empty.
// ctr points at 8 counters; returns -1 when every segment is exhausted.
constexpr int kWorkCounters = 64;
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_next(int32_t *ctr, int n) {
  const int x = (int)(blockIdx.x % kXcds);
  for (int k = 0; k < kXcds; k++) {
    const int seg = (x + k) % kXcds;
    const int lo = (int)((int64_t)n * seg / kXcds), hi = (int)((int64_t)n * (seg + 1) / kXcds);
    if (lo >= hi) continue;
    const int i = atomicAdd(&ctr[seg], 1);
    if (lo + i < hi) return lo + i;
  }
  return -1;
}

// A walk batch: a run of sibling groups [g0, g1) of the group list; its
// particles are one contiguous key-order range and its box the union of the
// members' boxes (max eps and h over the members, summed gas counts).
struct Batch {
  int first, count, ngas;
  int root;  // root node of the batch's member: where its walks start
  NodeBox box;
};

__device__ __forceinline__ Batch load_batch(const int2 *batches, const int32_t *groups, const NodeTopo *topo,
                                            const NodeBox *nbox, const int32_t *nngas, const Members &M, int b) {
  const int2 r = sload(batches + b);
  Batch B;
  const int k0 = uniform(sload(groups + r.x));
  const NodeTopo t0 = sload(topo + k0);
  B.first = t0.first;
  B.root = uniform(member_of(M, t0.first));
  B.count = 0;
  B.ngas = 0;
  B.box = sload(nbox + k0);
  for (int g = r.x; g < r.y; g++) {
    const int k = uniform(sload(groups + g));
    const NodeTopo t = sload(topo + k);
    const NodeBox x = sload(nbox + k);
    B.count += t.count;
    B.ngas += sload(nngas + k);
    B.box.lox = fmin(B.box.lox, x.lox);
    B.box.loy = fmin(B.box.loy, x.loy);
    B.box.loz = fmin(B.box.loz, x.loz);
    B.box.hix = fmax(B.box.hix, x.hix);
    B.box.hiy = fmax(B.box.hiy, x.hiy);
    B.box.hiz = fmax(B.box.hiz, x.hiz);
    B.box.epsmax = fmax(B.box.epsmax, x.epsmax);
    B.box.hmax = fmax(B.box.hmax, x.hmax);
  }
  return B;
}

// host-side launch helpers (defined in the translation units)
int blocks_for(int64_t n, int threads, int max_blocks);
// a[0, n) = v (tree.hip)
__global__ __launch_bounds__(256) void k_fill_i32(int64_t n, int32_t *__restrict__ a, int32_t v);
// grid of a persistent one-wave-per-workgroup kernel: resident workgroups per
// CU (from its register and LDS use) times the CU count
int persistent_blocks(Ctx *c, const void *kernel);

}  // namespace tsph

// implemented per translation unit, called by the ABI layer
tsph_status tsph_impl_build_tree(tsph::Ctx *c, const tsph_state *s, hipStream_t st);
tsph_status tsph_impl_density(tsph::Ctx *c, hipStream_t st);
tsph_status tsph_impl_gravity(tsph::Ctx *c, bool want_pot, hipStream_t st);
tsph_status tsph_impl_sph(tsph::Ctx *c, hipStream_t st);
tsph_status tsph_impl_finish(tsph::Ctx *c, tsph_state *s, hipStream_t st);
tsph_status tsph_impl_kick_drift(tsph::Ctx *c, tsph_state *s, double dt, const double *dt_dev, int phase,
                                 hipStream_t st);
tsph_status tsph_impl_timestep(tsph::Ctx *c, const tsph_state *s, double *dt_device, hipStream_t st);
// per-particle time-step criteria of the state into c->acc + 5 cap_n (caller order)
tsph_status tsph_impl_criteria(tsph::Ctx *c, const tsph_state *s, hipStream_t st);
// neighbour minima of the step lengths for the wake-up (sph.hip)
tsph_status tsph_impl_wake(tsph::Ctx *c, hipStream_t st);
// the Ewald table of the context's periodic box (gravity.hip)
tsph_status tsph_impl_ewald(tsph::Ctx *c);
// active flags into key order for a force pass over the active sinks (blocks.hip)
tsph_status tsph_impl_gather_active(tsph::Ctx *c, hipStream_t st);
tsph_status tsph_impl_diagnostics(tsph::Ctx *c, const tsph_state *s, double *out, hipStream_t st);
tsph_status tsph_impl_reset_work(tsph::Ctx *c, hipStream_t st);

#define TSPH_HIP_CHECK(c, call)                                                               \
  do {                                                                                        \
    hipError_t _e = (call);                                                                   \
    if (_e != hipSuccess) {                                                                   \
      snprintf((c)->err, sizeof((c)->err), "%s:%d %s: %s", __FILE__, __LINE__, #call,          \
               hipGetErrorString(_e));                                                        \
      return TSPH_EHIP;                                                                       \
    }                                                                                         \
  } while (0)
