// sph.hip -- SPH acceleration and heating over the symmetric neighbour set
// r_ij < 2 max(h_i, h_j).
//
// Merlin et al., arXiv:0912.1786: Sect. 3 (Eqs. dvdt, drhodr, dudrho,
// motionvarmass, thermalvarmass, Thomas & Couchman gradient), Sect. 3.1
// (symmetric neighbour definition), Sect. 3.3 (Eq. mu_visc and the averaged
// gradient), App. B.  With grad_i W_ij(h) = W'(r, h) (x_i - x_j)/r:
//   a_i  = -sum_j m_j [A_ij gW(h_i) + A_ji gW(h_j) + Pi_ij Gbar_ij]
//   du_i =  sum_j m_j [A_ij v_ij . gW(h_i) + 1/2 Pi_ij v_ij . Gbar_ij]
//   A_ij = (P_i / rho_i^2) f_ij,  f_ij = fa_i + zeta_i / (m_j Omega*_i)
//   (fa = 1 with the number-density relation, 1/Omega with the mass-density
//   one, and f = 1 in the standard scheme),
//   Gbar_ij = 1/2 [f_ij gW(h_i) + f_ji gW(h_j)],
//   Pi_ij = (-alpha cbar mu + beta mu^2) / rhobar  when v_ij . x_ij < 0,
//   mu = hbar v_ij . x_ij / (r^2 + av_eps2 hbar^2), bars = pair means,
// evaluated with the predicted velocities and energies.  Variants: the
// signal-velocity viscosity Pi_ij = -alpha (2 cbar - w) w / rhobar,
// w = v_ij . x_ij / r (Sect. 3.3.1, Eqs. pvsig, vsig); the entropic function
// as energy variable, whose rate is the viscous heating times
// (gamma - 1) rho^(1 - gamma) (Sect. 3.4, Eq. SPHentr); the X-SPH velocity
// correction eta sum_j m_j (v_j - v_i) Wbar_ij / rhobar (Sect. 3.5, Eq.
// xsph).  Every pair also gives the signal velocity 2 cbar - min(w, 0),
// whose largest value per particle is kept.  Dissipation switches (Sect.
// 3.3.1, 3.3.2): a first pass over the same pairs (mode 1) forms the
// velocity curl, the Balsara factor f = |div v| / (|div v| + |curl v| +
// 1e-4 c/h) and the record (alpha, alpha_u, f, u) of every gas particle;
// the force pass then takes the pair mean of alpha, multiplies Pi_ij by the
// pair mean of f, and adds the conductivity term m_j Pi^u_ij |Gbar_ij| to
// du/dt and the Laplacian of u to its own sum.
//
// The FP32-bulk form (mode 3) runs the force pass's pair arithmetic in
// single precision: the pair set is still decided by the double-precision
// distance tests, each pair takes its double-precision displacement rounded
// once and its partner's fields from a single-precision record, and each
// lane's sums over one tile are carried into double-precision totals after
// the tile.
//
// One wavefront per walk group that holds gas; the wave walks the tree once
// (opening nodes with gas within 2 max(h_group, h_node) of the group box),
// lists the candidate leaves in LDS and flushes them in batches.  A flush
// stages the candidates 64 at a time in LDS (position and h), every lane
// tests the whole tile and keeps a mask of its own pairs, and then each lane
// evaluates only its own pairs, in candidate order, reading the partner's
// record itself; lanes do not step through pairs that only other lanes have.
// Once a batch has evaluated split_leaves x leaf_size / 4 candidates itself,
// its further flushes go as work items (the flush's leaf ranges) to
// k_sph_split, and k_sph_reduce adds the items' partial sums to the batch's
// sinks along each batch's item chain, in creation order.
#include <stdio.h>

#include "tsph_internal.h"

namespace tsph {

constexpr int kSStackCap = 1024;
constexpr int kSListCap = 128;
constexpr int kSLeafFlush = 32;
constexpr double kInvPiS = 0.31830988618379067154;
constexpr int kSphPart = 3;  // partial-sum records per lane of a handed-off item

// candidates of a flush staged for the pair tests
struct SphTile {
  double4 pos[kWave];  // x, y, z, (2h)^2
  int q[kWave];
};

// the force passes: double precision (0) and single-precision pairs (3)
constexpr bool force_mode(int m) { return m == 0 || m == 3; }

struct SphArgs {
  int64_t cap_n;
  const int32_t *groups;
  const int32_t *ngroups;
  const int2 *batches;
  const int32_t *nbatches;
  const NodeTopo *topo;
  const NodeBox *nbox;
  const int32_t *nngas;
  Members mem;
  const double4 *pm;
  const double4 *vu;
  const double4 *sph;   // h, rho, c, P/rho^2
  const double *zo;     // zeta / Omega*
  const SphRec *srec;
  const SphRec32 *srec32;  // single-precision partner fields (mode 3)
  const uint8_t *gas;
  const int32_t *perm;
  const int32_t *nnodes;
  double *acc;
  double *solve;
  int32_t *cnt;
  int32_t *work;
  uint32_t *flags;
  int32_t *dbg;
  int32_t dbg_max;
  double alpha, beta, av_eps2, gamma, xsph_eta;
  int32_t tc92, visc_signal, entropy;
  // dissipation switches
  int32_t f2, balsara, alpha_switch, conduction;
  double4 *srec2;      // alpha, alpha_u, Balsara factor, u (gas, key order)
  const double2 *av;   // alpha, alpha_u (key order)
  // hand-off of flushes (0 split_particles: none); the buffers are those of
  // the gravity walk's near-field hand-off, free again by now
  int32_t split_particles;
  int64_t split_cap;  // items; each keeps two partial records per lane
  int2 *split_rng;
  SplitItem *split_item;
  double4 *split_part;
  int32_t *split_head;
  // individual time-steps: force pass over the active sinks (act, key
  // order; NULL: all), and the wake-up pass (mode 2) over the step lengths
  const uint8_t *act;
  const int32_t *bcur_s;
  int32_t *bm, *bw;
  double L;  // periodic box side (0: open)
};

// The sink side of the pairs of one lane: particle p (a gas sink when
// `sink`), its accumulated sums and its debug list.
struct SphLane {
  double4 a;   // x, y, z, m
  double4 v;   // predicted velocity, u
  double4 hd;  // h, rho, c, P/rho^2
  double zi;   // zeta / Omega*
  double fa;   // f_ij = fa + zi / m_j
  double ax, ay, az, du, mumax;
  double duv, vsig;     // viscous heating, largest pair signal velocity
  double xsx, xsy, xsz; // X-SPH sum (without eta); the curl sum in mode 1
  double lapu;          // Laplacian of u (conduction)
  double4 e2;           // alpha, alpha_u, Balsara factor, u
  int bm, bw;           // mode 2: shortest step around; the sink's own step
  int p, npair, ndbg;
  bool sink;
  int32_t *dbg;
};

// kFull: the kernel form with the dissipation switches, the conductivity and
// X-SPH (the plain form keeps none of their state in registers)
template <bool kFull>
__device__ __forceinline__ void sph_lane(const SphArgs &A, SphLane &L, int p, bool sink) {
  L.p = p;
  L.sink = sink;
  L.a = A.pm[p];
  L.v = A.vu[p];
  L.hd = A.sph[p];
  L.zi = A.zo[p];
  L.fa = A.srec[p].fa;
  L.ax = L.ay = L.az = L.du = L.mumax = 0.0;
  L.duv = L.vsig = L.xsx = L.xsy = L.xsz = L.lapu = 0.0;
  L.e2 = (kFull && A.f2) ? A.srec2[p] : make_double4(A.alpha, 0.0, 1.0, 0.0);
  L.npair = 0;
  L.ndbg = 0;
  L.bm = L.bw = INT32_MAX;
  L.dbg = (A.dbg && sink) ? A.dbg + ((int64_t)1 * A.cap_n + A.perm[p]) * A.dbg_max : nullptr;
}

// Pairs of the lane's sink among the nt staged candidates: the distance
// tests of the whole tile first, then the lane's own pairs in tile order.
// kMode 0: forces and heating; kMode 1: the velocity curl sum
// sum_j v_ij x grad_i W_ij(h_i) (plain kernel gradient) in xsx, xsy, xsz;
// kMode 2 (active sinks only): the least step length among the sink's
// neighbours, and the sink's own step scattered as a minimum to each of
// them (coincident ones included).  The pair test is symmetric in i and j,
// so a particle's minimum over its active neighbours is complete once every
// active sink has been walked; integer minima make it independent of order.
template <int kMode, bool kFull>
__device__ __forceinline__ void tile_pairs(const SphArgs &A, SphLane &L, const SphTile &T, int nt, bool tc) {
  const double hi = L.hd.x;
  // (2 max(h_i, h_j))^2 as the larger of the two staged squares: squaring
  // is monotone, so it is the same rounded value
  const double R2i = (2.0 * hi) * (2.0 * hi);
  uint64_t mask = tile_mask(nt, [&](int j) {
    const double4 b = T.pos[j];
    const double r2x = A.L > 0.0 ? dist2_disp(wrap_d(L.a.x - b.x, A.L), wrap_d(L.a.y - b.y, A.L),
                                              wrap_d(L.a.z - b.z, A.L))
                                 : dist2_pair(L.a.x, L.a.y, L.a.z, b.x, b.y, b.z);
    return L.sink && r2x < fmax(R2i, b.w);
  });
  const double ihi = 1.0 / hi, imi = 1.0 / L.a.w;
  const double ihi4 = ihi * ihi * ihi * ihi * kInvPiS;
  while (mask) {
    const int j = __builtin_ctzll(mask);
    mask &= mask - 1;
    const int q = T.q[j];
    if (q == L.p) continue;  // the sink itself
    if constexpr (kMode == 2) {
      L.bm = min(L.bm, A.bcur_s[q]);
      atomicMin(A.bw + A.perm[q], L.bw);
      continue;
    }
    const SphRec b = A.srec[q];
    if (L.dbg) {
      if (L.ndbg < A.dbg_max) L.dbg[L.ndbg] = A.perm[q];
      L.ndbg++;
    }
    L.npair++;
    double dx = L.a.x - b.x, dy = L.a.y - b.y, dz = L.a.z - b.z;
    if (A.L > 0.0) {  // the nearest image
      dx = wrap_d(dx, A.L);
      dy = wrap_d(dy, A.L);
      dz = wrap_d(dz, A.L);
    }
    const double r2 = dist2_disp(dx, dy, dz);
    if (!(r2 > 0.0)) continue;
    const double ir = rsq64(r2);
    const double r = r2 * ir;
    if constexpr (kMode == 1) {
      const double g = m4_dw(r * ihi) * ihi4 * ir;  // dW/dr(r, h_i) / r, zero beyond 2 h_i
      const double vx = L.v.x - b.vx, vy = L.v.y - b.vy, vz = L.v.z - b.vz;
      L.xsx += g * (vy * dz - vz * dy);
      L.xsy += g * (vz * dx - vx * dz);
      L.xsz += g * (vx * dy - vy * dx);
      continue;
    }
    const double ihj2 = b.ih * b.ih;
    const double gi = m4_grad(r * ihi, tc) * ihi4 * ir;
    const double gj = m4_grad(r * b.ih, tc) * (ihj2 * ihj2 * kInvPiS) * ir;
    const double mj = b.m;
    const double fij = L.fa + L.zi * b.im;
    const double fji = b.fa + b.zo * imi;
    const double Ai = L.hd.w * fij;
    const double Aj = b.pr2 * fji;
    const double vx = L.v.x - b.vx, vy = L.v.y - b.vy, vz = L.v.z - b.vz;
    const double vd = vx * dx + vy * dy + vz * dz;
    double sf = mj * (Ai * gi + Aj * gj);
    double e = mj * Ai * gi * vd;
    const double cb = 0.5 * (L.hd.z + b.c);
    const double rb = 0.5 * (L.hd.y + b.rho);
    const double w = vd * ir;  // v_ij . x_ij / r
    if (vd < 0.0) {
      const double hb = 0.5 * (hi + b.h);
      const double mu = hb * vd / (r2 + A.av_eps2 * hb * hb);
      // per-particle alpha: the pair mean replaces alpha; Balsara: times the
      // pair mean of f (Sect. 3.3.1)
      const double4 e2j = (kFull && A.f2) ? A.srec2[q] : make_double4(A.alpha, 0.0, 1.0, 0.0);
      const double al = (kFull && A.alpha_switch) ? 0.5 * (L.e2.x + e2j.x) : A.alpha;
      double Pi = A.visc_signal ? -al * (2.0 * cb - w) * w / rb : (-al * cb * mu + A.beta * mu * mu) / rb;
      if (kFull && A.balsara) Pi *= 0.5 * (L.e2.z + e2j.z);
      const double Gb = 0.5 * (fij * gi + fji * gj);
      sf += mj * Pi * Gb;
      const double ev = 0.5 * mj * Pi * Gb * vd;
      e += ev;
      L.duv += ev;
      L.mumax = fmax(L.mumax, fabs(mu));
    }
    L.vsig = fmax(L.vsig, 2.0 * cb - fmin(w, 0.0));
    if (kFull && A.conduction) {
      // artificial conductivity (Sect. 3.3.2) through |Gbar| = |Gb| r, and
      // Brookshaw's Laplacian of u
      const double4 e2j = A.srec2[q];
      const double Gbm = fabs(0.5 * (fij * gi + fji * gj)) * r;
      const double du_ij = L.e2.w - e2j.w;
      const double Pd = L.hd.w * L.hd.y * L.hd.y - b.pr2 * b.rho * b.rho;  // P_i - P_j
      const double Piu = -0.5 * (L.e2.y + e2j.y) * sqrt(fabs(Pd) / rb) * du_ij / rb;
      e += mj * Piu * Gbm;
      L.lapu -= 2.0 * mj * du_ij / b.rho * Gbm * ir;
    }
    if (kFull && A.xsph_eta > 0.0) {
      double wi, dwi, wj, dwj;
      m4(r * ihi, wi, dwi);
      m4(r * b.ih, wj, dwj);
      const double wb = 0.5 * (wi * (ihi * ihi * ihi) + wj * (b.ih * b.ih * b.ih)) * kInvPiS / rb;
      L.xsx -= mj * vx * wb;
      L.xsy -= mj * vy * wb;
      L.xsz -= mj * vz * wb;
    }
    L.ax -= sf * dx;
    L.ay -= sf * dy;
    L.az -= sf * dz;
    L.du += e;
  }
  __syncthreads();
}

// The force pass of tile_pairs with single-precision pair arithmetic (the
// same pairs, in the same order).
template <bool kFull>
__device__ __forceinline__ void tile_pairs32(const SphArgs &A, SphLane &L, const SphTile &T, int nt, bool tc) {
  const double hi = L.hd.x;
  // (2 max(h_i, h_j))^2 as the larger of the two staged squares: squaring
  // is monotone, so it is the same rounded value
  const double R2i = (2.0 * hi) * (2.0 * hi);
  uint64_t mask = tile_mask(nt, [&](int j) {
    const double4 b = T.pos[j];
    const double r2x = A.L > 0.0 ? dist2_disp(wrap_d(L.a.x - b.x, A.L), wrap_d(L.a.y - b.y, A.L),
                                              wrap_d(L.a.z - b.z, A.L))
                                 : dist2_pair(L.a.x, L.a.y, L.a.z, b.x, b.y, b.z);
    return L.sink && r2x < fmax(R2i, b.w);
  });
  const float ihi = (float)(1.0 / hi), imi = (float)(1.0 / L.a.w), hif = (float)hi;
  const float ihi4 = ihi * ihi * ihi * ihi * (float)kInvPiS;
  const float vix = (float)L.v.x, viy = (float)L.v.y, viz = (float)L.v.z;
  const float fai = (float)L.fa, zii = (float)L.zi;
  const float rhoi = (float)L.hd.y, ci = (float)L.hd.z, pri = (float)L.hd.w;
  const float alpha = (float)A.alpha, beta = (float)A.beta, aveps2 = (float)A.av_eps2;
  float ax = 0.0f, ay = 0.0f, az = 0.0f, du = 0.0f, duv = 0.0f, mumax = 0.0f, vsig = 0.0f;
  float xsx = 0.0f, xsy = 0.0f, xsz = 0.0f, lapu = 0.0f;
  while (mask) {
    const int j = __builtin_ctzll(mask);
    mask &= mask - 1;
    const int q = T.q[j];
    if (q == L.p) continue;  // the sink itself
    const SphRec32 b = A.srec32[q];
    if (L.dbg) {
      if (L.ndbg < A.dbg_max) L.dbg[L.ndbg] = A.perm[q];
      L.ndbg++;
    }
    L.npair++;
    const double4 pj = T.pos[j];
    double ddx = L.a.x - pj.x, ddy = L.a.y - pj.y, ddz = L.a.z - pj.z;
    if (A.L > 0.0) {  // the nearest image
      ddx = wrap_d(ddx, A.L);
      ddy = wrap_d(ddy, A.L);
      ddz = wrap_d(ddz, A.L);
    }
    const float dx = (float)ddx, dy = (float)ddy, dz = (float)ddz;
    const float r2 = dx * dx + dy * dy + dz * dz;
    if (!(r2 > 0.0f)) continue;
    const float ir = rsq32(r2);
    const float r = r2 * ir;
    const float ihj2 = b.ih * b.ih;
    const float gi = m4_grad(r * ihi, tc) * ihi4 * ir;
    const float gj = m4_grad(r * b.ih, tc) * (ihj2 * ihj2 * (float)kInvPiS) * ir;
    const float mj = b.m;
    const float fij = fai + zii * b.im;
    const float fji = b.fa + b.zo * imi;
    const float Ai = pri * fij;
    const float Aj = b.pr2 * fji;
    const float vx = vix - b.vx, vy = viy - b.vy, vz = viz - b.vz;
    const float vd = vx * dx + vy * dy + vz * dz;
    float sf = mj * (Ai * gi + Aj * gj);
    float e = mj * Ai * gi * vd;
    const float cb = 0.5f * (ci + b.c);
    const float rb = 0.5f * (rhoi + b.rho);
    const float irb = rcp32(rb);
    const float w = vd * ir;  // v_ij . x_ij / r
    double4 e2j = make_double4(0.0, 0.0, 1.0, 0.0);
    if (kFull && A.f2) e2j = A.srec2[q];
    if (vd < 0.0f) {
      const float hb = 0.5f * (hif + b.h);
      const float mu = hb * vd * rcp32(r2 + aveps2 * hb * hb);
      const float al = (kFull && A.alpha_switch) ? 0.5f * (float)(L.e2.x + e2j.x) : alpha;
      float Pi = A.visc_signal ? -al * (2.0f * cb - w) * w * irb : (-al * cb * mu + beta * mu * mu) * irb;
      if (kFull && A.balsara) Pi *= 0.5f * (float)(L.e2.z + e2j.z);
      const float Gb = 0.5f * (fij * gi + fji * gj);
      sf += mj * Pi * Gb;
      const float ev = 0.5f * mj * Pi * Gb * vd;
      e += ev;
      duv += ev;
      mumax = fmaxf(mumax, fabsf(mu));
    }
    vsig = fmaxf(vsig, 2.0f * cb - fminf(w, 0.0f));
    if (kFull && A.conduction) {
      const float Gbm = fabsf(0.5f * (fij * gi + fji * gj)) * r;
      const float du_ij = (float)(L.e2.w - e2j.w);
      const float Pd = pri * rhoi * rhoi - b.pr2 * b.rho * b.rho;  // P_i - P_j
      const float Piu = -0.5f * (float)(L.e2.y + e2j.y) * sqrtf(fabsf(Pd) * irb) * du_ij * irb;
      e += mj * Piu * Gbm;
      lapu -= 2.0f * mj * du_ij * rcp32(b.rho) * Gbm * ir;
    }
    if (kFull && A.xsph_eta > 0.0) {
      float wi, dwi, wj, dwj;
      m4_t(r * ihi, wi, dwi);
      m4_t(r * b.ih, wj, dwj);
      const float wb = 0.5f * (wi * (ihi * ihi * ihi) + wj * (b.ih * b.ih * b.ih)) * (float)kInvPiS * irb;
      xsx -= mj * vx * wb;
      xsy -= mj * vy * wb;
      xsz -= mj * vz * wb;
    }
    ax -= sf * dx;
    ay -= sf * dy;
    az -= sf * dz;
    du += e;
  }
  L.ax += (double)ax;
  L.ay += (double)ay;
  L.az += (double)az;
  L.du += (double)du;
  L.duv += (double)duv;
  L.mumax = fmax(L.mumax, (double)mumax);
  L.vsig = fmax(L.vsig, (double)vsig);
  if (kFull) {
    L.xsx += (double)xsx;
    L.xsy += (double)xsy;
    L.xsz += (double)xsz;
    L.lapu += (double)lapu;
  }
  __syncthreads();
}

// one tile of the pass of mode kMode
template <int kMode, bool kFull>
__device__ __forceinline__ void tile_eval(const SphArgs &A, SphLane &L, const SphTile &T, int nt, bool tc) {
  if constexpr (kMode == 3)
    tile_pairs32<kFull>(A, L, T, nt, tc);
  else
    tile_pairs<kMode, kFull>(A, L, T, nt, tc);
}

// The gas among the candidates of the lanes' raw slots (slot ln holds
// candidate q, nt valid) appended to the tile of gas candidates, which holds
// fill of them: a full tile is evaluated and the remainder carried over to
// the next.  Non-gas candidates never reach the pair tests, and each lane
// still meets its pairs in candidate order.  Returns the new fill.
template <int kMode, bool kFull>
__device__ __forceinline__ int stage_gas(const SphArgs &A, SphLane &L, SphTile &T, int nt, int q, int fill, bool tc) {
  const int ln = lane();
  // the species flag and the leading part of the record in one round trip
  // (a non-gas record is read but not used)
  const bool in = ln < nt;
  const bool g = in && A.gas[q] != 0;
  const SphRec *r = A.srec + (in ? q : 0);
  const double4 pos = make_double4(r->x, r->y, r->z, (2.0 * r->h) * (2.0 * r->h));
  const uint64_t gm = ballot(g);
  const int slot = fill + mbcnt(gm);
  const int ng = __popcll(gm);
  if (g && slot < kWave) {
    T.pos[slot] = pos;
    T.q[slot] = q;
  }
  __syncthreads();
  if (fill + ng < kWave) return fill + ng;
  tile_eval<kMode, kFull>(A, L, T, kWave, tc);
  // the remainder (its record read again: fewer registers live across the
  // pair evaluation)
  if (g && slot >= kWave) {
    const SphRec *r = A.srec + q;
    T.pos[slot - kWave] = make_double4(r->x, r->y, r->z, (2.0 * r->h) * (2.0 * r->h));
    T.q[slot - kWave] = q;
  }
  __syncthreads();
  return fill + ng - kWave;
}

// particle ranges (first, count) of listed leaves, or given explicitly
struct SphLeafSrc {
  const NodeTopo *topo;
  const int *leaf;
  __device__ int2 operator()(int i) const {
    const NodeTopo t = topo[leaf[i]];
    return make_int2(t.first, t.count);
  }
};
struct SphRangeSrc {
  const int2 *rng;
  __device__ int2 operator()(int i) const { return rng[i]; }
};

// Pairs of the lane's sink with the particles of ranges [0, n), packed 64
// to a tile in range order.  Returns the number of particles scanned.
template <int kMode, bool kFull, class Src>
__device__ __forceinline__ int sph_ranges(const SphArgs &A, SphLane &L, SphTile &T, const Src &src, int n, bool tc) {
  const int ln = lane();
  int fill = 0, rq = 0, scanned = 0, gfill = 0;
  for (int c1 = 0; c1 < n; c1 += kWave) {
    const int nc = min(kWave, n - c1);
    const int2 my = ln < nc ? src(c1 + ln) : make_int2(0, 0);
    for (int j = 0; j < nc; j++) {
      const int first = __builtin_amdgcn_readlane(my.x, j);
      const int count = __builtin_amdgcn_readlane(my.y, j);
      scanned += count;
      for (int off = 0; off < count;) {
        const int tk = min(count - off, kWave - fill);
        if (ln >= fill && ln < fill + tk) rq = first + off + (ln - fill);
        fill += tk;
        off += tk;
        if (fill == kWave) {
          gfill = stage_gas<kMode, kFull>(A, L, T, kWave, rq, gfill, tc);
          fill = 0;
        }
      }
    }
  }
  if (fill > 0) gfill = stage_gas<kMode, kFull>(A, L, T, fill, rq, gfill, tc);
  if (gfill > 0) tile_eval<kMode, kFull>(A, L, T, gfill, tc);
  return scanned;
}

// The gas particles c0 .. c0 + 63 of batch bt (in key order) listed in
// s_gs: the lanes of one chunk of the batch's gas sinks.  The SPH batches are
// packed by gas count, so one chunk holds them all unless a single group has
// more than 64 (an unsplittable clump).
__device__ __forceinline__ void gas_sinks(const SphArgs &A, const Batch &bt, int c0, int *s_gs) {
  const int ln = lane();
  int n = 0;
  __syncthreads();
  for (int o = 0; o < bt.count && n < c0 + kWave; o += kWave) {
    const int q = bt.first + o + ln;
    const bool g = o + ln < bt.count && A.gas[q] != 0;
    const uint64_t m = ballot(g);
    const int slot = n + mbcnt(m) - c0;
    if (g && slot >= 0 && slot < kWave) s_gs[slot] = q;
    n += __popcll(m);
  }
  __syncthreads();
}

// kPer: the periodic-box form; the open one takes L = 0 as a constant, so
// that no nearest-image code is left in it
template <int kMode, bool kFull, bool kPer>
__global__ __launch_bounds__(64, 4) void k_sph(SphArgs A) {
  if constexpr (!kPer) A.L = 0.0;
  __shared__ int s_stack[kSStackCap];
  __shared__ int s_leaf[kSListCap];
  __shared__ double4 s_snk[kSnkRecs];
  __shared__ SphTile s_t;
  __shared__ int s_g;
  __shared__ int s_gs[kWave];
  const int ln = lane();
  const int ng = *A.nbatches;
  const bool tc = A.tc92 != 0;
  for (;;) {
    if (ln == 0) s_g = xcd_next(A.work + 24, ng);
    __syncthreads();
    const int g = s_g;
    __syncthreads();
    if (g < 0) break;
    const Batch bt = load_batch(A.batches, A.groups, A.topo, A.nbox, A.nngas, A.mem, g);
    if (bt.ngas == 0) continue;
    const NodeBox gb = bt.box;
    const double ghmax = gb.hmax;
    const int ngs = bt.ngas;
    int prev_item = -1;  // last handed-off item of this batch
    for (int c0 = 0; c0 < ngs; c0 += kWave) {
      gas_sinks(A, bt, c0, s_gs);
      const bool act = c0 + ln < ngs;
      const int p = act ? s_gs[ln] : bt.first;
      SphLane L;
      // the force and wake-up passes of individual time-steps take active
      // sinks only
      sph_lane<kFull>(A, L, p, act && ((!force_mode(kMode) && kMode != 2) || !A.act || A.act[p]));
      if (ballot(L.sink) == 0) continue;
      if (kMode == 2) {
        L.dbg = nullptr;
        if (L.sink) L.bw = A.bcur_s[p];
      }
      const double hi = L.hd.x;
      int done = 0;  // candidates evaluated by this wave
      int sp = 1, nleaf = 0;
      bool overflow = false;
      int rounds = 0;
      const int guard = *A.nnodes + 2;
      if (ln == 0) s_stack[0] = bt.root;
      const double4 ball = make_double4(L.a.x, L.a.y, L.a.z, L.sink ? 2.0 * hi : 0.0);
      s_snk[ln] = ball;
      if constexpr (kPer) stage_ball_groups_p(s_snk, ball, A.L);
      else stage_ball_groups(s_snk, ball);
      __syncthreads();
      for (;;) {
        if (sp > 0 && ++rounds > guard) {
          atomicOr(A.flags, TSPH_FLAG_INTERNAL);
          overflow = true;
        }
        if (sp > 0 && !overflow) {
          const int take = walk_take(sp, kSStackCap);
          const int k = ln < take ? s_stack[sp - take + ln] : -1;
          sp -= take;
          __syncthreads();
          bool hit = false, leaf = false;
          NodeTopo nd{0, 0, -1, 0};
          // box, gas count and topology in one round trip
          NodeBox b = A.nbox[k >= 0 ? k : 0];
          const NodeTopo ndk = A.topo[k >= 0 ? k : 0];
          if (k >= 0 && A.nngas[k] > 0) {
            double d2 = axis_gap_box_p(gb.lox, gb.hix, b.lox, b.hix, A.L);
            d2 = d2 + axis_gap_box_p(gb.loy, gb.hiy, b.loy, b.hiy, A.L);
            d2 = d2 + axis_gap_box_p(gb.loz, gb.hiz, b.loz, b.hiz, A.L);
            const double R = 2.0 * fmax(ghmax, b.hmax);
            hit = d2 < R * R;
          }
          // keep the node only if some gas sink reaches it: |x_i - box| < 2 max(h_i, h_node)
          hit = balls_reach_box(s_snk, b.lox, b.loy, b.loz, b.hix, b.hiy, b.hiz, 2.0 * b.hmax, hit, A.L) && hit;
          if (hit) {
            nd = ndk;
            leaf = nd.nchild == 0;
          }
          const uint64_t lm = ballot(leaf);
          if (leaf) s_leaf[nleaf + mbcnt(lm)] = k;
          nleaf += __popcll(lm);
          const int nch = (hit && !leaf) ? nd.nchild : 0;
          const int incl = wave_incl_scan(nch);
          const int tot = __shfl(incl, kWave - 1, kWave);
          if (sp + tot > kSStackCap) {
            overflow = true;
          } else {
            for (int q = 0; q < nch; q++) s_stack[sp + incl - nch + q] = nd.child + q;
            sp += tot;
          }
          __syncthreads();
        }
        const bool last = (sp == 0) || overflow;
        if (nleaf >= kSLeafFlush || (last && nleaf > 0)) {
          bool handed = false;
          if (A.split_particles > 0 && done >= A.split_particles) {
            // this flush's leaves as one work item for k_sph_split
            int rb = 0, it = 0;
            if (ln == 0) {
              rb = atomicAdd(&A.work[34], nleaf);
              it = rb + nleaf <= A.split_cap * kSplitItemRanges ? atomicAdd(&A.work[35], 1) : INT32_MAX;
            }
            rb = __shfl(rb, 0, kWave);
            it = __shfl(it, 0, kWave);
            if (it < A.split_cap) {
              for (int a = ln; a < nleaf; a += kWave) {
                const NodeTopo t = A.topo[s_leaf[a]];
                A.split_rng[rb + a] = make_int2(t.first, t.count);
              }
              if (ln == 0) {
                A.split_item[it] = SplitItem{g, c0, rb, nleaf, -1, 0, 0, 0};
                if (prev_item >= 0) A.split_item[prev_item].next = it;
                else A.split_head[g] = it;
              }
              prev_item = it;
              handed = true;
            } else if (ln == 0) {
              atomicOr(A.flags, TSPH_FLAG_HANDOFF_CAPACITY);
            }
          }
          if (!handed) done += sph_ranges<kMode, kFull>(A, L, s_t, SphLeafSrc{A.topo, s_leaf}, nleaf, tc);
          nleaf = 0;
        }
        __syncthreads();
        if (last) break;
      }
      if (overflow) atomicOr(A.flags, TSPH_FLAG_STACK_OVERFLOW);
      if (L.dbg && L.ndbg > A.dbg_max) atomicOr(A.flags, TSPH_FLAG_LIST_OVERFLOW);
      if (kMode == 1 && L.sink) {
        // the batch's own share of the curl sum; handed-off items add theirs
        // (k_sph_reduce) before k_curl_finish normalises it
        A.solve[kCurlx * A.cap_n + p] = L.xsx;
        A.solve[kCurly * A.cap_n + p] = L.xsy;
        A.solve[kCurlz * A.cap_n + p] = L.xsz;
      }
      if (kMode == 2 && L.sink) A.bm[A.perm[p]] = L.bm;
      if (force_mode(kMode) && L.sink) {
        A.acc[0 * A.cap_n + p] += L.ax;
        A.acc[1 * A.cap_n + p] += L.ay;
        A.acc[2 * A.cap_n + p] += L.az;
        A.acc[4 * A.cap_n + p] = L.du;
        A.solve[kMaxmu * A.cap_n + p] = L.mumax;
        A.solve[kVsig * A.cap_n + p] = L.vsig;
        A.solve[kDuv * A.cap_n + p] = L.duv;
        A.solve[kXsx * A.cap_n + p] = L.xsx;
        A.solve[kXsy * A.cap_n + p] = L.xsy;
        A.solve[kXsz * A.cap_n + p] = L.xsz;
        A.solve[kLapu * A.cap_n + p] = L.lapu;
        A.cnt[2 * A.cap_n + A.perm[p]] = L.npair;
      }
    }
  }
}

// The handed-off flushes: each item's ranges on the sinks of its batch
// chunk; per-lane partial sums to split_part (kSphPart records per lane).
template <int kMode, bool kFull, bool kPer>
__global__ __launch_bounds__(64, 4) void k_sph_split(SphArgs A) {
  if constexpr (!kPer) A.L = 0.0;
  __shared__ int2 s_rng[kSplitItemRanges];
  __shared__ SphTile s_t;
  __shared__ int s_i;
  __shared__ int s_gs[kWave];
  const int ln = lane();
  const bool tc = A.tc92 != 0;
  const int nitems = (int)min((int64_t)A.work[35], A.split_cap);
  for (;;) {
    if (ln == 0) s_i = atomicAdd(&A.work[36], 1);
    __syncthreads();
    const int it = s_i;
    __syncthreads();
    if (it >= nitems) break;
    const SplitItem I = A.split_item[it];
    const Batch bt = load_batch(A.batches, A.groups, A.topo, A.nbox, A.nngas, A.mem, I.g);
    gas_sinks(A, bt, I.c0, s_gs);
    const bool act = I.c0 + ln < bt.ngas;
    const int p = act ? s_gs[ln] : bt.first;
    SphLane L;
    sph_lane<kFull>(A, L, p, act && (kMode == 1 || !A.act || A.act[p]));
    L.dbg = nullptr;
    for (int a = ln; a < I.count; a += kWave) s_rng[a] = A.split_rng[I.start + a];
    __syncthreads();
    sph_ranges<kMode, kFull>(A, L, s_t, SphRangeSrc{s_rng}, I.count, tc);
    double4 *part = A.split_part + (int64_t)kSphPart * it * kWave;
    part[ln] = make_double4(L.ax, L.ay, L.az, L.du);
    part[kWave + ln] = make_double4(L.mumax, (double)L.npair, L.duv, L.vsig);
    part[2 * kWave + ln] = make_double4(L.xsx, L.xsy, L.xsz, L.lapu);
  }
}

// Adds the items' partial sums to each batch's sinks along the batch's item
// chain (creation order).
template <int kMode>
__global__ __launch_bounds__(64) void k_sph_reduce(SphArgs A) {
  __shared__ int s_gs[kWave];
  const int ln = lane();
  const int ng = *A.nbatches;
  for (int g = blockIdx.x; g < ng; g += gridDim.x) {
    int it = A.split_head[g];
    if (it < 0) continue;
    const Batch bt = load_batch(A.batches, A.groups, A.topo, A.nbox, A.nngas, A.mem, g);
    int guard = 0;
    while (it >= 0 && it < A.split_cap && ++guard <= A.split_cap) {
      const SplitItem I = A.split_item[it];
      gas_sinks(A, bt, I.c0, s_gs);
      const int p = I.c0 + ln < bt.ngas ? s_gs[ln] : bt.first;
      if (kMode == 1 && I.c0 + ln < bt.ngas) {
        const double4 x = A.split_part[(int64_t)kSphPart * it * kWave + 2 * kWave + ln];
        A.solve[kCurlx * A.cap_n + p] += x.x;
        A.solve[kCurly * A.cap_n + p] += x.y;
        A.solve[kCurlz * A.cap_n + p] += x.z;
      } else if (I.c0 + ln < bt.ngas) {
        const double4 *part = A.split_part + (int64_t)kSphPart * it * kWave;
        const double4 v = part[ln], w = part[kWave + ln], x = part[2 * kWave + ln];
        A.acc[0 * A.cap_n + p] += v.x;
        A.acc[1 * A.cap_n + p] += v.y;
        A.acc[2 * A.cap_n + p] += v.z;
        A.acc[4 * A.cap_n + p] += v.w;
        A.solve[kMaxmu * A.cap_n + p] = fmax(A.solve[kMaxmu * A.cap_n + p], w.x);
        A.cnt[2 * A.cap_n + A.perm[p]] += (int)w.y;
        A.solve[kDuv * A.cap_n + p] += w.z;
        A.solve[kVsig * A.cap_n + p] = fmax(A.solve[kVsig * A.cap_n + p], w.w);
        A.solve[kXsx * A.cap_n + p] += x.x;
        A.solve[kXsy * A.cap_n + p] += x.y;
        A.solve[kXsz * A.cap_n + p] += x.z;
        A.solve[kLapu * A.cap_n + p] += x.w;
      }
      it = I.next;
    }
  }
}

// The curl with the divergence's normalisation, the Balsara factor and the
// switches' record of every gas particle (key order).
__global__ __launch_bounds__(256) void k_curl_finish(SphArgs A, int64_t n) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    if (!A.gas[p]) continue;
    const double nom = A.solve[kNh * A.cap_n + p] * A.solve[kOmega * A.cap_n + p];
    const double cx = A.solve[kCurlx * A.cap_n + p] / nom, cy = A.solve[kCurly * A.cap_n + p] / nom,
                 cz = A.solve[kCurlz * A.cap_n + p] / nom;
    A.solve[kCurlx * A.cap_n + p] = cx;
    A.solve[kCurly * A.cap_n + p] = cy;
    A.solve[kCurlz * A.cap_n + p] = cz;
    const double4 hd = A.sph[p];
    const double dv = fabs(A.solve[kDivv * A.cap_n + p]);
    const double fb = dv / (dv + sqrt(cx * cx + cy * cy + cz * cz) + 1e-4 * hd.z / hd.x);
    A.solve[kFbal * A.cap_n + p] = fb;
    const double2 al = A.av[p];
    A.srec2[p] = make_double4(A.alpha_switch ? al.x : A.alpha, al.y, fb, A.vu[p].w);
  }
}

__global__ __launch_bounds__(256) void k_zero_sph(int64_t n, int64_t cap_n, double *__restrict__ acc,
                                                  double *__restrict__ solve, int32_t *__restrict__ cnt,
                                                  const int32_t *__restrict__ perm) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    acc[4 * cap_n + p] = 0.0;
    solve[kMaxmu * cap_n + p] = 0.0;
    solve[kVsig * cap_n + p] = 0.0;
    solve[kDuv * cap_n + p] = 0.0;
    solve[kXsx * cap_n + p] = 0.0;
    solve[kXsy * cap_n + p] = 0.0;
    solve[kXsz * cap_n + p] = 0.0;
    solve[kLapu * cap_n + p] = 0.0;
    solve[kCurlx * cap_n + p] = 0.0;
    solve[kCurly * cap_n + p] = 0.0;
    solve[kCurlz * cap_n + p] = 0.0;
    solve[kFbal * cap_n + p] = 1.0;
    cnt[2 * cap_n + perm[p]] = 0;
  }
}

// alpha and alpha_u of the state (caller order; NULL: the fixed alpha, 0)
// gathered into key order
__global__ __launch_bounds__(256) void k_gather_alpha(int64_t n, const int32_t *__restrict__ perm,
                                                      const double *__restrict__ alpha,
                                                      const double *__restrict__ alpha_u, double2 *__restrict__ av) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const int i = perm[p];
    av[p] = make_double2(alpha ? alpha[i] : 0.0, alpha_u ? alpha_u[i] : 0.0);
  }
}

// the wake-up pass's minima over active neighbours start at "none"
__global__ __launch_bounds__(256) void k_wake_clear(int64_t n, int32_t *__restrict__ bw) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    bw[i] = INT32_MAX;
}

// zero k work-queue counters (the curl pass used the SPH walk's queues)
__global__ void k_reset_counter(int32_t *ctr, int k) {
  if ((int)threadIdx.x < k) ctr[threadIdx.x] = 0;
}

}  // namespace tsph

using namespace tsph;

// the periodic or the open form of a walk kernel
template <int kMode, bool kFull>
static void launch_sph(Ctx *c, const SphArgs &A, hipStream_t st) {
  if (A.L > 0.0) {
    const void *k = (const void *)k_sph<kMode, kFull, true>;
    hipLaunchKernelGGL((k_sph<kMode, kFull, true>), dim3(persistent_blocks(c, k)), dim3(64), 0, st, A);
  } else {
    const void *k = (const void *)k_sph<kMode, kFull, false>;
    hipLaunchKernelGGL((k_sph<kMode, kFull, false>), dim3(persistent_blocks(c, k)), dim3(64), 0, st, A);
  }
}
template <int kMode, bool kFull>
static void launch_sph_split(Ctx *c, const SphArgs &A, hipStream_t st) {
  if (A.L > 0.0) {
    const void *k = (const void *)k_sph_split<kMode, kFull, true>;
    hipLaunchKernelGGL((k_sph_split<kMode, kFull, true>), dim3(persistent_blocks(c, k)), dim3(64), 0, st, A);
  } else {
    const void *k = (const void *)k_sph_split<kMode, kFull, false>;
    hipLaunchKernelGGL((k_sph_split<kMode, kFull, false>), dim3(persistent_blocks(c, k)), dim3(64), 0, st, A);
  }
}

static SphArgs sph_args(Ctx *c) {
  SphArgs A;
  A.cap_n = c->cap_n;
  A.groups = c->groups;
  A.ngroups = c->ngroups;
  A.batches = c->sbatches;
  A.nbatches = c->nsbatches;
  A.topo = c->topo;
  A.nbox = c->nbox;
  A.nngas = c->nngas;
  A.mem = members_of(c, c->n, c->n_gas);
  A.pm = c->pm;
  A.vu = c->vu;
  A.sph = c->sph;
  A.zo = c->zo;
  A.srec = c->srec;
  A.srec32 = c->srec32;
  A.gas = c->gas;
  A.perm = c->perm;
  A.nnodes = c->lvl + 46;
  A.acc = c->acc;
  A.solve = c->solve;
  A.cnt = c->cnt;
  A.work = c->work;
  A.flags = c->flags;
  A.dbg = c->dbg_nbr;
  A.dbg_max = c->dbg_max;
  A.alpha = c->p.alpha;
  A.beta = c->p.beta;
  A.av_eps2 = c->p.av_eps2;
  A.tc92 = c->p.tc92;
  A.gamma = c->p.gamma;
  A.xsph_eta = c->p.xsph_eta;
  A.visc_signal = c->p.visc_form == TSPH_VISC_SIGNAL;
  A.entropy = c->p.entropy;
  A.balsara = c->p.balsara;
  A.alpha_switch = c->p.alpha_switch;
  A.conduction = c->p.conduction;
  A.f2 = (A.balsara || A.alpha_switch || A.conduction) ? 1 : 0;
  A.srec2 = c->srec2;
  A.av = c->av;
  A.split_particles = 0;
  A.split_cap = split_cap_used(c) / kSphPart;
  A.split_rng = c->split_rng;
  A.split_item = c->split_item;
  A.split_part = c->split_part;
  A.split_head = c->split_head;
  A.act = nullptr;
  A.bcur_s = c->bcur_s;
  A.bm = c->bm;
  A.bw = c->bw;
  A.L = c->p.period;
  return A;
}

tsph_status tsph_impl_sph(Ctx *c, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_sph, dim3(blocks_for(c->n, 256, 8192)), dim3(256), 0, st, c->n, c->cap_n, c->acc,
                     c->solve, c->cnt, c->perm);
  if (!c->p.hydro || c->n_gas == 0) {
    TSPH_HIP_CHECK(c, hipGetLastError());
    return TSPH_OK;
  }
  SphArgs A = sph_args(c);
  A.act = c->blk_on ? c->bact_s : nullptr;
  // debug lists are written in the batch's own order: no hand-off then.  The
  // SPH pairs cost more per candidate than the near-field gravity pairs, so
  // the batch keeps a quarter of the gravity walk's share.
  A.split_particles = c->dbg_nbr ? 0 : c->p.split_leaves * c->p.leaf_size / 4;
  if (A.split_particles > 0)
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(c->cap_nodes, 256, 4096)), dim3(256), 0, st, c->cap_nodes,
                       c->split_head, -1);
  if (A.f2) {
    // the switches' inputs in key order, then the curl pass (its own walk,
    // with the same hand-off as the forces), the curl's normalisation and
    // Balsara factors, then the forces with the queues and hand-off reset
    hipLaunchKernelGGL(k_gather_alpha, dim3(blocks_for(c->n, 256, 8192)), dim3(256), 0, st, c->n, c->perm,
                       c->alpha_state, c->alpha_u_state, c->av);
    launch_sph<1, true>(c, A, st);
    if (A.split_particles > 0) {
      launch_sph_split<1, true>(c, A, st);
      hipLaunchKernelGGL(k_sph_reduce<1>, dim3(4096), dim3(64), 0, st, A);
      hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, A.work + 34, 3);
      hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(c->cap_nodes, 256, 4096)), dim3(256), 0, st, c->cap_nodes,
                         c->split_head, -1);
    }
    hipLaunchKernelGGL(k_curl_finish, dim3(blocks_for(c->n, 256, 8192)), dim3(256), 0, st, A, (int64_t)c->n);
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, A.work + 24, 8);
  }
  // the plain form without the switches, the conductivity and X-SPH; the
  // FP32-bulk form's pairs in single precision
  const bool full = A.f2 || A.xsph_eta > 0.0;
  const bool f32 = c->p.precision == TSPH_FP32_BULK;
  if (f32) {
    if (full)
      launch_sph<3, true>(c, A, st);
    else
      launch_sph<3, false>(c, A, st);
  } else {
    if (full)
      launch_sph<0, true>(c, A, st);
    else
      launch_sph<0, false>(c, A, st);
  }
  if (A.split_particles > 0) {
    if (f32) {
      if (full)
        launch_sph_split<3, true>(c, A, st);
      else
        launch_sph_split<3, false>(c, A, st);
    } else {
      if (full)
        launch_sph_split<0, true>(c, A, st);
      else
        launch_sph_split<0, false>(c, A, st);
    }
    hipLaunchKernelGGL(k_sph_reduce<0>, dim3(4096), dim3(64), 0, st, A);
  }
  TSPH_HIP_CHECK(c, hipGetLastError());
  return TSPH_OK;
}

// Wake-up minima of the individual time-steps: for every active gas particle
// the least current step length among its SPH neighbours (bm), and for every
// gas particle the least step among its active neighbours (bw), both walked
// from the active particles alone.
tsph_status tsph_impl_wake(Ctx *c, hipStream_t st) {
  if (!c->p.hydro || c->n_gas == 0) return TSPH_OK;
  // the active flags in key order (the opening force pass of the steps
  // gathers none: all particles are active then)
  tsph_status r = tsph_impl_gather_active(c, st);
  if (r != TSPH_OK) return r;
  SphArgs A = sph_args(c);
  A.act = c->bact_s;
  A.dbg = nullptr;
  A.split_particles = 0;
  hipLaunchKernelGGL(k_wake_clear, dim3(blocks_for(c->n_gas, 256, 1 << 16)), dim3(256), 0, st, (int64_t)c->n_gas,
                     A.bw);
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, A.work + 24, 8);
  launch_sph<2, false>(c, A, st);
  TSPH_HIP_CHECK(c, hipGetLastError());
  return TSPH_OK;
}
