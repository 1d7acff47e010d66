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

#include "tsph_internal.h"

namespace tsph {

constexpr int kGStackCap = 1024;
constexpr int kGListCap = 128;
constexpr int kGCellFlush = 64;
constexpr int kGLeafFlush = 32;
constexpr double kInvPiG = 0.31830988618379067154;

struct GravArgs {
  int64_t cap_n;
  const int32_t *groups;
  const int32_t *ngroups;
  const int2 *batches;
  const int32_t *nbatches;
  const int32_t *nngas;
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
  double G;
  int32_t quadrupole, corr, want_pot;
};

struct Sink {
  double x, y, z, m, im, eps, ieps, xiu;
  double ax, ay, az, pot;
  int p;
  bool act;
  int32_t *dbg;
  int ndbg;
};

// kernel variants: bit 0 quadrupoles, bit 1 correction terms, bit 2 potential
constexpr int kQuad = 1, kCorr = 2, kPot = 4;

template <int M>
__device__ __forceinline__ void far_field(const GravArgs &A, Sink &s, const NodeFar &f) {
  const double dx = s.x - f.cx, dy = s.y - f.cy, dz = s.z - f.cz;
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double ir = rsqrt(r2);
  const double ir2 = ir * ir;
  const double ir3 = ir * ir2;
  double fm = f.m * ir3;
  double ph = f.m * ir;
  double ex = 0.0, ey = 0.0, ez = 0.0;
  if (M & kQuad) {
    const double qx = f.qxx * dx + f.qxy * dy + f.qxz * dz;
    const double qy = f.qxy * dx + f.qyy * dy + f.qyz * dz;
    const double qz = f.qxz * dx + f.qyz * dy + f.qzz * dz;
    const double rqr = dx * qx + dy * qy + dz * qz;
    const double ir5 = ir3 * ir2;
    const double ir7 = ir5 * ir2;
    fm += 2.5 * rqr * ir7;
    ex = qx * ir5;
    ey = qy * ir5;
    ez = qz * ir5;
    ph += 0.5 * rqr * ir5;
  }
  s.ax += A.G * (ex - fm * dx);
  s.ay += A.G * (ey - fm * dy);
  s.az += A.G * (ez - fm * dz);
  if (M & kPot) s.pot -= A.G * ph;
}

// Newtonian pair (both lengths reached): the common case, branch free
template <int M>
__device__ __forceinline__ void newton_pair(const GravArgs &A, Sink &s, const GravRec &b) {
  const double dx = s.x - b.x, dy = s.y - b.y, dz = s.z - b.z;
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double ir = rsqrt(r2);
  const double mr = b.m * ir;
  const double f = A.G * mr * ir * ir;
  s.ax -= f * dx;
  s.ay -= f * dy;
  s.az -= f * dz;
  if (M & kPot) s.pot -= A.G * mr;
}

__device__ __forceinline__ bool softened(const Sink &s, const GravRec &b) {
  const double dx = s.x - b.x, dy = s.y - b.y, dz = s.z - b.z;
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double em = fmax(s.eps, b.eps);
  return r2 < 4.0 * em * em;
}

template <int M>
__device__ __forceinline__ void near_pair(const GravArgs &A, Sink &s, const GravRec &b) {
  const double dx = s.x - b.x, dy = s.y - b.y, dz = s.z - b.z;
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double em = fmax(s.eps, b.eps);
  if (r2 >= 4.0 * em * em) {
    const double ir = rsqrt(r2);
    const double mr = b.m * ir;
    const double f = A.G * mr * ir * ir;
    s.ax -= f * dx;
    s.ay -= f * dy;
    s.az -= f * dz;
    if (M & kPot) s.pot -= A.G * mr;
    return;
  }
  if (r2 > 0.0) {
    const double ir = rsqrt(r2);
    const double r = r2 * ir;
    const double qi = r * s.ieps, qj = r * b.ieps;
    double F = 0.5 * b.m * (soft_fr_q(qi, s.ieps, ir) + soft_fr_q(qj, b.ieps, ir));
    if (M & kCorr) {
      const double ii2 = s.ieps * s.ieps, ij2 = b.ieps * b.ieps;
      const double Wi = m4_dw(qi) * (ii2 * ii2) * kInvPiG;
      const double Wj = m4_dw(qj) * (ij2 * ij2) * kInvPiG;
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

__device__ __forceinline__ void debug_pair(const GravArgs &A, Sink &s, const GravRec &b, int q) {
  const double r2 = dist2_pair(s.x, s.y, s.z, b.x, b.y, b.z);
  const double R = 2.0 * fmax(s.eps, b.eps);
  if (r2 < R * R) {
    if (s.ndbg < A.dbg_max) s.dbg[s.ndbg] = A.perm[q];
    s.ndbg++;
  }
}

// Evaluates the nt particle records staged in rec (indices in tq) on sink s.
template <int M>
__device__ __forceinline__ void near_tile(const GravArgs &A, Sink &s, const GravRec *rec, const int *tq, int nt) {
  int j = 0;
  for (; j + 2 <= nt; j += 2) {
    const GravRec b0 = rec[j], b1 = rec[j + 1];
    const int q0 = tq[j], q1 = tq[j + 1];
    // the self pair and every pair inside 2 max(eps) take the general path
    const bool slow = q0 == s.p || q1 == s.p || softened(s, b0) || softened(s, b1);
    if (!__any(slow)) {
      newton_pair<M>(A, s, b0);
      newton_pair<M>(A, s, b1);
    } else {
      if (q0 != s.p) near_pair<M>(A, s, b0);
      if (q1 != s.p) near_pair<M>(A, s, b1);
    }
    if (s.dbg) {
      if (q0 != s.p) debug_pair(A, s, b0, q0);
      if (q1 != s.p) debug_pair(A, s, b1, q1);
    }
  }
  if (j < nt) {
    const GravRec b = rec[j];
    const int q = tq[j];
    if (q != s.p) {
      near_pair<M>(A, s, b);
      if (s.dbg) debug_pair(A, s, b, q);
    }
  }
}

template <int M>
__global__ __launch_bounds__(64) void k_gravity(GravArgs A) {
  __shared__ int s_stack[kGStackCap];
  __shared__ int s_cell[kGListCap];
  __shared__ int s_leaf[kGListCap];
  // staging tile: 64 node records (far flush) or 64 particle records (near
  // flush), filled with one vector load per lane and read back as broadcasts
  __shared__ union {
    NodeFar far[kWave];
    GravRec rec[kWave];
  } s_t;
  __shared__ int s_tq[kWave];
  __shared__ int s_g;
  NodeFar *const s_tile = s_t.far;
  GravRec *const s_rec = s_t.rec;
  const int ln = lane();
  const int ng = *A.nbatches;
  for (;;) {
    if (ln == 0) s_g = atomicAdd(&A.work[1], 1);
    __syncthreads();
    const int g = s_g;
    __syncthreads();
    if (g >= ng) break;
    const Batch bt = load_batch(A.batches, A.groups, A.topo, A.nbox, A.nngas, g);
    const NodeTopo gnd{bt.first, bt.count, -1, 0};
    const NodeBox gb = bt.box;
    const double gemax = gb.epsmax;
    for (int c0 = 0; c0 < gnd.count; c0 += kWave) {
      Sink s;
      s.act = c0 + ln < gnd.count;
      s.p = gnd.first + c0 + (s.act ? ln : 0);
      {
        const GravRec r = A.grec[s.p];
        s.x = r.x; s.y = r.y; s.z = r.z; s.m = r.m; s.im = 1.0 / r.m;
        s.eps = r.eps; s.ieps = r.ieps; s.xiu = r.xiu;
      }
      s.ax = s.ay = s.az = s.pot = 0.0;
      s.dbg = (A.dbg && s.act) ? A.dbg + ((int64_t)2 * A.cap_n + A.perm[s.p]) * A.dbg_max : nullptr;
      s.ndbg = 0;
      int nfar = 0, npair = 0;
      int sp = 1, ncell = 0, nleaf = 0;
      bool overflow = false;
      int rounds = 0;
      const int guard = *A.nnodes + 2;
      if (ln == 0) s_stack[0] = 0;
      __syncthreads();

      for (;;) {
        if (sp > 0 && ++rounds > guard) {
          atomicOr(A.flags, TSPH_FLAG_INTERNAL);
          overflow = true;
        }
        if (sp > 0 && !overflow) {
          const int take = walk_take(sp, kGStackCap);
          const int k = ln < take ? s_stack[sp - take + ln] : -1;
          sp -= take;
          __syncthreads();
          bool acc = false, leaf = false;
          NodeTopo nd{0, 0, -1, 0};
          if (k >= 0) {
            const NodeFar f = A.nfar[k];
            const NodeBox b = A.nbox[k];
            double d2 = axis_gap_point(gb.lox, gb.hix, f.cx);
            d2 = d2 + axis_gap_point(gb.loy, gb.hiy, f.cy);
            d2 = d2 + axis_gap_point(gb.loz, gb.hiz, f.cz);
            if (d2 > f.rmac * f.rmac) {
              double c2 = axis_gap_box(gb.lox, gb.hix, b.lox, b.hix);
              c2 = c2 + axis_gap_box(gb.loy, gb.hiy, b.loy, b.hiy);
              c2 = c2 + axis_gap_box(gb.loz, gb.hiz, b.loz, b.hiz);
              const double sr = 2.0 * fmax(gemax, b.epsmax);
              acc = c2 >= sr * sr;
            }
            if (!acc) {
              nd = A.topo[k];
              leaf = nd.nchild == 0;
            }
          }
          const uint64_t am = ballot(acc);
          if (acc) s_cell[ncell + mbcnt(am)] = k;
          ncell += __popcll(am);
          const uint64_t lm = ballot(leaf);
          if (leaf) s_leaf[nleaf + mbcnt(lm)] = k;
          nleaf += __popcll(lm);
          const int nch = (k >= 0 && !acc && !leaf) ? nd.nchild : 0;
          const int incl = wave_incl_scan(nch);
          const int tot = __shfl(incl, kWave - 1, kWave);
          if (sp + tot > kGStackCap) {
            overflow = true;
          } else {
            for (int a = 0; a < nch; a++) s_stack[sp + incl - nch + a] = nd.child + a;
            sp += tot;
          }
          __syncthreads();
        }
        const bool last = (sp == 0) || overflow;
        if (ncell >= kGCellFlush || (last && ncell > 0)) {
          // accepted nodes, 64 per tile
          for (int t0 = 0; t0 < ncell; t0 += kWave) {
            const int nt = min(kWave, ncell - t0);
            if (ln < nt) s_tile[ln] = A.nfar[s_cell[t0 + ln]];
            __syncthreads();
            for (int j = 0; j < nt; j++) far_field<M>(A, s, s_tile[j]);
            __syncthreads();
          }
          nfar += ncell;
          ncell = 0;
        }
        if (nleaf >= kGLeafFlush || (last && nleaf > 0)) {
          // particles of the opened leaves, packed 64 per tile: the leaves are
          // scanned in order, each lane noting the particle of its slot, and a
          // full tile is loaded with one vector load per lane
          int fill = 0, rq = -1;
          for (int c1 = 0; c1 < nleaf; c1 += kWave) {
            const int nc = min(kWave, nleaf - c1);
            const NodeTopo my = ln < nc ? A.topo[s_leaf[c1 + ln]] : NodeTopo{0, 0, -1, 0};
            for (int j = 0; j < nc; j++) {
              const int first = __builtin_amdgcn_readlane(my.first, j);
              const int count = __builtin_amdgcn_readlane(my.count, j);
              npair += count;
              for (int off = 0; off < count;) {
                const int tk = min(count - off, kWave - fill);
                if (ln >= fill && ln < fill + tk) rq = first + off + (ln - fill);
                fill += tk;
                off += tk;
                if (fill == kWave) {
                  s_rec[ln] = A.grec[rq];
                  s_tq[ln] = rq;
                  __syncthreads();
                  near_tile<M>(A, s, s_rec, s_tq, kWave);
                  __syncthreads();
                  fill = 0;
                }
              }
            }
          }
          if (fill > 0) {
            if (ln < fill) {
              s_rec[ln] = A.grec[rq];
              s_tq[ln] = rq;
            }
            __syncthreads();
            near_tile<M>(A, s, s_rec, s_tq, fill);
            __syncthreads();
          }
          nleaf = 0;
        }
        __syncthreads();
        if (last) break;
      }
      if (overflow) atomicOr(A.flags, TSPH_FLAG_STACK_OVERFLOW);
      if (s.dbg && s.ndbg > A.dbg_max) atomicOr(A.flags, TSPH_FLAG_LIST_OVERFLOW);
      if (s.act) {
        if (M & kPot) s.pot += A.G * s.m * (-1.4 * s.ieps);  // self term phi(0, eps_i)
        A.acc[0 * A.cap_n + s.p] = s.ax;
        A.acc[1 * A.cap_n + s.p] = s.ay;
        A.acc[2 * A.cap_n + s.p] = s.az;
        A.acc[3 * A.cap_n + s.p] = s.pot;
        const int ci = A.perm[s.p];
        A.cnt[0 * A.cap_n + ci] = nfar;
        A.cnt[1 * A.cap_n + ci] = npair - 1;
      }
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
  A.want_pot = want_pot ? 1 : 0;
  const int mode = (A.quadrupole ? kQuad : 0) | (A.corr ? kCorr : 0) | (A.want_pot ? kPot : 0);
  void (*kern)(GravArgs) = nullptr;
  switch (mode) {
    case 0: kern = k_gravity<0>; break;
    case 1: kern = k_gravity<1>; break;
    case 2: kern = k_gravity<2>; break;
    case 3: kern = k_gravity<3>; break;
    case 4: kern = k_gravity<4>; break;
    case 5: kern = k_gravity<5>; break;
    case 6: kern = k_gravity<6>; break;
    default: kern = k_gravity<7>; break;
  }
  hipLaunchKernelGGL(kern, dim3(persistent_blocks(c, (const void *)kern)), dim3(64), 0, st, A);
  TSPH_HIP_CHECK(c, hipGetLastError());
  return TSPH_OK;
}
