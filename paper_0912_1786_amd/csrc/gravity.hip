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
// opened leaves to LDS lists.  Full lists are flushed: every lane (sink)
// evaluates every listed interaction, the node or particle record being read
// with wave-uniform loads.  Accepted nodes act unsoftened through their
// monopole and quadrupole; particles of opened leaves interact through
//   a_i -= G m_j 1/2 [phi'(r, eps_i) + phi'(r, eps_j)] r_hat
//   a_i -= G/2 [xi_i/Ups_i W'(r, eps_i) + (m_j/m_i) xi_j/Ups_j W'(r, eps_j)] r_hat
// (r_hat = (x_i - x_j)/r, xi carrying the neighbour masses).
#include <stdio.h>

#include "tsph_internal.h"

namespace tsph {

constexpr int kGStackCap = 2048;
constexpr int kGListCap = 128;
constexpr int kGCellFlush = 64;
constexpr int kGLeafFlush = 32;
constexpr double kPiG = 3.14159265358979323846;

struct GravArgs {
  int64_t cap_n;
  const int32_t *groups;
  const int32_t *ngroups;
  const NodeTopo *topo;
  const NodeBox *nbox;
  const NodeFar *nfar;
  const double4 *pm;
  const double2 *soft;
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
  double x, y, z, m, eps, xiu;
  double ax, ay, az, pot;
  int p;
  bool act;
  int32_t *dbg;
  int ndbg;
};

__device__ __forceinline__ void far_field(const GravArgs &A, Sink &s, const NodeFar &f) {
  const double dx = s.x - f.cx, dy = s.y - f.cy, dz = s.z - f.cz;
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double ir = 1.0 / sqrt(r2);
  const double ir2 = ir * ir;
  const double ir3 = ir * ir2;
  double fm = f.m * ir3;
  double ph = f.m * ir;
  double ex = 0.0, ey = 0.0, ez = 0.0;
  if (A.quadrupole) {
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
  s.pot -= A.G * ph;
}

__device__ __forceinline__ void near_pair(const GravArgs &A, Sink &s, const double4 &b, const double2 &sb) {
  const double dx = s.x - b.x, dy = s.y - b.y, dz = s.z - b.z;
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double ei = s.eps, ej = sb.x;
  const double em = fmax(ei, ej);
  if (r2 >= 4.0 * em * em) {
    const double ir = 1.0 / sqrt(r2);
    const double mr = b.w * ir;
    const double f = mr * ir * ir;
    s.ax -= A.G * f * dx;
    s.ay -= A.G * f * dy;
    s.az -= A.G * f * dz;
    s.pot -= A.G * mr;
    return;
  }
  if (r2 > 0.0) {
    const double r = sqrt(r2);
    double F = 0.5 * b.w * (soft_fr(r, ei) + soft_fr(r, ej));
    if (A.corr) {
      double wi, dwi, wj, dwj;
      m4(r / ei, wi, dwi);
      m4(r / ej, wj, dwj);
      const double Wi = dwi / (kPiG * ei * ei * ei * ei);
      const double Wj = dwj / (kPiG * ej * ej * ej * ej);
      F += 0.5 * (s.xiu * Wi + (b.w / s.m) * sb.y * Wj);
    }
    const double fr = A.G * F / r;
    s.ax -= fr * dx;
    s.ay -= fr * dy;
    s.az -= fr * dz;
    if (A.want_pot) s.pot += A.G * b.w * 0.5 * (soft_ph(r, ei) + soft_ph(r, ej));
  } else if (A.want_pot) {
    s.pot += A.G * b.w * 0.5 * (-1.4 / ei - 1.4 / ej);
  }
}

__global__ __launch_bounds__(64) void k_gravity(GravArgs A) {
  __shared__ int s_stack[kGStackCap];
  __shared__ int s_cell[kGListCap];
  __shared__ int s_leaf[kGListCap];
  __shared__ int s_g;
  const int ln = lane();
  const int ng = *A.ngroups;
  for (;;) {
    if (ln == 0) s_g = atomicAdd(&A.work[1], 1);
    __syncthreads();
    const int g = s_g;
    __syncthreads();
    if (g >= ng) break;
    const int gk = A.groups[g];
    const NodeTopo gnd = A.topo[gk];
    const NodeBox gb = A.nbox[gk];
    const double gemax = gb.epsmax;
    for (int c0 = 0; c0 < gnd.count; c0 += kWave) {
      Sink s;
      s.act = c0 + ln < gnd.count;
      s.p = gnd.first + c0 + (s.act ? ln : 0);
      {
        const double4 a = A.pm[s.p];
        const double2 e = A.soft[s.p];
        s.x = a.x; s.y = a.y; s.z = a.z; s.m = a.w;
        s.eps = e.x; s.xiu = e.y;
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
          for (int j = 0; j < ncell; j++) {
            const int k = uniform(s_cell[j]);
            const NodeFar f = A.nfar[k];
            far_field(A, s, f);
          }
          nfar += ncell;
          ncell = 0;
        }
        if (nleaf >= kGLeafFlush || (last && nleaf > 0)) {
          for (int j = 0; j < nleaf; j++) {
            const int k = uniform(s_leaf[j]);
            const NodeTopo nd = A.topo[k];
            for (int q = nd.first; q < nd.first + nd.count; q++) {
              const double4 b = A.pm[q];
              const double2 sb = A.soft[q];
              if (q != s.p) {
                near_pair(A, s, b, sb);
                if (s.dbg) {
                  const double r2 = dist2_pair(s.x, s.y, s.z, b.x, b.y, b.z);
                  const double R = 2.0 * fmax(s.eps, sb.x);
                  if (r2 < R * R) {
                    if (s.ndbg < A.dbg_max) s.dbg[s.ndbg] = A.perm[q];
                    s.ndbg++;
                  }
                }
              }
            }
            npair += nd.count;
          }
          nleaf = 0;
        }
        __syncthreads();
        if (last) break;
      }
      if (overflow) atomicOr(A.flags, TSPH_FLAG_STACK_OVERFLOW);
      if (s.dbg && s.ndbg > A.dbg_max) atomicOr(A.flags, TSPH_FLAG_LIST_OVERFLOW);
      if (s.act) {
        if (A.want_pot) s.pot += A.G * s.m * (-1.4 / s.eps);  // self term phi(0, eps_i)
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
  A.topo = c->topo;
  A.nbox = c->nbox;
  A.nfar = c->nfar;
  A.pm = c->pm;
  A.soft = c->soft;
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
  hipLaunchKernelGGL(k_gravity, dim3(256 * 8), dim3(64), 0, st, A);
  TSPH_HIP_CHECK(c, hipGetLastError());
  return TSPH_OK;
}
