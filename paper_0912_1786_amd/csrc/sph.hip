// sph.hip -- SPH acceleration and heating over the symmetric neighbour set
// r_ij < 2 max(h_i, h_j).
//
// Merlin et al., arXiv:0912.1786: Sect. 3 (Eqs. dvdt, drhodr, dudrho,
// motionvarmass, thermalvarmass, Thomas & Couchman gradient), Sect. 3.1
// (symmetric neighbour definition), Sect. 3.3 (Eq. mu_visc and the averaged
// gradient), App. B.  With grad_i W_ij(h) = W'(r, h) (x_i - x_j)/r:
//   a_i  = -sum_j m_j [A_ij gW(h_i) + A_ji gW(h_j) + Pi_ij Gbar_ij]
//   du_i =  sum_j m_j [A_ij v_ij . gW(h_i) + 1/2 Pi_ij v_ij . Gbar_ij]
//   A_ij = (P_i / rho_i^2) f_ij,  f_ij = 1 + zeta_i / (m_j Omega*_i),
//   Gbar_ij = 1/2 [f_ij gW(h_i) + f_ji gW(h_j)],
//   Pi_ij = (-alpha cbar mu + beta mu^2) / rhobar  when v_ij . x_ij < 0,
//   mu = hbar v_ij . x_ij / (r^2 + av_eps2 hbar^2), bars = pair means,
// evaluated with the predicted velocities and energies.
//
// One wavefront per walk group that holds gas; the wave walks the tree once
// (opening nodes with gas within 2 max(h_group, h_node) of the group box),
// lists the candidate leaves in LDS and flushes them in batches.  A flush
// stages the candidates 64 at a time in LDS (position and h), every lane
// tests the whole tile and keeps a mask of its own pairs, and then each lane
// evaluates only its own pairs, in candidate order, reading the partner's
// record itself; lanes do not step through pairs that only other lanes have.
#include <stdio.h>

#include "tsph_internal.h"

namespace tsph {

constexpr int kSStackCap = 1024;
constexpr int kSListCap = 128;
constexpr int kSLeafFlush = 32;
constexpr double kInvPiS = 0.31830988618379067154;

// candidates of a flush staged for the pair tests
struct SphTile {
  double4 pos[kWave];  // x, y, z, h (non-gas candidates at infinity)
  int q[kWave];
};

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
  double alpha, beta, av_eps2;
  int32_t tc92;
};

__global__ __launch_bounds__(64, 4) void k_sph(SphArgs A) {
  __shared__ int s_stack[kSStackCap];
  __shared__ int s_leaf[kSListCap];
  __shared__ double4 s_snk[kWave];
  __shared__ SphTile s_t;
  __shared__ int s_g;
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
    const NodeTopo gnd{bt.first, bt.count, -1, 0};
    const NodeBox gb = bt.box;
    const double ghmax = gb.hmax;
    for (int c0 = 0; c0 < gnd.count; c0 += kWave) {
      const bool act = c0 + ln < gnd.count;
      const int p = gnd.first + c0 + (act ? ln : 0);
      const bool sink = act && A.gas[p];
      const double4 a = A.pm[p];
      const double4 v = A.vu[p];
      const double4 hd = A.sph[p];  // h, rho, c, P/rho^2
      const double zi = A.zo[p];
      const double hi = hd.x;
      const double mi = a.w;
      double ax = 0.0, ay = 0.0, az = 0.0, du = 0.0, mumax = 0.0;
      int npair = 0;
      int32_t *dbg = (A.dbg && sink) ? A.dbg + ((int64_t)1 * A.cap_n + A.perm[p]) * A.dbg_max : nullptr;
      int ndbg = 0;
      int sp = 1, nleaf = 0;
      bool overflow = false;
      int rounds = 0;
      const int guard = *A.nnodes + 2;
      if (ln == 0) s_stack[0] = bt.root;
      s_snk[ln] = make_double4(a.x, a.y, a.z, sink ? 2.0 * hi : 0.0);
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
          NodeBox b = A.nbox[k >= 0 ? k : 0];
          if (k >= 0 && A.nngas[k] > 0) {
            double d2 = axis_gap_box(gb.lox, gb.hix, b.lox, b.hix);
            d2 = d2 + axis_gap_box(gb.loy, gb.hiy, b.loy, b.hiy);
            d2 = d2 + axis_gap_box(gb.loz, gb.hiz, b.loz, b.hiz);
            const double R = 2.0 * fmax(ghmax, b.hmax);
            hit = d2 < R * R;
          }
          // keep the node only if some gas sink reaches it: |x_i - box| < 2 max(h_i, h_node)
          hit = balls_reach_box(s_snk, b.lox, b.loy, b.loz, b.hix, b.hiy, b.hiz, 2.0 * b.hmax, hit) && hit;
          if (hit) {
            nd = A.topo[k];
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
          const double ihi = 1.0 / hi, imi = 1.0 / mi;
          const double ihi4 = ihi * ihi * ihi * ihi * kInvPiS;
          // pairs of this lane among nt staged candidates
          auto tile_pairs = [&](int nt) {
            uint64_t mask = 0;
            for (int j = 0; j < nt; j++) {
              const double4 b = s_t.pos[j];
              const double r2x = dist2_pair(a.x, a.y, a.z, b.x, b.y, b.z);
              const double R = 2.0 * fmax(hi, b.w);
              if (sink && s_t.q[j] != p && r2x < R * R) mask |= 1ull << j;
            }
            while (mask) {
              const int j = __builtin_ctzll(mask);
              mask &= mask - 1;
              const int q = s_t.q[j];
              const SphRec b = A.srec[q];
              if (dbg) {
                if (ndbg < A.dbg_max) dbg[ndbg] = A.perm[q];
                ndbg++;
              }
              npair++;
              const double dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
              const double r2 = dist2_pair(a.x, a.y, a.z, b.x, b.y, b.z);
              if (!(r2 > 0.0)) continue;
              const double ir = rsqrt(r2);
              const double r = r2 * ir;
              const double ihj2 = b.ih * b.ih;
              const double gi = m4_grad(r * ihi, tc) * ihi4 * ir;
              const double gj = m4_grad(r * b.ih, tc) * (ihj2 * ihj2 * kInvPiS) * ir;
              const double mj = b.m;
              const double fij = 1.0 + zi * b.im;
              const double fji = 1.0 + b.zo * imi;
              const double Ai = hd.w * fij;
              const double Aj = b.pr2 * fji;
              const double vx = v.x - b.vx, vy = v.y - b.vy, vz = v.z - b.vz;
              const double vd = vx * dx + vy * dy + vz * dz;
              double sf = mj * (Ai * gi + Aj * gj);
              double e = mj * Ai * gi * vd;
              if (vd < 0.0) {
                const double hb = 0.5 * (hi + b.h);
                const double mu = hb * vd / (r2 + A.av_eps2 * hb * hb);
                const double cb = 0.5 * (hd.z + b.c);
                const double rb = 0.5 * (hd.y + b.rho);
                const double Pi = (-A.alpha * cb * mu + A.beta * mu * mu) / rb;
                const double Gb = 0.5 * (fij * gi + fji * gj);
                sf += mj * Pi * Gb;
                e += 0.5 * mj * Pi * Gb * vd;
                mumax = fmax(mumax, fabs(mu));
              }
              ax -= sf * dx;
              ay -= sf * dy;
              az -= sf * dz;
              du += e;
            }
            __syncthreads();
          };
          // candidates in leaf order, packed 64 to a tile, one per lane
          auto stage = [&](int nt, int q) {
            if (ln < nt) {
              const bool g = A.gas[q] != 0;
              const SphRec *r = A.srec + q;
              s_t.pos[ln] = g ? make_double4(r->x, r->y, r->z, r->h) : make_double4(INFINITY, INFINITY, INFINITY, 0.0);
              s_t.q[ln] = g ? q : -1;
            }
            __syncthreads();
          };
          int fill = 0, rq = 0;
          for (int c1 = 0; c1 < nleaf; c1 += kWave) {
            const int nc = min(kWave, nleaf - c1);
            const NodeTopo my = ln < nc ? A.topo[s_leaf[c1 + ln]] : NodeTopo{0, 0, -1, 0};
            for (int j = 0; j < nc; j++) {
              const int first = __builtin_amdgcn_readlane(my.first, j);
              const int count = __builtin_amdgcn_readlane(my.count, j);
              for (int off = 0; off < count;) {
                const int tk = min(count - off, kWave - fill);
                if (ln >= fill && ln < fill + tk) rq = first + off + (ln - fill);
                fill += tk;
                off += tk;
                if (fill == kWave) {
                  stage(kWave, rq);
                  tile_pairs(kWave);
                  fill = 0;
                }
              }
            }
          }
          if (fill > 0) {
            stage(fill, rq);
            tile_pairs(fill);
          }
          nleaf = 0;
        }
        __syncthreads();
        if (last) break;
      }
      if (overflow) atomicOr(A.flags, TSPH_FLAG_STACK_OVERFLOW);
      if (dbg && ndbg > A.dbg_max) atomicOr(A.flags, TSPH_FLAG_LIST_OVERFLOW);
      if (sink) {
        A.acc[0 * A.cap_n + p] += ax;
        A.acc[1 * A.cap_n + p] += ay;
        A.acc[2 * A.cap_n + p] += az;
        A.acc[4 * A.cap_n + p] = du;
        A.solve[kMaxmu * A.cap_n + p] = mumax;
        A.cnt[2 * A.cap_n + A.perm[p]] = npair;
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_zero_sph(int64_t n, int64_t cap_n, double *__restrict__ acc,
                                                  double *__restrict__ solve, int32_t *__restrict__ cnt,
                                                  const int32_t *__restrict__ perm) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    acc[4 * cap_n + p] = 0.0;
    solve[kMaxmu * cap_n + p] = 0.0;
    cnt[2 * cap_n + perm[p]] = 0;
  }
}

}  // namespace tsph

using namespace tsph;

tsph_status tsph_impl_sph(Ctx *c, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_sph, dim3(blocks_for(c->n, 256, 8192)), dim3(256), 0, st, c->n, c->cap_n, c->acc,
                     c->solve, c->cnt, c->perm);
  if (!c->p.hydro || c->n_gas == 0) {
    TSPH_HIP_CHECK(c, hipGetLastError());
    return TSPH_OK;
  }
  SphArgs A;
  A.cap_n = c->cap_n;
  A.groups = c->groups;
  A.ngroups = c->ngroups;
  A.batches = c->batches;
  A.nbatches = c->nbatches;
  A.topo = c->topo;
  A.nbox = c->nbox;
  A.nngas = c->nngas;
  A.mem = members_of(c, c->n, c->n_gas);
  A.pm = c->pm;
  A.vu = c->vu;
  A.sph = c->sph;
  A.zo = c->zo;
  A.srec = c->srec;
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
  hipLaunchKernelGGL(k_sph, dim3(persistent_blocks(c, (const void *)k_sph)), dim3(64), 0, st, A);
  TSPH_HIP_CHECK(c, hipGetLastError());
  return TSPH_OK;
}
