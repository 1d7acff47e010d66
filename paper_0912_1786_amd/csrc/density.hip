// density.hip -- self-consistent smoothing length h (gas) and softening
// length eps (all species), densities and correction factors.
//
// Merlin et al., arXiv:0912.1786: Sect. 2.1 (Eqs. rho0, etan, iter, zeta and
// the derivative terms between them), Sect. 3 (Eqs. densitySPH, hn, nsum,
// drhodr), Sect. 3.1 (gather view, enlarged search radius), Sect. 3.2
// (independent eps and h).
//
// One wavefront per walk group (a maximal tree node of at most 64 particles);
// lane i owns sink i.  The wave walks the tree once per search radius and
// keeps the candidate leaves in LDS; every Newton pass then streams those
// leaves with wave-uniform (scalar) loads while each lane evaluates its own
// sink.  The relation eta = h n^(1/3) is solved as g(h) = h^3 n(h) - eta^3 = 0,
// monotone in h, with a bracket, Newton steps and a bisection fallback; the
// candidate radius 2 h_guess (1 + kappa) is doubled when the root lies beyond
// it.
#include <stdio.h>

#include "tsph_internal.h"

namespace tsph {

// LDS lists of a density wavefront: cached candidate leaves (a batch with
// more than split_leaves of them is handed on, so the batch walk needs little
// room; the one-sink walk of k_density_sink caches more) and the walk stack
constexpr int kDensLeafCap = 512;
constexpr int kDensSinkLeafCap = 1024;
constexpr int kDensStackCap = 1024;
constexpr double kPi = 3.14159265358979323846;

struct DensArgs {
  int64_t n, n_gas, cap_n;
  const int32_t *groups;
  const int32_t *ngroups;
  const int2 *batches;
  const int32_t *nbatches;
  const NodeTopo *topo;
  const NodeBox *nbox;
  const int32_t *nngas;
  const int32_t *nlevel;
  const DevRoot *root;  // root cube of each member
  Members mem;
  const double4 *pm;
  const double4 *vu;
  const uint8_t *gas;
  const int32_t *leaf_of;
  const int32_t *perm;
  const int32_t *nnodes;
  double *hs, *es;
  double4 *sph;
  double *zo;
  double2 *soft;
  GravRec *grec;
  SphRec *srec;
  SphRec32 *srec32;  // the FP32-bulk form's single-precision SPH partner fields (else NULL)
  double *solve;
  int32_t *work;
  uint32_t *flags;
  int32_t *noconv;
  int32_t *dbg;
  int32_t dbg_max;
  int32_t *heavy;      // batches handed to k_density_sink, in hand-off order
  int32_t *heavy_key;  // their candidate-leaf counts (a list that overflowed: INT32_MAX)
  int32_t *heavy_ord;  // the same batches, largest key class first
  int32_t heavy_cap;   // 0: no hand-off
  int32_t split_leaves;  // hand off batches with more candidate leaves
  double eta_h, eta_eps, kappa, h_tol, gamma;
  int32_t maxit, soft_mode, hydro, gravity, shared;
  int32_t corr_lit;  // d phi / d eps summed without masses (the printed Eq. zeta)
  int32_t hmass;     // h from the mass density: a gas neighbour counts m_j / m_i
  int32_t hstd;      // standard scheme: h from a fixed neighbour count nstd
  int32_t nstd;
  int32_t entropy;   // vu.w holds the entropic function A = P / rho^gamma
  double L;          // periodic box side (0: open)
};

struct Sums {
  double n, sdh, rho, msdh, mdphi, divv;
};

// One walk over the leaves that some staged sink ball reaches (s_snk[s] =
// sink position and ball radius); the group box grown by the largest radius R
// is a cheap first filter.  Leaves are handed to visit(count, last) in
// batches of at least `batch` held in s_leaf (capacity batch + 64); visit
// returns false to stop the walk.  Returns false if the walk was stopped or a
// structural check failed.  whole (a walk for the single sink at the corner
// of the point box gb): a node lying entirely inside the ball of radius R is
// listed as it is, its particle range standing for all its leaves, instead
// of being opened.
template <class V>
__device__ bool walk_leaves(const DensArgs &A, int root, const NodeBox &gb, double R, bool gas_only, int *s_stack,
                            int *s_leaf, double4 *s_snk, int batch, V &&visit, bool whole = false) {
  const int ln = lane();
  int nleaf = 0, sp = 1, rounds = 0;
  const int guard = *A.nnodes + 2;
  if (A.L > 0.0) stage_ball_groups_p(s_snk, s_snk[ln], A.L);
  else stage_ball_groups(s_snk, s_snk[ln]);
  if (ln == 0) s_stack[0] = root;
  __syncthreads();
  const double R2 = R * R;
  while (sp > 0) {
    if (++rounds > guard) {
      atomicOr(A.flags, TSPH_FLAG_INTERNAL);
      return false;
    }
    const int take = walk_take(sp, kDensStackCap);
    const int k = ln < take ? s_stack[sp - take + ln] : -1;
    sp -= take;
    __syncthreads();
    bool hit = false, leaf = false;
    NodeTopo nd{0, 0, -1, 0};
    // box, gas count and topology in one round trip
    const NodeBox b = A.nbox[k >= 0 ? k : 0];
    const NodeTopo ndk = A.topo[k >= 0 ? k : 0];
    if (k >= 0 && (!gas_only || A.nngas[k] > 0)) {
      double d2 = axis_gap_box_p(gb.lox, gb.hix, b.lox, b.hix, A.L);
      d2 = d2 + axis_gap_box_p(gb.loy, gb.hiy, b.loy, b.hiy, A.L);
      d2 = d2 + axis_gap_box_p(gb.loz, gb.hiz, b.loz, b.hiz, A.L);
      hit = d2 < R2;
    }
    hit = balls_reach_box(s_snk, b.lox, b.loy, b.loz, b.hix, b.hiy, b.hiz, 0.0, hit, A.L) && hit;
    if (hit) {
      nd = ndk;
      leaf = nd.nchild == 0;
      if (whole && !leaf && !(A.L > 0.0)) {
        const double fx = fmax(fabs(gb.lox - b.lox), fabs(b.hix - gb.lox));
        const double fy = fmax(fabs(gb.loy - b.loy), fabs(b.hiy - gb.loy));
        const double fz = fmax(fabs(gb.loz - b.loz), fabs(b.hiz - gb.loz));
        leaf = fx * fx + fy * fy + fz * fz < R2;
      }
    }
    const uint64_t lm = ballot(leaf);
    if (leaf) s_leaf[nleaf + mbcnt(lm)] = k;
    nleaf += __popcll(lm);
    const int nch = (hit && !leaf) ? nd.nchild : 0;
    const int incl = wave_incl_scan(nch);
    const int tot = __shfl(incl, kWave - 1, kWave);
    if (sp + tot > kDensStackCap) {  // excluded by walk_take; kept as a guard
      atomicOr(A.flags, TSPH_FLAG_STACK_OVERFLOW);
      return false;
    }
    for (int a = 0; a < nch; a++) s_stack[sp + incl - nch + a] = nd.child + a;
    sp += tot;
    __syncthreads();
    if (nleaf >= batch) {
      if (!visit(nleaf, false)) return false;
      nleaf = 0;
      __syncthreads();
    }
  }
  bool ok = visit(nleaf, true);
  __syncthreads();
  return ok;
}

// Candidate particles staged in LDS: position and mass (a species filtered
// out is moved to infinity), predicted velocity, particle index.
struct DensTile {
  double4 pm[kWave];
  double4 vu[kWave];
  int q[kWave];
};

// Pair geometry with the nearest image in a periodic box of side L (the open
// forms, exactly, for L = 0): a component of x_i - x_j, and the squared
// distance in the order of dist2_pair.
__device__ __forceinline__ double pdx(double L, double pi, double pj) { return wrap_d(pi - pj, L); }
__device__ __forceinline__ double pd2(double L, double px, double py, double pz, const double4 &a) {
  return L > 0.0 ? dist2_disp(pdx(L, px, a.x), pdx(L, py, a.y), pdx(L, pz, a.z))
                 : dist2_pair(px, py, pz, a.x, a.y, a.z);
}

// Per-lane kernel sums over the nt staged candidates at length h.  The
// distance tests of all candidates come first (broadcast reads) and leave
// each lane a mask of its neighbours in the tile; each lane then evaluates
// only its own neighbours, in tile order, so the lanes of the wave do not
// all step through every candidate some other lane needs.  The sums are
// the same, term for term and in the same order, as a plain loop over the
// tile that skips the candidates out of range.
template <bool kFull>
__device__ __forceinline__ void tile_sums(const DensArgs &A, const DensTile &T, int nt, double px, double py,
                                          double pz, const double4 &vp, double h, bool want_div, bool want_phi,
                                          int32_t *dbg_row, int &ndbg, Sums &s) {
  const double L = A.L;
  const double ih = 1.0 / h;
  const double ih3 = ih * ih * ih / kPi;
  const double ih4 = ih3 * ih;
  const double two_h = 2.0 * h;
  const double R2 = two_h * two_h;
  uint64_t mask = tile_mask(nt, [&](int j) {
    const double4 a = T.pm[j];
    return pd2(L, px, py, pz, a) < R2;
  });
  while (mask) {
    const int j = __builtin_ctzll(mask);
    mask &= mask - 1;
    const double4 a = T.pm[j];
    const double r2 = pd2(L, px, py, pz, a);
    if (kFull && dbg_row) {
      if (ndbg < A.dbg_max) dbg_row[ndbg] = A.perm[T.q[j]];
      ndbg++;
    }
    const double ir = r2 > 0.0 ? rsq64(r2) : 0.0;
    const double r = r2 * ir;
    const double qq = r * ih;
    double w, dw;
    m4(qq, w, dw);
    const double W = w * ih3;
    const double dWdh = -(3.0 * w + qq * dw) * ih4;
    s.n += W;
    s.sdh += dWdh;
    if (kFull) {
      s.rho += a.w * W;
      s.msdh += a.w * dWdh;
      if (want_phi) s.mdphi += (A.corr_lit ? 1.0 : a.w) * soft_pe_q(qq, ih);
      if (want_div && r > 0.0) {
        const double4 v = T.vu[j];
        const double g = dw * ih4 * ir;  // dW/dr / r
        s.divv += g * ((vp.x - v.x) * pdx(L, px, a.x) + (vp.y - v.y) * pdx(L, py, a.y) + (vp.z - v.z) * pdx(L, pz, a.z));
      }
    }
  }
}

// Loads the candidate of this lane's slot (lanes below nt) into the tile.
__device__ __forceinline__ void stage_tile(const DensArgs &A, DensTile &T, int nt, int q, bool gas_only,
                                           bool want_div) {
  const int ln = lane();
  if (ln < nt) {
    double4 a = A.pm[q];
    if (gas_only && !A.gas[q]) a = make_double4(INFINITY, INFINITY, INFINITY, 0.0);
    T.pm[ln] = a;
    if (want_div) T.vu[ln] = A.vu[q];
    T.q[ln] = q;
  }
  __syncthreads();
}

// The gas among the candidates of the lanes' raw slots (slot ln holds q, nt
// valid) appended to the tile, which holds fill gas candidates: a full tile
// is evaluated and the remainder carried over.  Each lane meets its
// neighbours in candidate order, as without the compaction.  Returns the new
// fill.
template <bool kFull>
__device__ __forceinline__ int stage_gas_sums(const DensArgs &A, DensTile &T, int nt, int q, int fill, double px,
                                              double py, double pz, const double4 &vp, double h, bool want_div,
                                              bool want_phi, int32_t *dbg_row, int &ndbg, Sums &s) {
  const int ln = lane();
  const bool g = ln < nt && A.gas[q] != 0;
  const uint64_t gm = ballot(g);
  const int slot = fill + mbcnt(gm);
  const int ng = __popcll(gm);
  if (g && slot < kWave) {
    T.pm[slot] = A.pm[q];
    if (kFull && want_div) T.vu[slot] = A.vu[q];
    T.q[slot] = q;
  }
  __syncthreads();
  if (fill + ng < kWave) return fill + ng;
  tile_sums<kFull>(A, T, kWave, px, py, pz, vp, h, want_div, want_phi, dbg_row, ndbg, s);
  __syncthreads();
  if (g && slot >= kWave) {
    T.pm[slot - kWave] = A.pm[q];
    if (kFull && want_div) T.vu[slot - kWave] = A.vu[q];
    T.q[slot - kWave] = q;
  }
  __syncthreads();
  return fill + ng - kWave;
}

// Kernel sums over the particles of a batch of candidate leaves at length h
// (per lane).  The leaves are scanned in order and their particles packed 64
// to a tile, each lane loading the particle of its slot (gas solves: only
// the gas particles, compacted); every lane then evaluates the whole tile.
// kFull adds the mass density, the mass-weighted h-derivative, the velocity
// divergence (gas solve) and the mass-weighted d phi / d eps (softening).
template <bool kFull>
__device__ void leaf_sums(const DensArgs &A, int nleaf, const int *s_leaf, DensTile &T, bool gas_only, double px,
                          double py, double pz, const double4 &vp, double h, bool want_div, bool want_phi,
                          int32_t *dbg_row, int &ndbg, Sums &s) {
  const int ln = lane();
  int fill = 0, rq = 0, gfill = 0;
  // among particles that are all gas there is nothing to compact
  const bool compact = gas_only && A.n_gas < A.n;
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
          if (compact) {
            gfill = stage_gas_sums<kFull>(A, T, kWave, rq, gfill, px, py, pz, vp, h, want_div, want_phi, dbg_row,
                                          ndbg, s);
          } else {
            stage_tile(A, T, kWave, rq, gas_only, kFull && want_div);
            tile_sums<kFull>(A, T, kWave, px, py, pz, vp, h, want_div, want_phi, dbg_row, ndbg, s);
            __syncthreads();
          }
          fill = 0;
        }
      }
    }
  }
  if (compact) {
    if (fill > 0)
      gfill = stage_gas_sums<kFull>(A, T, fill, rq, gfill, px, py, pz, vp, h, want_div, want_phi, dbg_row, ndbg,
                                    s);
    if (gfill > 0) {
      tile_sums<kFull>(A, T, gfill, px, py, pz, vp, h, want_div, want_phi, dbg_row, ndbg, s);
      __syncthreads();
    }
  } else if (fill > 0) {
    stage_tile(A, T, fill, rq, gas_only, kFull && want_div);
    tile_sums<kFull>(A, T, fill, px, py, pz, vp, h, want_div, want_phi, dbg_row, ndbg, s);
    __syncthreads();
  }
}

// The candidate set of the current sink balls: cached in s_leaf when it fits,
// otherwise streamed by re-walking the tree on every pass.
struct Cands {
  int nleaf;
  bool cached;
  double R;
  bool gas_only;
};

__device__ Cands gather(const DensArgs &A, int root, const NodeBox &gb, double R, bool gas_only, int *s_stack, int *s_leaf,
                        double4 *s_snk, bool &fail, bool whole = false, int leaf_cap = kDensLeafCap) {
  Cands c{0, true, R, gas_only};
  bool full = false;
  bool ok = walk_leaves(A, root, gb, R, gas_only, s_stack, s_leaf, s_snk, leaf_cap - kWave,
                        [&](int nl, bool last) {
                          if (!last) {
                            full = true;
                            return false;
                          }
                          c.nleaf = nl;
                          return true;
                        },
                        whole);
  if (full) {
    c.cached = false;
    c.nleaf = 0;
  } else if (!ok) {
    fail = true;
  }
  return c;
}

template <bool kFull>
__device__ Sums pass(const DensArgs &A, int root, const NodeBox &gb, const Cands &c, int *s_stack, int *s_leaf,
                     DensTile &T, double4 *s_snk, double px, double py, double pz, const double4 &vp, double h,
                     bool want_div, bool want_phi, int32_t *dbg_row, int &ndbg, bool &fail) {
  Sums s{0, 0, 0, 0, 0, 0};
  ndbg = 0;
  if (c.cached) {
    leaf_sums<kFull>(A, c.nleaf, s_leaf, T, c.gas_only, px, py, pz, vp, h, want_div, want_phi, dbg_row, ndbg, s);
  } else {
    bool ok = walk_leaves(A, root, gb, c.R, c.gas_only, s_stack, s_leaf, s_snk, kWave, [&](int nl, bool) {
      leaf_sums<kFull>(A, nl, s_leaf, T, c.gas_only, px, py, pz, vp, h, want_div, want_phi, dbg_row, ndbg, s);
      return true;
    });
    if (!ok) fail = true;
  }
  return s;
}

struct SolveOut {
  double h;
  Sums s;
  bool ok;
  bool handed;  // the batch was handed to k_density_sink; nothing else is valid
};

// Newton update of a length: safeguarded step on the monotone g(h) with the
// bracket [lo, hi]; returns true when converged (step below h_tol h).
__device__ __forceinline__ bool newton_update(double &h, double &lo, double &hi, double &dx_old, double n, double sdh,
                                              double eta3, double tol) {
  const double g = h * h * h * n - eta3;
  const double gp = 3.0 * h * h * n + h * h * h * sdh;
  if (g < 0.0) lo = h;
  else hi = h;
  const double dx = g / gp;
  if (fabs(dx) < tol * h) return true;
  double hn = h - dx;
  if (!(hn > lo && hn < hi) || fabs(dx) > 0.5 * dx_old || (isinf(hi) && hn > 2.0 * h))
    hn = isinf(hi) ? 2.0 * h : 0.5 * (lo + hi);
  dx_old = fabs(hn - h);
  h = hn;
  return false;
}

// Hands batch g to k_density_sink when its candidate leaves exceed
// split_leaves or overflow the LDS cache (sinks whose kernel reaches into a
// dense neighbourhood); false when the hand-off list is full or disabled.
__device__ __forceinline__ bool hand_off(const DensArgs &A, int g, const Cands &c) {
  if (A.heavy_cap <= 0 || A.dbg) return false;
  int slot = 0;
  if (lane() == 0) slot = atomicAdd(&A.work[6], 1);
  slot = __shfl(slot, 0, kWave);
  if (slot >= A.heavy_cap) return false;
  if (lane() == 0) {
    A.heavy[slot] = g;
    A.heavy_key[slot] = c.cached ? c.nleaf : INT32_MAX;
  }
  return true;
}

// One self-consistent length per lane (inactive lanes follow along).
__device__ SolveOut solve_length(const DensArgs &A, int g, int root, const NodeBox &gb, bool sink, bool gas_only, double eta,
                                 double guess, double px, double py, double pz, double4 vp, bool want_div,
                                 bool want_phi, int *s_stack, int *s_leaf, DensTile &T, double4 *s_snk, bool cold,
                                 int32_t *dbg_row, double imi = 0.0) {
  SolveOut o;
  o.handed = false;
  const double eta3 = eta * eta * eta;
  const int64_t set_size = gas_only ? A.nngas[root] : A.topo[root].count;
  const bool solvable = sink && ((double)set_size / kPi > eta3) && (guess > 0.0);
  bool fail = false;
  // Newton from the starting value (half the volume guess on a cold start);
  // candidates cover r < 2 rc and are gathered again, with the margin kappa,
  // when some lane's iterate leaves its radius.  A step that leaves the
  // bracket [lo, hi], does not halve the previous step, or more than doubles
  // h while no upper end is known (g' vanishes when only the particle itself
  // lies within 2h) is replaced by bisection, or by doubling while no upper
  // end is known.  Converged when the Newton step is below h_tol h; the
  // result is the last evaluated length.
  double h = guess > 0.0 ? (solvable && cold ? 0.5 * guess : guess) : 1.0;
  double lo = 0.0, hi = INFINITY, dx_old = INFINITY, rc = h * (1.0 + A.kappa);
  Cands c{0, true, 0.0, gas_only};
  bool done = !sink, ok = false, gathered = false;
  int ndbg_keep = 0, ndbg_max = 0;
  Sums keep{0, 0, 0, 0, 0, 0};
  double h_keep = h;
  for (int it = 0; it < A.maxit && __any(!done); it++) {
    bool need = !gathered;
    if (!done && h > rc) {
      rc = h * (1.0 + A.kappa);
      need = true;
    }
    if (__any(need)) {
      const double R = wave_max(done ? 0.0 : 2.0 * rc);
      s_snk[lane()] = make_double4(px, py, pz, done ? 0.0 : 2.0 * rc);
      __syncthreads();
      c = gather(A, root, gb, R, gas_only, s_stack, s_leaf, s_snk, fail);
      gathered = true;
      if (fail) break;
      if ((!c.cached || c.nleaf > A.split_leaves) && hand_off(A, g, c)) {
        o.handed = true;
        return o;
      }
    }
    int ndbg = 0;
    const Sums s = pass<true>(A, root, gb, c, s_stack, s_leaf, T, s_snk, px, py, pz, vp, h, want_div, want_phi,
                              done ? nullptr : dbg_row, ndbg, fail);
    if (fail) break;
    if (!done) {
      keep = s;
      h_keep = h;
      ndbg_keep = ndbg;
      ndbg_max = max(ndbg_max, ndbg);
      if (!solvable) {
        done = true;
      } else if (newton_update(h, lo, hi, dx_old, imi > 0.0 ? s.rho * imi : s.n, imi > 0.0 ? s.msdh * imi : s.sdh,
                               eta3, A.h_tol)) {
        done = true;
        ok = true;
      }
    }
  }
  // the exported list is that of the last evaluated length; earlier passes
  // may have been longer
  if (dbg_row) {
    for (int k = ndbg_keep; k < min(ndbg_max, A.dbg_max); k++) dbg_row[k] = -1;
    if (ndbg_keep > A.dbg_max) atomicOr(A.flags, TSPH_FLAG_LIST_OVERFLOW);
  }
  o.h = h_keep;
  o.ok = ok && !fail;
  o.s = keep;
  return o;
}

// ---- standard scheme (Sect. 3): h from a fixed number nstd of gas
// neighbours, the sink included, instead of the kernel-weighted relation.
// Bisection on h over the count of gas candidates inside 2h.  The count is
// reached at the first distance shell (candidates at one distance) whose
// cumulative count is at least nstd, and 2h is put midway between that
// shell's distance and the next larger distance, so that the shell is
// taken whole.  A pass gives, per lane, the count inside 2h, the largest
// squared distance inside with the count at it, and the smallest squared
// distance outside within the gathered radius.
struct CountOut {
  double c, r2in, cin, r2out;
};

__device__ __forceinline__ void tile_count(const DensTile &T, int nt, double px, double py, double pz, double R2,
                                           CountOut &k, double L) {
  for (int j = 0; j < nt; j++) {
    const double4 a = T.pm[j];
    const double r2 = pd2(L, px, py, pz, a);  // non-gas: at infinity
    if (r2 < R2) {
      k.c += 1.0;
      if (r2 > k.r2in) {
        k.r2in = r2;
        k.cin = 1.0;
      } else if (r2 == k.r2in) {
        k.cin += 1.0;
      }
    } else if (r2 < k.r2out) {
      k.r2out = r2;
    }
  }
}

__device__ void leaf_count(const DensArgs &A, int nleaf, const int *s_leaf, DensTile &T, double px, double py,
                           double pz, double R2, CountOut &k) {
  const int ln = lane();
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
          stage_tile(A, T, kWave, rq, true, false);
          tile_count(T, kWave, px, py, pz, R2, k, A.L);
          __syncthreads();
          fill = 0;
        }
      }
    }
  }
  if (fill > 0) {
    stage_tile(A, T, fill, rq, true, false);
    tile_count(T, fill, px, py, pz, R2, k, A.L);
    __syncthreads();
  }
}

__device__ SolveOut solve_count(const DensArgs &A, int root, const NodeBox &gb, bool sink, double guess, double px,
                                double py, double pz, double4 vp, int *s_stack, int *s_leaf, DensTile &T,
                                double4 *s_snk, int32_t *dbg_row) {
  SolveOut o;
  o.handed = false;
  o.s = Sums{0, 0, 0, 0, 0, 0};
  const bool solvable = sink && A.nngas[root] > A.nstd && guess > 0.0;
  // the iteration runs on the squared radius R2 = (2h)^2 of the count: a
  // bracket [lo2, hi2] on the crossing shell's squared distance, bisection
  // while it makes progress, otherwise a step to the next shell (shells a
  // rounding apart are then still separated)
  double R2 = 4.0 * (guess > 0.0 ? guess * guess : 1.0), lo2 = 0.0, hi2 = INFINITY, h = 0.5 * sqrt(R2);
  double rc = h * (1.0 + A.kappa);
  bool done = !sink, ok = false, gathered = false, fail = false, grow = false;
  Cands c{0, true, 0.0, true};
  const double N = (double)A.nstd;
  const int maxit = A.maxit > 400 ? A.maxit : 400;
  for (int it = 0; it < maxit && __any(!done); it++) {
    bool need = !gathered || grow;
    grow = false;
    if (!done && sqrt(R2) > 2.0 * rc) {
      rc = 0.5 * sqrt(R2) * (1.0 + A.kappa);
      need = true;
    }
    if (__any(need)) {
      const double R = wave_max(done ? 0.0 : 2.0 * rc);
      s_snk[lane()] = make_double4(px, py, pz, done ? 0.0 : 2.0 * rc);
      __syncthreads();
      c = gather(A, root, gb, R, true, s_stack, s_leaf, s_snk, fail);
      gathered = true;
      if (fail) break;
    }
    CountOut k{0.0, -1.0, 0.0, INFINITY};
    if (c.cached) {
      leaf_count(A, c.nleaf, s_leaf, T, px, py, pz, R2, k);
    } else {
      const bool wok = walk_leaves(A, root, gb, c.R, true, s_stack, s_leaf, s_snk, kWave, [&](int nl, bool) {
        leaf_count(A, nl, s_leaf, T, px, py, pz, R2, k);
        return true;
      });
      if (!wok) {
        fail = true;
        break;
      }
    }
    if (done) continue;
    if (!solvable) {
      done = true;
    } else if (k.c >= N && k.c - k.cin < N) {
      // the crossing shell is the outermost one inside
      if (k.r2out < INFINITY) {
        h = 0.25 * (sqrt(k.r2in) + sqrt(k.r2out));
        done = true;
        ok = true;
      } else {
        rc *= 2.0;  // the next distance lies beyond the gathered radius
        grow = true;
      }
    } else if (k.c < N) {
      // the crossing shell lies at or beyond the nearest distance outside
      lo2 = k.r2out < INFINITY ? k.r2out : R2;
      if (isinf(hi2)) {
        R2 = 4.0 * R2;
        if (k.r2out < INFINITY && R2 <= k.r2out) R2 = nextafter(k.r2out, INFINITY);
      } else {
        const double mid = 0.5 * (lo2 + hi2);
        R2 = (mid > lo2 && mid < hi2) ? mid : nextafter(lo2, INFINITY);
      }
    } else {
      // too many: the crossing shell lies below the largest distance inside
      hi2 = k.r2in;
      const double mid = 0.5 * (lo2 + hi2);
      R2 = (mid > lo2 && mid < hi2) ? mid : hi2;
    }
  }
  // the sums at the final lengths, over candidates gathered again for every
  // sink (lanes that finished early dropped out of the last gathers); each
  // final 2h lies below a distance found inside that lane's radius 2 rc
  if (!fail) {
    const double rad = sink ? 2.0 * rc : 0.0;
    const double R = wave_max(rad);
    s_snk[lane()] = make_double4(px, py, pz, rad);
    __syncthreads();
    c = gather(A, root, gb, R, true, s_stack, s_leaf, s_snk, fail);
  }
  int ndbg = 0;
  if (!fail)
    o.s = pass<true>(A, root, gb, c, s_stack, s_leaf, T, s_snk, px, py, pz, vp, h, true, false, dbg_row, ndbg, fail);
  if (dbg_row && ndbg > A.dbg_max) atomicOr(A.flags, TSPH_FLAG_LIST_OVERFLOW);
  o.h = h;
  o.ok = ok && !fail;
  return o;
}

// ---- both lengths of a sink in one pass: the smoothing length over gas
// neighbours (gas sinks) and the softening length over all neighbours (all
// sinks) share the candidate walk and the staged tiles, each keeping the
// Newton iteration of solve_length.

// the sums each length needs: the gas one n, dn/dh, rho, mass-weighted
// dW/dh and div v; the softening one n, dn/deps, mass-weighted d phi/d eps
// and div v (kept in the same slots: rho <-> mdphi, msdh unused)
struct Sums5 {
  double n, sdh, rho, msdh, divv;
};

struct Solver {
  double h, lo, hi, dx_old, rc, h_keep;
  bool done, ok, solvable;
  Sums5 keep;
};

__device__ __forceinline__ void solver_init(Solver &v, const DensArgs &A, int root, bool sink, bool gas_only, double eta,
                                            double guess, bool cold) {
  const int64_t set_size = gas_only ? A.nngas[root] : A.topo[root].count;
  v.solvable = sink && ((double)set_size / kPi > eta * eta * eta) && (guess > 0.0);
  v.h = guess > 0.0 ? (v.solvable && cold ? 0.5 * guess : guess) : 1.0;
  v.lo = 0.0;
  v.hi = INFINITY;
  v.dx_old = INFINITY;
  v.rc = v.h * (1.0 + A.kappa);
  v.h_keep = v.h;
  v.done = !sink;
  v.ok = false;
  v.keep = Sums5{0, 0, 0, 0, 0};
}

// one evaluation's sums into the solver
// imi > 0: the mass-density relation (a neighbour counts m_j / m_i, 1/m_i = imi)
__device__ __forceinline__ void solver_update(Solver &v, const DensArgs &A, const Sums5 &s, double eta,
                                              double imi = 0.0) {
  if (v.done) return;
  v.keep = s;
  v.h_keep = v.h;
  if (!v.solvable) {
    v.done = true;
  } else if (newton_update(v.h, v.lo, v.hi, v.dx_old, imi > 0.0 ? s.rho * imi : s.n,
                           imi > 0.0 ? s.msdh * imi : s.sdh, eta * eta * eta, A.h_tol)) {
    v.done = true;
    v.ok = true;
  }
}

// Per-lane sums of both lengths over the nt staged candidates (gas flag in
// vu.w and in bit j of gas).  do_h / do_e: the solver still iterates.
__device__ __forceinline__ void tile_sums2(const DensArgs &A, const DensTile &T, int nt, uint64_t gas, double px,
                                           double py, double pz, const double4 &vp, bool do_h, double hh, bool do_e,
                                           double he, int32_t *dbg_row, int &ndbg, Sums5 &sh, Sums5 &se) {
  const double L = A.L;
  const double ihh = 1.0 / hh, ihe = 1.0 / he;
  const double ihh3 = ihh * ihh * ihh / kPi, ihe3 = ihe * ihe * ihe / kPi;
  const double ihh4 = ihh3 * ihh, ihe4 = ihe3 * ihe;
  const double R2h = do_h ? (2.0 * hh) * (2.0 * hh) : -1.0;
  const double R2e = do_e ? (2.0 * he) * (2.0 * he) : -1.0;
  // neighbour mask first, then each lane's own neighbours in tile order
  // (as in tile_sums).  A gas candidate is a neighbour within the larger of
  // the two radii, any other within the softening radius: the gas bit of
  // candidate j (bit j of gas) is the same for every lane.
  const double R2g = fmax(R2h, R2e);
  uint64_t mask = tile_mask(nt, [&](int j) {
    const double4 a = T.pm[j];
    const double r2 = pd2(L, px, py, pz, a);
    return r2 < (((gas >> j) & 1) ? R2g : R2e);
  });
  while (mask) {
    const int j = __builtin_ctzll(mask);
    mask &= mask - 1;
    const double4 a = T.pm[j];
    const double r2 = pd2(L, px, py, pz, a);
    const double4 v = T.vu[j];
    const bool in_h = r2 < R2h && v.w != 0.0;
    const bool in_e = r2 < R2e;
    const double ir = r2 > 0.0 ? rsq64(r2) : 0.0;
    const double r = r2 * ir;
    const double dot = (vp.x - v.x) * pdx(L, px, a.x) + (vp.y - v.y) * pdx(L, py, a.y) + (vp.z - v.z) * pdx(L, pz, a.z);
    if (in_h) {
      if (dbg_row) {
        if (ndbg < A.dbg_max) dbg_row[ndbg] = A.perm[T.q[j]];
        ndbg++;
      }
      const double qq = r * ihh;
      double w, dw;
      m4(qq, w, dw);
      const double W = w * ihh3;
      const double dWdh = -(3.0 * w + qq * dw) * ihh4;
      sh.n += W;
      sh.sdh += dWdh;
      sh.rho += a.w * W;
      sh.msdh += a.w * dWdh;
      if (r > 0.0) sh.divv += dw * ihh4 * ir * dot;
    }
    if (in_e) {
      const double qq = r * ihe;
      double w, dw;
      m4(qq, w, dw);
      const double W = w * ihe3;
      se.n += W;
      se.sdh += -(3.0 * w + qq * dw) * ihe4;
      se.rho += (A.corr_lit ? 1.0 : a.w) * soft_pe_q(qq, ihe);  // mass-weighted d phi / d eps
      if (r > 0.0) se.divv += dw * ihe4 * ir * dot;
    }
  }
}

// Returns the gas bits of the staged candidates (bit j: candidate j is gas).
__device__ __forceinline__ uint64_t stage_tile2(const DensArgs &A, DensTile &T, int nt, int q) {
  const int ln = lane();
  bool g = false;
  if (ln < nt) {
    T.pm[ln] = A.pm[q];
    double4 v = A.vu[q];
    g = A.gas[q] != 0;
    v.w = g ? 1.0 : 0.0;
    T.vu[ln] = v;
    T.q[ln] = q;
  }
  const uint64_t gas = ballot(g);
  __syncthreads();
  return gas;
}

__device__ void leaf_sums2(const DensArgs &A, int nleaf, const int *s_leaf, DensTile &T, double px, double py,
                           double pz, const double4 &vp, bool do_h, double hh, bool do_e, double he, int32_t *dbg_row,
                           int &ndbg, Sums5 &sh, Sums5 &se) {
  const int ln = lane();
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
          const uint64_t gas = stage_tile2(A, T, kWave, rq);
          tile_sums2(A, T, kWave, gas, px, py, pz, vp, do_h, hh, do_e, he, dbg_row, ndbg, sh, se);
          __syncthreads();
          fill = 0;
        }
      }
    }
  }
  if (fill > 0) {
    const uint64_t gas = stage_tile2(A, T, fill, rq);
    tile_sums2(A, T, fill, gas, px, py, pz, vp, do_h, hh, do_e, he, dbg_row, ndbg, sh, se);
    __syncthreads();
  }
}

struct BothOut {
  SolveOut h, e;
  bool handed;
};

__device__ BothOut solve_both(const DensArgs &A, int g, int root, const NodeBox &gb, bool act, bool is_gas, double guess_h,
                              bool cold_h, double guess_e, bool cold_e, double px, double py, double pz,
                              const double4 &vp, int *s_stack, int *s_leaf, DensTile &T, double4 *s_snk,
                              int32_t *dbg_row, double imi) {
  BothOut o;
  o.handed = false;
  Solver H, E;
  solver_init(H, A, root, is_gas, true, A.eta_h, guess_h, cold_h);
  solver_init(E, A, root, act, false, A.eta_eps, guess_e, cold_e);
  bool fail = false, gathered = false;
  Cands c{0, true, 0.0, false};
  int ndbg_keep = 0, ndbg_max = 0;
  for (int it = 0; it < A.maxit && __any(!H.done || !E.done); it++) {
    bool need = !gathered;
    if (!H.done && H.h > H.rc) {
      H.rc = H.h * (1.0 + A.kappa);
      need = true;
    }
    if (!E.done && E.h > E.rc) {
      E.rc = E.h * (1.0 + A.kappa);
      need = true;
    }
    if (__any(need)) {
      const double rad = fmax(H.done ? 0.0 : 2.0 * H.rc, E.done ? 0.0 : 2.0 * E.rc);
      const double R = wave_max(rad);
      s_snk[lane()] = make_double4(px, py, pz, rad);
      __syncthreads();
      c = gather(A, root, gb, R, false, s_stack, s_leaf, s_snk, fail);
      gathered = true;
      if (fail) break;
      if ((!c.cached || c.nleaf > A.split_leaves) && hand_off(A, g, c)) {
        o.handed = true;
        return o;
      }
    }
    Sums5 sh{0, 0, 0, 0, 0}, se{0, 0, 0, 0, 0};
    int ndbg = 0;
    int32_t *drow = H.done ? nullptr : dbg_row;
    if (c.cached) {
      leaf_sums2(A, c.nleaf, s_leaf, T, px, py, pz, vp, !H.done, H.h, !E.done, E.h, drow, ndbg, sh, se);
    } else {
      const bool ok = walk_leaves(A, root, gb, c.R, false, s_stack, s_leaf, s_snk, kWave, [&](int nl, bool) {
        leaf_sums2(A, nl, s_leaf, T, px, py, pz, vp, !H.done, H.h, !E.done, E.h, drow, ndbg, sh, se);
        return true;
      });
      if (!ok) {
        fail = true;
        break;
      }
    }
    if (!H.done) {
      ndbg_keep = ndbg;
      ndbg_max = max(ndbg_max, ndbg);
    }
    solver_update(H, A, sh, A.eta_h, imi);
    solver_update(E, A, se, A.eta_eps);
  }
  if (dbg_row) {
    for (int k = ndbg_keep; k < min(ndbg_max, A.dbg_max); k++) dbg_row[k] = -1;
    if (ndbg_keep > A.dbg_max) atomicOr(A.flags, TSPH_FLAG_LIST_OVERFLOW);
  }
  o.h.h = H.h_keep;
  o.h.s = Sums{H.keep.n, H.keep.sdh, H.keep.rho, H.keep.msdh, 0.0, H.keep.divv};
  o.h.ok = H.ok && !fail;
  o.h.handed = false;
  o.e.h = E.h_keep;
  o.e.s = Sums{E.keep.n, E.keep.sdh, 0.0, 0.0, E.keep.rho, E.keep.divv};
  o.e.ok = E.ok && !fail;
  o.e.handed = false;
  return o;
}

__device__ __forceinline__ double cold_guess(const DensArgs &A, int p, bool gas_only, double eta) {
  int k = A.leaf_of[p];
  NodeTopo nd = A.topo[k];
  double cnt = (double)nd.count;
  if (gas_only && A.nngas[k] > 0) cnt = (double)A.nngas[k];
  double s = ldexp(A.root[member_of(A.mem, p)].side, -A.nlevel[k]);
  return eta * cbrt(s * s * s / cnt);
}

// Writes the solved lengths, densities and correction factors of particle p
// (key order) and its gravity and SPH source records.
__device__ __forceinline__ void store_outputs(const DensArgs &A, int p, bool is_gas, const double4 &a,
                                              const double4 &vp, double h_gas, const Sums &sh, double eps,
                                              double neps, double ups, double xi, double divve) {
  double h = 0.0, rho = 0.0, omega = 0.0, zeta = 0.0, divv = 0.0, c = 0.0, pr2 = 0.0, fa = 1.0;
  if (is_gas) {
    h = h_gas;
    rho = sh.rho;
    // grad-h factor f_ij = fa_i + zeta_i / (m_j Omega*_i): the number-density
    // relation's Omega*, zeta (fa = 1); the mass-density relation's 1/Omega
    // (zeta = 0); none in the standard scheme
    if (A.hstd) {
      omega = 1.0;
      zeta = 0.0;
    } else if (A.hmass) {
      omega = 1.0 + (h / (3.0 * rho)) * sh.msdh;
      zeta = 0.0;
      fa = 1.0 / omega;
    } else {
      omega = 1.0 + (h / (3.0 * sh.n)) * sh.sdh;
      zeta = -(h / (3.0 * sh.n)) * sh.msdh;
    }
    divv = -sh.divv / (sh.n * omega);
    if (A.entropy) {
      // the energy variable is A: P = A rho^gamma, c^2 = gamma A rho^(gamma - 1)
      const double P = vp.w * pow(rho, A.gamma);
      c = sqrt(A.gamma * vp.w * pow(rho, A.gamma - 1.0));
      pr2 = P / (rho * rho);
    } else {
      c = sqrt(A.gamma * (A.gamma - 1.0) * vp.w);
      pr2 = (A.gamma - 1.0) * vp.w / rho;  // P / rho^2 with P = (gamma - 1) rho u
    }
  }
  A.hs[p] = h;
  A.es[p] = eps;
  // nearest images cover a kernel only while its reach stays below half the box
  if (A.L > 0.0 && (4.0 * h >= A.L || 4.0 * eps >= A.L)) atomicOr(A.flags, TSPH_FLAG_PERIOD);
  A.sph[p] = make_double4(h, rho, c, pr2);
  const double zo = is_gas ? zeta / omega : 0.0;
  A.zo[p] = zo;
  const double xiu = (A.gravity && A.soft_mode == TSPH_SOFT_ADAPTIVE) ? xi / ups : 0.0;
  A.soft[p] = make_double2(eps, xiu);
  GravRec gr;
  gr.x = a.x; gr.y = a.y; gr.z = a.z; gr.m = a.w;
  gr.eps = eps; gr.ieps = eps > 0.0 ? 1.0 / eps : 0.0; gr.xiu = xiu;
  gr.s4 = (2.0 * eps) * (2.0 * eps);
  A.grec[p] = gr;
  if (is_gas) {
    SphRec sr;
    sr.x = a.x; sr.y = a.y; sr.z = a.z; sr.m = a.w;
    sr.vx = vp.x; sr.vy = vp.y; sr.vz = vp.z; sr.im = 1.0 / a.w;
    sr.h = h; sr.ih = 1.0 / h; sr.rho = rho; sr.c = c;
    sr.pr2 = pr2; sr.zo = zo; sr.fa = fa; sr.pad1 = 0.0;
    A.srec[p] = sr;
    if (A.srec32) {
      SphRec32 s32;
      s32.vx = (float)vp.x; s32.vy = (float)vp.y; s32.vz = (float)vp.z; s32.m = (float)a.w;
      s32.ih = (float)sr.ih; s32.rho = (float)rho; s32.c = (float)c; s32.pr2 = (float)pr2;
      s32.zo = (float)zo; s32.fa = (float)fa; s32.im = (float)sr.im; s32.h = (float)h;
      A.srec32[p] = s32;
    }
  }
  double *S = A.solve;
  S[kNh * A.cap_n + p] = is_gas ? sh.n : 0.0;
  S[kOmega * A.cap_n + p] = omega;
  S[kZeta * A.cap_n + p] = zeta;
  S[kDivv * A.cap_n + p] = divv;
  S[kNeps * A.cap_n + p] = neps;
  S[kUps * A.cap_n + p] = ups;
  S[kXi * A.cap_n + p] = xi;
  S[kDivvE * A.cap_n + p] = divve;
}

// kForm 1 (fused): gas and softening lengths solved together (independent
// solves, both species); 2 (shared): one length for both, a pure-gas
// Lagrangian system with equal eta, so the kernel holds only that solve;
// 0: one or the other separately, any scheme.
// kPer: the periodic-box form; the open one takes L = 0 as a constant
template <int kForm, bool kPer>
__global__ __launch_bounds__(64, 3) void k_density(DensArgs A) {
  if constexpr (!kPer) A.L = 0.0;
  __shared__ int s_stack[kDensStackCap];
  __shared__ int s_leaf[kDensLeafCap];
  __shared__ double4 s_snk[kSnkRecs];
  __shared__ DensTile s_dt;
  __shared__ int s_g;
  const int ln = lane();
  const int ng = *A.nbatches;
  int nnoconv = 0;
  for (;;) {
    if (ln == 0) s_g = xcd_next(A.work + 8, ng);
    __syncthreads();
    const int g = s_g;
    __syncthreads();
    if (g < 0) break;
    const Batch bt = load_batch(A.batches, A.groups, A.topo, A.nbox, A.nngas, A.mem, g);
    const NodeTopo gnd{bt.first, bt.count, -1, 0};
    const NodeBox gb = bt.box;
    for (int c0 = 0; c0 < gnd.count; c0 += kWave) {
      const bool act = c0 + ln < gnd.count;
      const int p = gnd.first + c0 + (act ? ln : 0);
      const double4 a = A.pm[p];
      const double4 vp = A.vu[p];
      const bool is_gas = act && A.gas[p];
      const int ci = act ? A.perm[p] : 0;
      int32_t *dbg0 = A.dbg ? A.dbg + ((int64_t)0 * A.cap_n + ci) * A.dbg_max : nullptr;
      // ---- smoothing length over gas neighbours (gas sinks) ----
      bool handed = false;
      SolveOut oh;
      oh.h = 0.0;
      oh.ok = true;
      oh.handed = false;
      oh.s = Sums{0, 0, 0, 0, 0, 0};
      // both lengths solved in one pass when they are independent
      constexpr bool fused = kForm == 1;
      SolveOut oe_f;
      if constexpr (fused) {
        const double gh = A.hs[p], ge = A.es[p];
        const double guess_h = gh > 0.0 ? gh : (is_gas ? cold_guess(A, p, true, A.eta_h) : 0.0);
        const double guess_e = ge > 0.0 ? ge : (act ? cold_guess(A, p, false, A.eta_eps) : 0.0);
        const BothOut b = solve_both(A, g, bt.root, gb, act, is_gas, guess_h, !(gh > 0.0), guess_e, !(ge > 0.0), a.x, a.y,
                                     a.z, vp, s_stack, s_leaf, s_dt, s_snk, is_gas ? dbg0 : nullptr,
                                     A.hmass ? 1.0 / a.w : 0.0);
        handed = b.handed;
        oh = b.h;
        oe_f = b.e;
        if (!handed) {
          if (is_gas && !oh.ok) nnoconv++;
          if (act && !oe_f.ok) nnoconv++;
        }
      } else if (A.hydro) {  // (not fused)
        double g0 = A.hs[p];
        double guess = g0 > 0.0 ? g0 : (is_gas ? cold_guess(A, p, true, A.eta_h) : 0.0);
        if (kForm != 2 && A.hstd)
          oh = solve_count(A, bt.root, gb, is_gas, guess, a.x, a.y, a.z, vp, s_stack, s_leaf, s_dt, s_snk,
                           is_gas ? dbg0 : nullptr);
        else
          // (every particle is gas in the shared form: no species filter)
          oh = solve_length(A, g, bt.root, gb, is_gas, kForm != 2, A.eta_h, guess, a.x, a.y, a.z, vp, true,
                            kForm == 2 || A.shared != 0, s_stack, s_leaf, s_dt, s_snk, !(g0 > 0.0),
                            is_gas ? dbg0 : nullptr, (kForm != 2 && A.hmass) ? 1.0 / a.w : 0.0);
        handed = oh.handed;
        if (is_gas && !oh.ok && !handed) nnoconv++;
      }
      // ---- softening length over all neighbours (all sinks) ----
      double eps = 0.0, neps = 0.0, ups = 1.0, xi = 0.0, divve = 0.0;
      if constexpr (fused) {
        if (handed) break;
        eps = oe_f.h;
        neps = oe_f.s.n;
        ups = 1.0 + (oe_f.h / (3.0 * oe_f.s.n)) * oe_f.s.sdh;
        xi = (A.soft_mode == TSPH_SOFT_ADAPTIVE) ? -(oe_f.h / (3.0 * oe_f.s.n)) * oe_f.s.mdphi : 0.0;
        divve = -oe_f.s.divv / (oe_f.s.n * ups);
      } else if (A.gravity && !handed) {
        if (kForm != 2 && A.soft_mode == TSPH_SOFT_CONSTANT) {
          eps = A.es[p];
          if (act && !(eps > 0.0 && eps < INFINITY)) atomicOr(A.flags, TSPH_FLAG_NONFINITE);
        } else if (kForm == 2 || A.shared) {
          eps = oh.h;
          neps = oh.s.n;
          ups = 1.0 + (oh.h / (3.0 * oh.s.n)) * oh.s.sdh;
          xi = (A.soft_mode == TSPH_SOFT_ADAPTIVE) ? -(oh.h / (3.0 * oh.s.n)) * oh.s.mdphi : 0.0;
          divve = -oh.s.divv / (oh.s.n * ups);
        } else {
          double g0 = A.es[p];
          double guess = g0 > 0.0 ? g0 : (act ? cold_guess(A, p, false, A.eta_eps) : 0.0);
          SolveOut oe = solve_length(A, g, bt.root, gb, act, false, A.eta_eps, guess, a.x, a.y, a.z, vp, true, true,
                                     s_stack, s_leaf, s_dt, s_snk, !(g0 > 0.0), nullptr);
          handed = oe.handed;
          if (act && !oe.ok && !handed) nnoconv++;
          eps = oe.h;
          neps = oe.s.n;
          ups = 1.0 + (oe.h / (3.0 * oe.s.n)) * oe.s.sdh;
          xi = (A.soft_mode == TSPH_SOFT_ADAPTIVE) ? -(oe.h / (3.0 * oe.s.n)) * oe.s.mdphi : 0.0;
          divve = -oe.s.divv / (oe.s.n * ups);
        }
      }
      if (handed) break;
      if (act) store_outputs(A, p, is_gas, a, vp, oh.h, oh.s, eps, neps, ups, xi, divve);
    }
  }
  if (nnoconv) {
    atomicAdd(A.noconv, nnoconv);
    atomicOr(A.flags, TSPH_FLAG_NOCONV);
  }
}

// ---- one sink per wavefront: sinks of handed-off batches, whose kernel
// reaches into a dense neighbourhood.  The lanes share the candidates of the
// one sink and their partial sums are reduced across the wave in a fixed
// order; the iteration is that of solve_length.

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Contribution of a candidate (position and mass a, predicted velocity v;
// skip: filtered out) to the sums of the sink at (px, py, pz).
__device__ __forceinline__ void add_candidate(const double4 &a, const double4 &v, bool skip, double px, double py,
                                              double pz, const double4 &vp, double ih, double ih3, double ih4,
                                              double R2, bool want_div, bool want_phi, bool lit, Sums &s,
                                              double L) {
  if (skip) return;
  const double r2 = pd2(L, px, py, pz, a);
  if (!(r2 < R2)) return;
  const double ir = r2 > 0.0 ? rsq64(r2) : 0.0;
  const double r = r2 * ir;
  const double qq = r * ih;
  double w, dw;
  m4(qq, w, dw);
  const double W = w * ih3;
  const double dWdh = -(3.0 * w + qq * dw) * ih4;
  s.n += W;
  s.sdh += dWdh;
  s.rho += a.w * W;
  s.msdh += a.w * dWdh;
  if (want_phi) s.mdphi += (lit ? 1.0 : a.w) * soft_pe_q(qq, ih);
  if (want_div && r > 0.0) {
    const double g = dw * ih4 * ir;
    s.divv += g * ((vp.x - v.x) * pdx(L, px, a.x) + (vp.y - v.y) * pdx(L, py, a.y) + (vp.z - v.z) * pdx(L, pz, a.z));
  }
}

// Loads of one candidate (position and mass, predicted velocity, filter).
struct CandLoad {
  double4 a, v;
  bool skip;
};

__device__ __forceinline__ CandLoad load_candidate(const DensArgs &A, int q, bool gas_only, bool want_div) {
  CandLoad c;
  c.skip = gas_only && !A.gas[q];
  c.a = A.pm[q];
  c.v = want_div ? A.vu[q] : make_double4(0.0, 0.0, 0.0, 0.0);
  return c;
}

// Kernel sums of one sink over the particles of the leaves leaf[0, nleaf),
// packed 64 to a round, one candidate per lane (per-lane partial sums).  The
// candidates of four rounds are loaded together before any of them is
// evaluated (more loads in flight per lane); the rounds are evaluated in
// order, so the sums do not depend on the grouping.
__device__ __forceinline__ void sink_leaf_sums(const DensArgs &A, int nleaf, const int *leaf, bool gas_only,
                                               double px, double py, double pz, const double4 &vp, double h,
                                               bool want_div, bool want_phi, Sums &s) {
  const int ln = lane();
  const double ih = 1.0 / h;
  const double ih3 = ih * ih * ih / kPi;
  const double ih4 = ih3 * ih;
  const double R2 = (2.0 * h) * (2.0 * h);
  int fill = 0, rq = 0, nr = 0;
  int q0 = 0, q1 = 0, q2 = 0;  // candidates of the pending full rounds
  for (int c1 = 0; c1 < nleaf; c1 += kWave) {
    const int nc = min(kWave, nleaf - c1);
    const NodeTopo my = ln < nc ? A.topo[leaf[c1 + ln]] : NodeTopo{0, 0, -1, 0};
    for (int j = 0; j < nc; j++) {
      const int first = __builtin_amdgcn_readlane(my.first, j);
      const int count = __builtin_amdgcn_readlane(my.count, j);
      for (int off = 0; off < count;) {
        const int tk = min(count - off, kWave - fill);
        if (ln >= fill && ln < fill + tk) rq = first + off + (ln - fill);
        fill += tk;
        off += tk;
        if (fill == kWave) {
          fill = 0;
          if (nr == 0) q0 = rq;
          else if (nr == 1) q1 = rq;
          else if (nr == 2) q2 = rq;
          if (++nr == 4) {
            const CandLoad c0 = load_candidate(A, q0, gas_only, want_div);
            const CandLoad c1 = load_candidate(A, q1, gas_only, want_div);
            const CandLoad c2 = load_candidate(A, q2, gas_only, want_div);
            const CandLoad c3 = load_candidate(A, rq, gas_only, want_div);
            add_candidate(c0.a, c0.v, c0.skip, px, py, pz, vp, ih, ih3, ih4, R2, want_div, want_phi, A.corr_lit != 0, s, A.L);
            add_candidate(c1.a, c1.v, c1.skip, px, py, pz, vp, ih, ih3, ih4, R2, want_div, want_phi, A.corr_lit != 0, s, A.L);
            add_candidate(c2.a, c2.v, c2.skip, px, py, pz, vp, ih, ih3, ih4, R2, want_div, want_phi, A.corr_lit != 0, s, A.L);
            add_candidate(c3.a, c3.v, c3.skip, px, py, pz, vp, ih, ih3, ih4, R2, want_div, want_phi, A.corr_lit != 0, s, A.L);
            nr = 0;
          }
        }
      }
    }
  }
  // pending full rounds, in order, then the partial round
  if (nr > 0) {
    const CandLoad c = load_candidate(A, q0, gas_only, want_div);
    add_candidate(c.a, c.v, c.skip, px, py, pz, vp, ih, ih3, ih4, R2, want_div, want_phi, A.corr_lit != 0, s, A.L);
  }
  if (nr > 1) {
    const CandLoad c = load_candidate(A, q1, gas_only, want_div);
    add_candidate(c.a, c.v, c.skip, px, py, pz, vp, ih, ih3, ih4, R2, want_div, want_phi, A.corr_lit != 0, s, A.L);
  }
  if (nr > 2) {
    const CandLoad c = load_candidate(A, q2, gas_only, want_div);
    add_candidate(c.a, c.v, c.skip, px, py, pz, vp, ih, ih3, ih4, R2, want_div, want_phi, A.corr_lit != 0, s, A.L);
  }
  if (ln < fill) {
    const CandLoad c = load_candidate(A, rq, gas_only, want_div);
    add_candidate(c.a, c.v, c.skip, px, py, pz, vp, ih, ih3, ih4, R2, want_div, want_phi, A.corr_lit != 0, s, A.L);
  }
}

// One self-consistent length of one sink (wave-uniform).
__device__ __forceinline__ SolveOut solve_one(const DensArgs &A, int root, bool gas_only, double eta, double guess,
                                              bool cold, const double4 &a, const double4 &vp, bool want_div,
                                              bool want_phi, int *s_stack, int *s_leaf, double4 *s_snk) {
  SolveOut o;
  o.handed = false;
  const double eta3 = eta * eta * eta;
  const int64_t set_size = gas_only ? A.nngas[root] : A.topo[root].count;
  const bool solvable = ((double)set_size / kPi > eta3) && (guess > 0.0);
  const NodeBox pb{a.x, a.y, a.z, 0.0, a.x, a.y, a.z, 0.0};
  double h = guess > 0.0 ? (solvable && cold ? 0.5 * guess : guess) : 1.0;
  double lo = 0.0, hi = INFINITY, dx_old = INFINITY, rc = h * (1.0 + A.kappa);
  bool fail = false, ok = false, gathered = false;
  Cands c{0, true, 0.0, gas_only};
  Sums keep{0, 0, 0, 0, 0, 0};
  double h_keep = h;
  for (int it = 0; it < A.maxit; it++) {
    if (!gathered || h > rc) {
      if (gathered) rc = h * (1.0 + A.kappa);
      s_snk[lane()] = make_double4(a.x, a.y, a.z, lane() == 0 ? 2.0 * rc : 0.0);
      __syncthreads();
      c = gather(A, root, pb, 2.0 * rc, gas_only, s_stack, s_leaf, s_snk, fail, true, kDensSinkLeafCap);
      gathered = true;
      if (fail) break;
    }
    Sums s{0, 0, 0, 0, 0, 0};
    if (c.cached) {
      sink_leaf_sums(A, c.nleaf, s_leaf, gas_only, a.x, a.y, a.z, vp, h, want_div, want_phi, s);
    } else {
      const bool wok = walk_leaves(
          A, root, pb, c.R, gas_only, s_stack, s_leaf, s_snk, kWave,
          [&](int nl, bool) {
            sink_leaf_sums(A, nl, s_leaf, gas_only, a.x, a.y, a.z, vp, h, want_div, want_phi, s);
            return true;
          },
          true);
      if (!wok) {
        fail = true;
        break;
      }
    }
    s.n = wave_sum(s.n);
    s.sdh = wave_sum(s.sdh);
    s.rho = wave_sum(s.rho);
    s.msdh = wave_sum(s.msdh);
    s.mdphi = wave_sum(s.mdphi);
    s.divv = wave_sum(s.divv);
    keep = s;
    h_keep = h;
    if (!solvable) break;
    // the mass-density relation counts a gas neighbour m_j / m_i
    const bool mw = gas_only && A.hmass;
    if (newton_update(h, lo, hi, dx_old, mw ? s.rho / a.w : s.n, mw ? s.msdh / a.w : s.sdh, eta3, A.h_tol)) {
      ok = true;
      break;
    }
  }
  o.h = h_keep;
  o.ok = ok && !fail;
  o.s = keep;
  return o;
}

// Contribution of a candidate to both lengths' sums of the sink at
// (px, py, pz): the gas length over gas candidates within 2h (R2h < 0: that
// solve is done), the softening length over all candidates within 2 eps
// (R2e < 0: done); the terms of each are those of add_candidate, the
// softening length's mass-weighted d phi / d eps kept in the rho slot.
__device__ __forceinline__ void add_candidate2(const CandLoad &c, double px, double py, double pz, const double4 &vp,
                                               double R2h, double ih, double ih3, double ih4, double R2e, double ie,
                                               double ie3, double ie4, bool lit, Sums5 &sh, Sums5 &se, double L) {
  const double4 &a = c.a, &v = c.v;
  const double r2 = pd2(L, px, py, pz, a);
  const bool in_h = !c.skip && r2 < R2h;
  const bool in_e = r2 < R2e;
  if (!in_h && !in_e) return;
  const double ir = r2 > 0.0 ? rsq64(r2) : 0.0;
  const double r = r2 * ir;
  const double dot = (vp.x - v.x) * pdx(L, px, a.x) + (vp.y - v.y) * pdx(L, py, a.y) + (vp.z - v.z) * pdx(L, pz, a.z);
  if (in_h) {
    const double qq = r * ih;
    double w, dw;
    m4(qq, w, dw);
    const double W = w * ih3;
    const double dWdh = -(3.0 * w + qq * dw) * ih4;
    sh.n += W;
    sh.sdh += dWdh;
    sh.rho += a.w * W;
    sh.msdh += a.w * dWdh;
    if (r > 0.0) sh.divv += dw * ih4 * ir * dot;
  }
  if (in_e) {
    const double qq = r * ie;
    double w, dw;
    m4(qq, w, dw);
    se.n += w * ie3;
    se.sdh += -(3.0 * w + qq * dw) * ie4;
    se.rho += (lit ? 1.0 : a.w) * soft_pe_q(qq, ie);
    if (r > 0.0) se.divv += dw * ie4 * ir * dot;
  }
}

// Both lengths' sums of one sink over the particles of leaf[0, nleaf), 64
// candidates to a round (per-lane partial sums; the gas flag marks the
// candidates of the gas length), two rounds loaded before they are
// evaluated, in order.
__device__ __forceinline__ void sink_leaf_sums2(const DensArgs &A, int nleaf, const int *leaf, double px, double py,
                                                double pz, const double4 &vp, bool do_h, double hh, bool do_e,
                                                double he, Sums5 &sh, Sums5 &se) {
  const int ln = lane();
  const double ih = 1.0 / hh, ie = 1.0 / he;
  const double ih3 = ih * ih * ih / kPi, ie3 = ie * ie * ie / kPi;
  const double ih4 = ih3 * ih, ie4 = ie3 * ie;
  const double R2h = do_h ? (2.0 * hh) * (2.0 * hh) : -1.0;
  const double R2e = do_e ? (2.0 * he) * (2.0 * he) : -1.0;
  int fill = 0, rq = 0, q0 = 0;
  bool pending = false;
  for (int c1 = 0; c1 < nleaf; c1 += kWave) {
    const int nc = min(kWave, nleaf - c1);
    const NodeTopo my = ln < nc ? A.topo[leaf[c1 + ln]] : NodeTopo{0, 0, -1, 0};
    for (int j = 0; j < nc; j++) {
      const int first = __builtin_amdgcn_readlane(my.first, j);
      const int count = __builtin_amdgcn_readlane(my.count, j);
      for (int off = 0; off < count;) {
        const int tk = min(count - off, kWave - fill);
        if (ln >= fill && ln < fill + tk) rq = first + off + (ln - fill);
        fill += tk;
        off += tk;
        if (fill == kWave) {
          fill = 0;
          if (!pending) {
            q0 = rq;
            pending = true;
          } else {
            const CandLoad c0 = load_candidate(A, q0, true, true);
            const CandLoad c1 = load_candidate(A, rq, true, true);
            add_candidate2(c0, px, py, pz, vp, R2h, ih, ih3, ih4, R2e, ie, ie3, ie4, A.corr_lit != 0, sh, se, A.L);
            add_candidate2(c1, px, py, pz, vp, R2h, ih, ih3, ih4, R2e, ie, ie3, ie4, A.corr_lit != 0, sh, se, A.L);
            pending = false;
          }
        }
      }
    }
  }
  if (pending) {
    const CandLoad c = load_candidate(A, q0, true, true);
    add_candidate2(c, px, py, pz, vp, R2h, ih, ih3, ih4, R2e, ie, ie3, ie4, A.corr_lit != 0, sh, se, A.L);
  }
  if (ln < fill) {
    const CandLoad c = load_candidate(A, rq, true, true);
    add_candidate2(c, px, py, pz, vp, R2h, ih, ih3, ih4, R2e, ie, ie3, ie4, A.corr_lit != 0, sh, se, A.L);
  }
}

__device__ __forceinline__ Sums5 wave_sum5(const Sums5 &s) {
  return Sums5{wave_sum(s.n), wave_sum(s.sdh), wave_sum(s.rho), wave_sum(s.msdh), wave_sum(s.divv)};
}

// Both self-consistent lengths of one gas sink when they are independent
// (as solve_both for a batch): one candidate set for the larger search
// ball, each length iterating until its own Newton step is small.
__device__ __forceinline__ BothOut solve_one_both(const DensArgs &A, int root, double guess_h, bool cold_h,
                                                  double guess_e, bool cold_e, const double4 &a, const double4 &vp,
                                                  int *s_stack, int *s_leaf, double4 *s_snk) {
  BothOut o;
  o.handed = false;
  Solver H, E;
  solver_init(H, A, root, true, true, A.eta_h, guess_h, cold_h);
  solver_init(E, A, root, true, false, A.eta_eps, guess_e, cold_e);
  const NodeBox pb{a.x, a.y, a.z, 0.0, a.x, a.y, a.z, 0.0};
  bool fail = false, gathered = false;
  Cands c{0, true, 0.0, false};
  for (int it = 0; it < A.maxit && (!H.done || !E.done); it++) {
    bool need = !gathered;
    if (!H.done && H.h > H.rc) {
      H.rc = H.h * (1.0 + A.kappa);
      need = true;
    }
    if (!E.done && E.h > E.rc) {
      E.rc = E.h * (1.0 + A.kappa);
      need = true;
    }
    if (need) {
      const double R = fmax(H.done ? 0.0 : 2.0 * H.rc, E.done ? 0.0 : 2.0 * E.rc);
      s_snk[lane()] = make_double4(a.x, a.y, a.z, lane() == 0 ? R : 0.0);
      __syncthreads();
      c = gather(A, root, pb, R, false, s_stack, s_leaf, s_snk, fail, true, kDensSinkLeafCap);
      gathered = true;
      if (fail) break;
    }
    Sums5 sh{0, 0, 0, 0, 0}, se{0, 0, 0, 0, 0};
    if (c.cached) {
      sink_leaf_sums2(A, c.nleaf, s_leaf, a.x, a.y, a.z, vp, !H.done, H.h, !E.done, E.h, sh, se);
    } else {
      const bool wok = walk_leaves(
          A, root, pb, c.R, false, s_stack, s_leaf, s_snk, kWave,
          [&](int nl, bool) {
            sink_leaf_sums2(A, nl, s_leaf, a.x, a.y, a.z, vp, !H.done, H.h, !E.done, E.h, sh, se);
            return true;
          },
          true);
      if (!wok) {
        fail = true;
        break;
      }
    }
    solver_update(H, A, wave_sum5(sh), A.eta_h, A.hmass ? 1.0 / a.w : 0.0);
    solver_update(E, A, wave_sum5(se), A.eta_eps);
  }
  o.h.h = H.h_keep;
  o.h.s = Sums{H.keep.n, H.keep.sdh, H.keep.rho, H.keep.msdh, 0.0, H.keep.divv};
  o.h.ok = H.ok && !fail;
  o.h.handed = false;
  o.e.h = E.h_keep;
  o.e.s = Sums{E.keep.n, E.keep.sdh, 0.0, 0.0, E.keep.rho, E.keep.divv};
  o.e.ok = E.ok && !fail;
  o.e.handed = false;
  return o;
}

// Power-of-two class of a hand-off key.
__device__ __forceinline__ int key_class(int32_t key) { return 31 - __clz(key > 1 ? key : 1); }

// Orders the handed-off batches by the class of their candidate-leaf count,
// largest first, so that the longest one-sink solves start first instead of
// trailing the kernel.  The order within a class is arbitrary: the sinks'
// solves are independent of one another and of the order they run in.
__global__ __launch_bounds__(1024) void k_heavy_order(DensArgs A) {
  __shared__ int s_cnt[32];
  const int n = min(A.work[6], A.heavy_cap);
  const int t = threadIdx.x;
  if (t < 32) s_cnt[t] = 0;
  __syncthreads();
  for (int i = t; i < n; i += blockDim.x) atomicAdd(&s_cnt[key_class(A.heavy_key[i])], 1);
  __syncthreads();
  if (t == 0) {
    int off = 0;
    for (int b = 31; b >= 0; b--) {
      const int k = s_cnt[b];
      s_cnt[b] = off;
      off += k;
    }
  }
  __syncthreads();
  for (int i = t; i < n; i += blockDim.x) A.heavy_ord[atomicAdd(&s_cnt[key_class(A.heavy_key[i])], 1)] = A.heavy[i];
}

__global__ __launch_bounds__(64, 2) void k_density_sink(DensArgs A) {
  __shared__ int s_stack[kDensStackCap];
  __shared__ int s_leaf[kDensSinkLeafCap];
  __shared__ double4 s_snk[kSnkRecs];
  __shared__ int s_t;
  const int ln = lane();
  const int nslot = min(A.work[6], A.heavy_cap);
  int nnoconv = 0;
  for (;;) {
    if (ln == 0) s_t = atomicAdd(&A.work[7], 1);
    __syncthreads();
    const int t = s_t;
    __syncthreads();
    if (t >= nslot * kWave) break;
    const int g = A.heavy_ord[t / kWave];
    const Batch bt = load_batch(A.batches, A.groups, A.topo, A.nbox, A.nngas, A.mem, g);
    for (int j = t % kWave; j < bt.count; j += kWave) {
      const int p = bt.first + j;
      const double4 a = A.pm[p];
      const double4 vp = A.vu[p];
      const bool is_gas = A.gas[p] != 0;
      SolveOut oh;
      oh.h = 0.0;
      oh.ok = true;
      oh.s = Sums{0, 0, 0, 0, 0, 0};
      const bool fused = A.hydro && A.gravity && !A.shared && A.soft_mode != TSPH_SOFT_CONSTANT;
      SolveOut oe_f;
      bool both = false;
      if (fused && is_gas) {  // both lengths of a gas sink in one candidate scan per pass
        const double gh = A.hs[p], ge = A.es[p];
        const BothOut b = solve_one_both(A, bt.root, gh > 0.0 ? gh : cold_guess(A, p, true, A.eta_h), !(gh > 0.0),
                                         ge > 0.0 ? ge : cold_guess(A, p, false, A.eta_eps), !(ge > 0.0), a, vp,
                                         s_stack, s_leaf, s_snk);
        oh = b.h;
        oe_f = b.e;
        both = true;
        if (!oh.ok) nnoconv++;
        if (!oe_f.ok) nnoconv++;
      } else if (A.hydro && is_gas) {
        const double g0 = A.hs[p];
        const double guess = g0 > 0.0 ? g0 : cold_guess(A, p, true, A.eta_h);
        oh = solve_one(A, bt.root, true, A.eta_h, guess, !(g0 > 0.0), a, vp, true, A.shared != 0, s_stack, s_leaf,
                       s_snk);
        if (!oh.ok) nnoconv++;
      }
      double eps = 0.0, neps = 0.0, ups = 1.0, xi = 0.0, divve = 0.0;
      if (A.gravity) {
        if (A.soft_mode == TSPH_SOFT_CONSTANT) {
          eps = A.es[p];
          if (!(eps > 0.0 && eps < INFINITY)) atomicOr(A.flags, TSPH_FLAG_NONFINITE);
        } else if (A.shared) {
          eps = oh.h;
          neps = oh.s.n;
          ups = 1.0 + (oh.h / (3.0 * oh.s.n)) * oh.s.sdh;
          xi = (A.soft_mode == TSPH_SOFT_ADAPTIVE) ? -(oh.h / (3.0 * oh.s.n)) * oh.s.mdphi : 0.0;
          divve = -oh.s.divv / (oh.s.n * ups);
        } else {
          SolveOut oe;
          if (both) {
            oe = oe_f;
          } else {
            const double g0 = A.es[p];
            const double guess = g0 > 0.0 ? g0 : cold_guess(A, p, false, A.eta_eps);
            oe = solve_one(A, bt.root, false, A.eta_eps, guess, !(g0 > 0.0), a, vp, true, true, s_stack, s_leaf,
                           s_snk);
            if (!oe.ok) nnoconv++;
          }
          eps = oe.h;
          neps = oe.s.n;
          ups = 1.0 + (oe.h / (3.0 * oe.s.n)) * oe.s.sdh;
          xi = (A.soft_mode == TSPH_SOFT_ADAPTIVE) ? -(oe.h / (3.0 * oe.s.n)) * oe.s.mdphi : 0.0;
          divve = -oe.s.divv / (oe.s.n * ups);
        }
      }
      if (ln == 0) store_outputs(A, p, is_gas, a, vp, oh.h, oh.s, eps, neps, ups, xi, divve);
    }
  }
  if (ln == 0 && nnoconv) {
    atomicAdd(A.noconv, nnoconv);
    atomicOr(A.flags, TSPH_FLAG_NOCONV);
  }
}

}  // namespace tsph

using namespace tsph;

tsph_status tsph_impl_refresh(Ctx *c, hipStream_t st);

tsph_status tsph_impl_density(Ctx *c, hipStream_t st) {
  DensArgs A;
  A.n = c->n;
  A.n_gas = c->n_gas;
  A.cap_n = c->cap_n;
  A.groups = c->groups;
  A.ngroups = c->ngroups;
  A.batches = c->batches;
  A.nbatches = c->nbatches;
  A.topo = c->topo;
  A.nbox = c->nbox;
  A.nngas = c->nngas;
  A.nlevel = c->nlevel;
  A.root = c->root;
  A.mem = members_of(c, c->n, c->n_gas);
  A.pm = c->pm;
  A.vu = c->vu;
  A.gas = c->gas;
  A.leaf_of = c->leaf_of;
  A.perm = c->perm;
  A.nnodes = c->lvl + 46;
  A.hs = c->hs;
  A.es = c->es;
  A.sph = c->sph;
  A.zo = c->zo;
  A.soft = c->soft;
  A.grec = c->grec;
  A.srec = c->srec;
  A.srec32 = c->p.precision == TSPH_FP32_BULK ? c->srec32 : nullptr;
  A.solve = c->solve;
  A.work = c->work;
  A.flags = c->flags;
  A.noconv = c->noconv;
  A.dbg = c->dbg_nbr;
  A.dbg_max = c->dbg_max;
  A.eta_h = c->p.eta_h;
  A.eta_eps = c->p.eta_eps;
  A.kappa = c->p.kappa;
  A.h_tol = c->p.h_tol;
  A.gamma = c->p.gamma;
  A.maxit = c->p.h_maxit;
  A.soft_mode = c->p.soft_mode;
  A.corr_lit = c->p.grav_corr_literal;
  A.hmass = c->p.h_weight == TSPH_HW_MASS;
  A.hstd = c->p.h_scheme == TSPH_H_STANDARD;
  A.nstd = (int32_t)llround(4.0 / 3.0 * 3.14159265358979323846 * pow(2.0 * c->p.eta_h, 3.0));
  A.entropy = c->p.entropy;
  A.L = c->p.period;
  A.hydro = c->p.hydro && c->n_gas > 0;
  A.gravity = c->p.gravity;
  // one shared length when the two solves are the same equation (pure gas,
  // equal eta, the number-density relation of the Lagrangian scheme)
  A.shared = (A.hydro && A.gravity && c->n_gas == c->n && c->p.eta_h == c->p.eta_eps &&
              c->p.soft_mode != TSPH_SOFT_CONSTANT && !A.hmass && !A.hstd)
                 ? 1
                 : 0;
  A.heavy = c->heavy;
  A.heavy_key = c->heavy + c->heavy_cap;
  A.heavy_ord = c->heavy + 2 * c->heavy_cap;
  // debug lists are written by the batch's own wave
  A.heavy_cap = (c->dbg_nbr || c->p.split_leaves == 0 || A.hstd) ? 0 : (int32_t)c->heavy_cap;
  A.split_leaves = c->p.split_leaves;
  const bool fused = A.hydro && A.gravity && !A.shared && A.soft_mode != TSPH_SOFT_CONSTANT && !A.hstd;
  const bool per = A.L > 0.0;
  void (*kd)(DensArgs) = fused      ? (per ? k_density<1, true> : k_density<1, false>)
                         : A.shared ? (per ? k_density<2, true> : k_density<2, false>)
                                    : (per ? k_density<0, true> : k_density<0, false>);
  hipLaunchKernelGGL(kd, dim3(persistent_blocks(c, (const void *)kd)), dim3(64), 0, st, A);
  if (A.heavy_cap > 0) {
    hipLaunchKernelGGL(k_heavy_order, dim3(1), dim3(1024), 0, st, A);
    hipLaunchKernelGGL(k_density_sink, dim3(persistent_blocks(c, (const void *)k_density_sink)), dim3(64), 0, st,
                       A);
  }
  TSPH_HIP_CHECK(c, hipGetLastError());
  return tsph_impl_refresh(c, st);
}
