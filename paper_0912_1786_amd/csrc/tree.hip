// tree.hip -- root cube, Morton keys, stable LSD radix sort, gather into key
// order, canonical oct-tree in level order, bottom-up node moments and walk
// groups (Sect. 2.2 of Merlin et al., arXiv:0912.1786: hierarchical cubes,
// each split into eight half-size children, leaves holding up to leaf_size
// particles, monopole + quadrupole moments, Dubinski opening radius).
//
// Every kernel is deterministic: reductions are either exact (min/max,
// integer sums) or run in a fixed order, so a build is bit-reproducible.
#include <stdio.h>

#include "tsph_internal.h"

namespace tsph {

int blocks_for(int64_t n, int threads, int max_blocks) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > max_blocks) b = max_blocks;
  return (int)b;
}

// Workgroups of a persistent walk kernel: what the device holds at once,
// but no more than one per 16 particles (walk batches hold ~45 on average),
// so that small systems leave the device to work running beside them.
static int persistent_cap(const Ctx *c, int blocks) {
  const int64_t cap = c->n / 16 + 1;
  return cap < blocks ? (int)cap : blocks;
}

int persistent_blocks(Ctx *c, const void *kernel) {
  for (int i = 0; i < 16; i++)
    if (c->occ_kernel[i] == kernel) return persistent_cap(c, c->occ_blocks[i]);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kWave, 0) != hipSuccess || per_cu < 1) {
    (void)hipGetLastError();
    per_cu = 8;
  }
  const int blocks = (c->n_cu > 0 ? c->n_cu : 256) * per_cu;
  for (int i = 0; i < 16; i++)
    if (!c->occ_kernel[i]) {
      c->occ_kernel[i] = kernel;
      c->occ_blocks[i] = blocks;
      break;
    }
  return persistent_cap(c, blocks);
}

// ---------------------------------------------------------------------------
// root cube
// ---------------------------------------------------------------------------
constexpr int kBBoxBlocks = 512;     // partial boxes of a single system

// grid (blocks per member, members): block (b, m) reduces a strided share of
// member m's particles into part[m * gridDim.x + b]
__global__ __launch_bounds__(256) void k_bbox_partial(Members M, const double *__restrict__ x,
                                                      const double *__restrict__ y,
                                                      const double *__restrict__ z,
                                                      const double *__restrict__ m,
                                                      double *__restrict__ part,
                                                      uint32_t *__restrict__ flags, double L) {
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  bool bad = false;
  const int mem = blockIdx.y;
  const int64_t i0 = member_begin(M, mem), i1 = member_end(M, mem);
  for (int64_t i = i0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < i1;
       i += (int64_t)gridDim.x * blockDim.x) {
    double p[3] = {in_box(x[i], L), in_box(y[i], L), in_box(z[i], L)};
    double mi = m[i];
    bad |= !(isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]) && isfinite(mi) && mi > 0.0);
#pragma unroll
    for (int d = 0; d < 3; d++) {
      lo[d] = fmin(lo[d], p[d]);
      hi[d] = fmax(hi[d], p[d]);
    }
  }
  if (bad) atomicOr(flags, TSPH_FLAG_NONFINITE);
  __shared__ double s[6][256];
#pragma unroll
  for (int d = 0; d < 3; d++) {
    s[d][threadIdx.x] = lo[d];
    s[3 + d][threadIdx.x] = hi[d];
  }
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
#pragma unroll
      for (int d = 0; d < 3; d++) {
        s[d][threadIdx.x] = fmin(s[d][threadIdx.x], s[d][threadIdx.x + o]);
        s[3 + d][threadIdx.x] = fmax(s[3 + d][threadIdx.x], s[3 + d][threadIdx.x + o]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[((int64_t)mem * gridDim.x + blockIdx.x) * 6 + threadIdx.x] = s[threadIdx.x][0];
}

// smallest power of two not below the largest extent; origin = minimum corner
// one block (256 threads) per member: nb partial boxes each, reduced in
// parallel (min and max are exact in any order)
__global__ __launch_bounds__(256) void k_bbox_final(int nb, const double *__restrict__ part,
                                                    DevRoot *__restrict__ roots) {
  part += (int64_t)blockIdx.x * nb * 6;
  double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int b = threadIdx.x; b < nb; b += blockDim.x)
    for (int d = 0; d < 3; d++) {
      v[d] = fmin(v[d], part[b * 6 + d]);
      v[3 + d] = fmax(v[3 + d], part[b * 6 + 3 + d]);
    }
  __shared__ double s[6][256];
  for (int k = 0; k < 6; k++) s[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int d = 0; d < 3; d++) {
        s[d][threadIdx.x] = fmin(s[d][threadIdx.x], s[d][threadIdx.x + o]);
        s[3 + d][threadIdx.x] = fmax(s[3 + d][threadIdx.x], s[3 + d][threadIdx.x + o]);
      }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  DevRoot *root = roots + blockIdx.x;
  double lo[3] = {s[0][0], s[1][0], s[2][0]}, hi[3] = {s[3][0], s[4][0], s[5][0]};
  // smallest power of two not below the largest extent; origin = minimum corner
  double L = 0.0;
  for (int d = 0; d < 3; d++) {
    double ext = hi[d] - lo[d];
    if (ext > L) L = ext;
  }
  int e = 0;
  if (L > 0.0) {
    int ex;
    double f = frexp(L, &ex);
    e = (f == 0.5) ? ex - 1 : ex;
  }
  root->x0 = lo[0];
  root->y0 = lo[1];
  root->z0 = lo[2];
  root->side = ldexp(1.0, e);
  root->scale = ldexp(1.0, kMaxLevel - e);
  root->e = e;
}

// ---------------------------------------------------------------------------
// Morton keys: x bit b -> key bit 3b+2, y -> 3b+1, z -> 3b
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t dilate3(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

__device__ __forceinline__ uint64_t cell_of(double v, double v0, double scale) {
#pragma clang fp contract(off)
  double c = floor((v - v0) * scale);
  c = fmax(c, 0.0);
  c = fmin(c, 2097151.0);
  return (uint64_t)c;
}

// key of particle i relative to the root cube of its member
__global__ __launch_bounds__(256) void k_keys(Members M, const double *__restrict__ x,
                                              const double *__restrict__ y,
                                              const double *__restrict__ z,
                                              const DevRoot *__restrict__ roots,
                                              uint64_t *__restrict__ key, int32_t *__restrict__ idx, double L) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= M.n) return;
  const DevRoot *root = roots + member_of(M, i);
  double sc = root->scale;
  uint64_t cx = cell_of(in_box(x[i], L), root->x0, sc), cy = cell_of(in_box(y[i], L), root->y0, sc),
           cz = cell_of(in_box(z[i], L), root->z0, sc);
  key[i] = (dilate3(cx) << 2) | (dilate3(cy) << 1) | dilate3(cz);
  idx[i] = (int32_t)i;
}

// ---------------------------------------------------------------------------
// generic exclusive scan of int32 counts (three kernels; n may live on the
// device).  out[i] = sum_{j<i} in[j]; *total (optional) = sum.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int block_excl_scan256(int v, int *s_tmp, int &total) {
  // 256 threads = 4 waves
  int incl = wave_incl_scan(v);
  int w = threadIdx.x >> 6;
  if (lane() == 63) s_tmp[w] = incl;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    int t = s_tmp[k];
    if (k < w) off += t;
    tot += t;
  }
  __syncthreads();
  total = tot;
  return off + incl - v;
}

__global__ __launch_bounds__(256) void k_scan_reduce(const int32_t *__restrict__ in, int64_t n_host,
                                                     const int32_t *__restrict__ n_dev,
                                                     int32_t *__restrict__ part) {
  int64_t n = n_dev ? *n_dev : n_host;
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  if (base >= n) {
    if (threadIdx.x == 0) part[blockIdx.x] = 0;
    return;
  }
  int s = 0;
  for (int k = 0; k < kScanTile / 256; k++) {
    int64_t i = base + k * 256 + threadIdx.x;
    if (i < n) s += in[i];
  }
  __shared__ int tmp[4];
  int tot;
  block_excl_scan256(s, tmp, tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// exclusive scan of the input of each block, offset by the sum of the
// blocks before it (read from the block sums, no separate pass).  Block 0
// also writes the grand total to *total; in level mode the total becomes the
// next level's node count and the node capacity is enforced.
__global__ __launch_bounds__(256) void k_scan_apply(const int32_t *__restrict__ in, int64_t n_host,
                                                    const int32_t *__restrict__ n_dev,
                                                    const int32_t *__restrict__ part, int nb,
                                                    int32_t *__restrict__ out, int32_t *__restrict__ total,
                                                    int32_t *__restrict__ lvl, int level, int64_t cap_nodes,
                                                    uint32_t *__restrict__ flags) {
  int64_t n = n_dev ? *n_dev : n_host;
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  __shared__ int tmp[4];
  int pre = 0, all = 0;
  for (int b = threadIdx.x; b < nb; b += 256) {
    const int v = part[b];
    all += v;
    if (b < (int)blockIdx.x) pre += v;
  }
  int pre_tot, all_tot;
  block_excl_scan256(pre, tmp, pre_tot);
  block_excl_scan256(all, tmp, all_tot);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int carry = all_tot;
    if (total) *total = carry;
    if (lvl) {
      // lvl[0..23) level begin, lvl[23..46) level count, lvl[46] total nodes
      int begin_next = lvl[level] + lvl[23 + level];
      if ((int64_t)begin_next + carry > cap_nodes) {
        atomicOr(flags, TSPH_FLAG_NODE_CAPACITY);
        carry = 0;
      }
      lvl[level + 1] = begin_next;
      lvl[23 + level + 1] = carry;
      lvl[46] = begin_next + carry;
    }
  }
  if (base >= n) return;
  int carry = pre_tot;
  for (int k = 0; k < kScanTile / 256; k++) {
    int64_t i = base + k * 256 + threadIdx.x;
    int v = (i < n) ? in[i] : 0;
    int tot;
    int ex = block_excl_scan256(v, tmp, tot);
    if (i < n) out[i] = carry + ex;
    carry += tot;
  }
}

static void launch_scan(Ctx *c, const int32_t *in, int64_t n_host, const int32_t *n_dev,
                        int64_t n_max, int32_t *out, int32_t *total, int32_t *lvl, int level,
                        hipStream_t st) {
  int nb = (int)((n_max + kScanTile - 1) / kScanTile);
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(256), 0, st, in, n_host, n_dev, c->scan_part);
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(256), 0, st, in, n_host, n_dev, c->scan_part, nb, out, total,
                     lvl, level, c->cap_nodes, c->flags);
}

// ---------------------------------------------------------------------------
// stable LSD radix sort of (key, index), 8-bit digits, 8 passes, segmented
// by member: every block sorts one tile of kSortTile keys of one member, and
// the digit counts are laid out member by member ([member][digit][tile]), so
// that one exclusive scan over all of them gives each member's keys the
// positions of its own range.  A single system is the one-member case
// ([digit][tile]).
// ---------------------------------------------------------------------------
struct SortTile {
  int64_t lo, hi;  // keys [lo, hi) of this block
  int64_t hbase;   // first count of its member
  int ntile, t;    // the member's tiles, this block's tile among them
};

__device__ __forceinline__ SortTile sort_tile(const Members &M, const int32_t *__restrict__ mtile, int b) {
  SortTile T;
  if (M.count <= 1) {
    T.lo = (int64_t)b * kSortTile;
    T.hi = min(T.lo + kSortTile, M.n);
    T.hbase = 0;
    T.ntile = gridDim.x;
    T.t = b;
    return T;
  }
  int lo = 0, hi = M.count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (mtile[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  T.t = b - mtile[lo];
  T.ntile = mtile[lo + 1] - mtile[lo];
  T.hbase = (int64_t)mtile[lo] * kSortBins;
  T.lo = M.off[lo] + (int64_t)T.t * kSortTile;
  T.hi = min(T.lo + kSortTile, M.off[lo + 1]);
  return T;
}

__global__ __launch_bounds__(256) void k_sort_hist(Members M, const int32_t *__restrict__ mtile,
                                                   const uint64_t *__restrict__ key, int shift,
                                                   uint32_t *__restrict__ hist) {
  __shared__ uint32_t s_h[kSortBins];
  s_h[threadIdx.x] = 0;
  __syncthreads();
  const SortTile T = sort_tile(M, mtile, blockIdx.x);
  for (int k = 0; k < kSortTile / 256; k++) {
    int64_t i = T.lo + k * 256 + threadIdx.x;
    if (i < T.hi) atomicAdd(&s_h[(key[i] >> shift) & (kSortBins - 1)], 1u);
  }
  __syncthreads();
  hist[T.hbase + (int64_t)threadIdx.x * T.ntile + T.t] = s_h[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_sort_scatter(Members M, const int32_t *__restrict__ mtile,
                                                      const uint64_t *__restrict__ kin,
                                                      const int32_t *__restrict__ iin,
                                                      uint64_t *__restrict__ kout,
                                                      int32_t *__restrict__ iout, int shift,
                                                      const int32_t *__restrict__ offs,
                                                      uint32_t *__restrict__ flags) {
  __shared__ int s_base[kSortBins];
  __shared__ int s_run[kSortBins];
  __shared__ int s_w[4][kSortBins];
  int t = threadIdx.x, w = t >> 6;
  const SortTile T = sort_tile(M, mtile, blockIdx.x);
  const int64_t n = M.n;
  s_base[t] = offs[T.hbase + (int64_t)t * T.ntile + T.t];
  s_run[t] = 0;
#pragma unroll
  for (int k = 0; k < 4; k++) s_w[k][t] = 0;
  __syncthreads();
  for (int r = 0; r < kSortTile / 256; r++) {
    int64_t i = T.lo + r * 256 + t;
    bool valid = i < T.hi;
    uint64_t k = valid ? kin[i] : 0;
    int id = valid ? iin[i] : 0;
    int d = (int)((k >> shift) & (kSortBins - 1));
    // lanes of this wave holding the same digit
    uint64_t peers = ballot(valid);
#pragma unroll
    for (int b = 0; b < kSortBits; b++) {
      uint64_t mb = ballot((d >> b) & 1);
      peers &= ((d >> b) & 1) ? mb : ~mb;
    }
    int rank = mbcnt(peers);
    if (valid && rank == 0) s_w[w][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int pos = s_base[d] + s_run[d] + rank;
      for (int q = 0; q < w; q++) pos += s_w[q][d];
      if (pos >= 0 && pos < n) {
        kout[pos] = k;
        iout[pos] = id;
      } else {
        atomicOr(flags, TSPH_FLAG_INTERNAL);
      }
    }
    __syncthreads();
    s_run[t] += s_w[0][t] + s_w[1][t] + s_w[2][t] + s_w[3][t];
#pragma unroll
    for (int q = 0; q < 4; q++) s_w[q][t] = 0;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// gather the caller-order state into key order
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gather(Members M, const int32_t *__restrict__ perm,
                                                const double *__restrict__ x, const double *__restrict__ y,
                                                const double *__restrict__ z, const double *__restrict__ m,
                                                const double *__restrict__ vpx, const double *__restrict__ vpy,
                                                const double *__restrict__ vpz, const double *__restrict__ up,
                                                const double *__restrict__ h, const double *__restrict__ eps,
                                                double4 *__restrict__ pm, double4 *__restrict__ vu,
                                                double *__restrict__ hs, double *__restrict__ es,
                                                uint8_t *__restrict__ gas, double L) {
  int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= M.n) return;
  int i = perm[p];
  bool g = member_gas(M, member_of(M, i), i);
  pm[p] = make_double4(in_box(x[i], L), in_box(y[i], L), in_box(z[i], L), m[i]);
  if (vpx) vu[p] = make_double4(vpx[i], vpy[i], vpz[i], (g && up) ? up[i] : 0.0);
  hs[p] = (g && h) ? h[i] : 0.0;
  es[p] = eps ? eps[i] : 0.0;
  gas[p] = g ? 1 : 0;
}

// ---------------------------------------------------------------------------
// topology, one level at a time
// ---------------------------------------------------------------------------
// level 0: the root of each member, in member order
__global__ void k_topo_init(Members M, NodeTopo *__restrict__ topo, int32_t *__restrict__ nlevel,
                            int32_t *__restrict__ nparent, int32_t *__restrict__ lvl) {
  int t = threadIdx.x;
  if (t < 47) lvl[t] = 0;
  for (int m = t; m < M.count; m += blockDim.x) {
    const int64_t b = member_begin(M, m);
    topo[m] = NodeTopo{(int32_t)b, (int32_t)(member_end(M, m) - b), -1, 0};
    nlevel[m] = 0;
    nparent[m] = -1;
  }
  __syncthreads();
  if (t == 0) {
    lvl[0] = 0;
    lvl[23] = M.count;
    lvl[46] = M.count;
  }
}

// children of the nodes of one level: the non-empty octants, in octant order,
// found by binary search on the sorted keys.  Eight threads per node (a
// group of eight lanes of one wavefront), one per octant, search their
// boundaries side by side: a long node costs one search of its range, not
// eight in a row.
__global__ __launch_bounds__(256) void k_topo_split(int level, int leaf_size, const int32_t *__restrict__ lvl,
                                                    const NodeTopo *__restrict__ topo,
                                                    const uint64_t *__restrict__ key,
                                                    int2 *__restrict__ ctmp, int32_t *__restrict__ ctmpn) {
  const int begin = lvl[level], count = lvl[23 + level];
  const int shift = 3 * (kMaxLevel - level - 1);
  const int oct = threadIdx.x & 7;
  // whole groups of eight walk the node list together (blockDim and the
  // grid stride are multiples of eight)
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u - oct < (int64_t)count * 8;
       u += (int64_t)gridDim.x * blockDim.x) {
    const int t = (int)(u >> 3);
    const bool valid = t < count;
    const NodeTopo nd = valid ? topo[begin + t] : NodeTopo{0, 0, -1, 0};
    const bool split = valid && nd.count > leaf_size && level < kMaxLevel;
    const int lo = nd.first, end = nd.first + nd.count;
    // first position in [lo, end) whose digit exceeds oct
    int a = lo, b = end;
    if (split) {
      while (a < b) {
        const int mid = (a + b) >> 1;
        if ((int)((key[mid] >> shift) & 7ull) <= oct) a = mid + 1;
        else b = mid;
      }
    }
    // start of this octant = end of the previous one (lane - 1 of the group)
    const int prev = __shfl_up(a, 1, 8);
    const int start = oct == 0 ? lo : prev;
    const bool has = split && a > start;
    const uint64_t m = ballot(has);
    const int gshift = lane() & ~7;
    const uint32_t gm = (uint32_t)((m >> gshift) & 0xffull);
    const int idx = __popc(gm & ((1u << oct) - 1u));
    if (has) ctmp[(int64_t)t * 8 + idx] = make_int2(start, a - start);
    if (valid && oct == 0) ctmpn[t] = split ? __popc(gm) : 0;
  }
}

__global__ __launch_bounds__(256) void k_topo_emit(int level, const int32_t *__restrict__ lvl,
                                                   NodeTopo *__restrict__ topo, int32_t *__restrict__ nlevel,
                                                   int32_t *__restrict__ nparent, const int2 *__restrict__ ctmp,
                                                   const int32_t *__restrict__ ctmpn,
                                                   const int32_t *__restrict__ cscan, int64_t cap_nodes,
                                                   uint32_t *__restrict__ flags) {
  int begin = lvl[level], count = lvl[23 + level];
  int nbegin = lvl[level + 1], ncount = lvl[23 + level + 1];
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < count; t += gridDim.x * blockDim.x) {
    int k = begin + t;
    int nch = ncount > 0 ? ctmpn[t] : 0;  // capacity exhausted: the level stays leaves
    int base = nbegin + cscan[t];
    if (nch > 0 && (base < nbegin || (int64_t)base + nch > cap_nodes || cscan[t] + nch > ncount)) {
      atomicOr(flags, TSPH_FLAG_INTERNAL);
      nch = 0;
    }
    topo[k].child = nch ? base : -1;
    topo[k].nchild = nch;
    for (int j = 0; j < nch; j++) {
      int2 fc = ctmp[(int64_t)t * 8 + j];
      topo[base + j] = NodeTopo{fc.x, fc.y, -1, 0};
      nlevel[base + j] = level + 1;
      nparent[base + j] = k;
    }
  }
}

// ---------------------------------------------------------------------------
// moments, bottom-up one level at a time
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_moments(int level, double theta, const int32_t *__restrict__ lvl,
                                                 const NodeTopo *__restrict__ topo,
                                                 const double4 *__restrict__ pm,
                                                 const uint8_t *__restrict__ gas,
                                                 const uint64_t *__restrict__ key,
                                                 const DevRoot *__restrict__ roots, Members mem,
                                                 NodeFar *__restrict__ far, NodeBox *__restrict__ box,
                                                 int32_t *__restrict__ nngas, int32_t *__restrict__ leaf_of) {
  int begin = lvl[level], count = lvl[23 + level];
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < count; t += gridDim.x * blockDim.x) {
    int k = begin + t;
    NodeTopo nd = topo[k];
    double M = 0, sx = 0, sy = 0, sz = 0;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double q[6] = {0, 0, 0, 0, 0, 0};
    int ng = 0;
    if (nd.nchild == 0) {
      for (int p = nd.first; p < nd.first + nd.count; p++) {
        double4 a = pm[p];
        M += a.w;
        sx += a.w * a.x;
        sy += a.w * a.y;
        sz += a.w * a.z;
        lo[0] = fmin(lo[0], a.x); hi[0] = fmax(hi[0], a.x);
        lo[1] = fmin(lo[1], a.y); hi[1] = fmax(hi[1], a.y);
        lo[2] = fmin(lo[2], a.z); hi[2] = fmax(hi[2], a.z);
        ng += gas[p];
        leaf_of[p] = k;
      }
      double cx = sx / M, cy = sy / M, cz = sz / M;
      for (int p = nd.first; p < nd.first + nd.count; p++) {
        double4 a = pm[p];
        double dx = a.x - cx, dy = a.y - cy, dz = a.z - cz;
        double d2 = dx * dx + dy * dy + dz * dz;
        q[0] += a.w * (3.0 * dx * dx - d2);
        q[1] += a.w * (3.0 * dy * dy - d2);
        q[2] += a.w * (3.0 * dz * dz - d2);
        q[3] += a.w * 3.0 * dx * dy;
        q[4] += a.w * 3.0 * dx * dz;
        q[5] += a.w * 3.0 * dy * dz;
      }
      sx = cx; sy = cy; sz = cz;
    } else {
      for (int c = nd.child; c < nd.child + nd.nchild; c++) {
        NodeFar f = far[c];
        M += f.m;
        sx += f.m * f.cx;
        sy += f.m * f.cy;
        sz += f.m * f.cz;
        NodeBox b = box[c];
        lo[0] = fmin(lo[0], b.lox); hi[0] = fmax(hi[0], b.hix);
        lo[1] = fmin(lo[1], b.loy); hi[1] = fmax(hi[1], b.hiy);
        lo[2] = fmin(lo[2], b.loz); hi[2] = fmax(hi[2], b.hiz);
        ng += nngas[c];
      }
      double cx = sx / M, cy = sy / M, cz = sz / M;
      // parallel-axis shift of each child's quadrupole to the parent's centre of mass
      for (int c = nd.child; c < nd.child + nd.nchild; c++) {
        NodeFar f = far[c];
        double dx = f.cx - cx, dy = f.cy - cy, dz = f.cz - cz;
        double d2 = dx * dx + dy * dy + dz * dz;
        q[0] += f.qxx + f.m * (3.0 * dx * dx - d2);
        q[1] += f.qyy + f.m * (3.0 * dy * dy - d2);
        q[2] += f.qzz + f.m * (3.0 * dz * dz - d2);
        q[3] += f.qxy + f.m * 3.0 * dx * dy;
        q[4] += f.qxz + f.m * 3.0 * dx * dz;
        q[5] += f.qyz + f.m * 3.0 * dy * dz;
      }
      sx = cx; sy = cy; sz = cz;
    }
    // cube geometry from the level, the key prefix of the node and the root
    // cube of its member
    const DevRoot *root = roots + member_of(mem, nd.first);
    uint64_t pre = key[nd.first] >> (3 * (kMaxLevel - level));
    uint64_t ix = 0, iy = 0, iz = 0;
    for (int b = 0; b < level; b++) {
      uint64_t dg = (pre >> (3 * b)) & 7ull;
      ix |= ((dg >> 2) & 1ull) << b;
      iy |= ((dg >> 1) & 1ull) << b;
      iz |= (dg & 1ull) << b;
    }
    double s = ldexp(1.0, root->e - level);
    double gx = root->x0 + (double)(2 * ix + 1) * (0.5 * s);
    double gy = root->y0 + (double)(2 * iy + 1) * (0.5 * s);
    double gz = root->z0 + (double)(2 * iz + 1) * (0.5 * s);
    double ox = sx - gx, oy = sy - gy, oz = sz - gz;
    double delta = sqrt(ox * ox + oy * oy + oz * oz);
    NodeFar f;
    f.cx = sx; f.cy = sy; f.cz = sz; f.m = M;
    f.qxx = q[0]; f.qyy = q[1]; f.qzz = q[2]; f.qxy = q[3]; f.qxz = q[4]; f.qyz = q[5];
    f.rmac = theta > 0.0 ? s / theta + delta : INFINITY;
    f.pad = 0.0;
    far[k] = f;
    NodeBox b;
    b.lox = lo[0]; b.loy = lo[1]; b.loz = lo[2];
    b.hix = hi[0]; b.hiy = hi[1]; b.hiz = hi[2];
    b.epsmax = 0.0; b.hmax = 0.0;
    box[k] = b;
    nngas[k] = ng;
  }
}

// refresh of the per-node largest eps (all) and h (gas) after the solves
// Per-node maxima of eps (all) and h (gas), one level at a time from the
// deepest; with nsoft (softened cells) also the node's sums of m eps and of
// m xi/Upsilon, from its particles (leaves) or its children.
__global__ __launch_bounds__(256) void k_refresh(int level, const int32_t *__restrict__ lvl,
                                                 const NodeTopo *__restrict__ topo,
                                                 const double *__restrict__ hs, const double *__restrict__ es,
                                                 const uint8_t *__restrict__ gas, NodeBox *__restrict__ box,
                                                 const double4 *__restrict__ pm, const double2 *__restrict__ soft,
                                                 double2 *__restrict__ nsoft) {
  int begin = lvl[level], count = lvl[23 + level];
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < count; t += gridDim.x * blockDim.x) {
    int k = begin + t;
    NodeTopo nd = topo[k];
    double em = 0.0, hm = 0.0, me = 0.0, mx = 0.0;
    if (nd.nchild == 0) {
      for (int p = nd.first; p < nd.first + nd.count; p++) {
        em = fmax(em, es[p]);
        if (gas[p]) hm = fmax(hm, hs[p]);
        if (nsoft) {
          const double m = pm[p].w;
          const double2 sf = soft[p];
          me += m * sf.x;
          mx += m * sf.y;
        }
      }
    } else {
      for (int c = nd.child; c < nd.child + nd.nchild; c++) {
        em = fmax(em, box[c].epsmax);
        hm = fmax(hm, box[c].hmax);
        if (nsoft) {
          me += nsoft[c].x;
          mx += nsoft[c].y;
        }
      }
    }
    box[k].epsmax = em;
    box[k].hmax = hm;
    if (nsoft) nsoft[k] = make_double2(me, mx);
  }
}

// ---------------------------------------------------------------------------
// walk groups: maximal nodes with at most group_size particles (or leaves),
// listed in order of their first particle
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_group_mark(int64_t n, int group_size, const int32_t *__restrict__ lvl,
                                                    const NodeTopo *__restrict__ topo,
                                                    const int32_t *__restrict__ nparent,
                                                    int32_t *__restrict__ gstart, int32_t *__restrict__ gcnt) {
  int nn = lvl[46];
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nn; k += gridDim.x * blockDim.x) {
    NodeTopo nd = topo[k];
    bool fits = nd.count <= group_size || nd.nchild == 0;
    int par = nparent[k];
    bool top = par < 0 || topo[par].count > group_size;
    if (fits && top) gstart[nd.first] = k;
  }
  (void)n;
  (void)gcnt;
}

__global__ __launch_bounds__(256) void k_fill_i32(int64_t n, int32_t *__restrict__ a, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

__global__ __launch_bounds__(256) void k_group_flag(int64_t n, const int32_t *__restrict__ gstart,
                                                    int32_t *__restrict__ f) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    f[i] = gstart[i] >= 0 ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_group_compact(int64_t n, const int32_t *__restrict__ gstart,
                                                       const int32_t *__restrict__ pos,
                                                       int32_t *__restrict__ groups, int64_t cap_nodes,
                                                       uint32_t *__restrict__ flags) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (gstart[i] >= 0) {
      int q = pos[i];
      if (q >= 0 && q < cap_nodes) groups[q] = gstart[i];
      else atomicOr(flags, TSPH_FLAG_INTERNAL);
    }
}

// Walk batches: a run of consecutive groups that are consecutive children of
// one parent is packed greedily, in octant order, into batches of at most
// batch_size particles.  One thread per run start marks the batch starts.
__device__ __forceinline__ bool next_sibling(const int32_t *groups, const int32_t *nparent, int g) {
  const int u = groups[g], v = groups[g - 1];
  return u == v + 1 && nparent[u] >= 0 && nparent[u] == nparent[v];
}

// weight: per-node particle counts to pack by (NULL: all particles; the SPH
// walks pack by gas count, so that their batches hold up to batch_size gas
// sinks)
__global__ __launch_bounds__(256) void k_batch_mark(const int32_t *__restrict__ ngroups,
                                                    const int32_t *__restrict__ groups,
                                                    const int32_t *__restrict__ nparent,
                                                    const NodeTopo *__restrict__ topo, int batch_size,
                                                    int32_t *__restrict__ bstart,
                                                    const int32_t *__restrict__ weight) {
  const int ng = *ngroups;
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < ng; g += gridDim.x * blockDim.x) {
    if (g > 0 && next_sibling(groups, nparent, g)) continue;  // not a run start
    int fill = 0;
    for (int h = g; h < ng && (h == g || next_sibling(groups, nparent, h)); h++) {
      const int c = weight ? weight[groups[h]] : topo[groups[h]].count;
      const bool start = (h == g) || (fill + c > batch_size);
      bstart[h] = start ? 1 : 0;
      fill = start ? c : fill + c;
    }
  }
}

__global__ __launch_bounds__(256) void k_batch_emit(const int32_t *__restrict__ ngroups,
                                                    const int32_t *__restrict__ bstart,
                                                    const int32_t *__restrict__ bpos, int2 *__restrict__ batches,
                                                    int64_t cap, uint32_t *__restrict__ flags) {
  const int ng = *ngroups;
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < ng; g += gridDim.x * blockDim.x) {
    if (!bstart[g]) continue;
    int e = g + 1;
    while (e < ng && !bstart[e]) e++;
    const int b = bpos[g];
    if (b >= 0 && b < cap) batches[b] = make_int2(g, e);
    else atomicOr(flags, TSPH_FLAG_INTERNAL);
  }
}

}  // namespace tsph

using namespace tsph;

tsph_status tsph_impl_build_tree(Ctx *c, const tsph_state *s, hipStream_t st) {
  const int64_t n = s->n;
  const int T = 256;
  const int gb = blocks_for(n, T, 1 << 20);
  const Members M = members_of(c, n, s->n_gas);
  // root cube of each member
  const int bbm = M.count > 1 ? kMemberBlocks : kBBoxBlocks;
  const double Lp = c->p.period;  // periodic box: positions modulo the side
  hipLaunchKernelGGL(k_bbox_partial, dim3(bbm, M.count), dim3(T), 0, st, M, s->x, s->y, s->z, s->m, c->bbox_part,
                     c->flags, Lp);
  hipLaunchKernelGGL(k_bbox_final, dim3(M.count), dim3(256), 0, st, bbm, c->bbox_part, c->root);
  // keys
  hipLaunchKernelGGL(k_keys, dim3(gb), dim3(T), 0, st, M, s->x, s->y, s->z, c->root, c->key[0], c->idx[0], Lp);
  // sort: 8 passes of 8 bits, ping-pong, result back in buffer 0
  const int nb = M.count > 1 ? c->sort_tiles : (int)((n + kSortTile - 1) / kSortTile);
  for (int pass = 0; pass < 8; pass++) {
    int src = pass & 1, dst = src ^ 1, shift = pass * kSortBits;
    hipLaunchKernelGGL(k_sort_hist, dim3(nb), dim3(T), 0, st, M, c->mtile, c->key[src], shift, c->hist);
    launch_scan(c, (const int32_t *)c->hist, (int64_t)nb * kSortBins, nullptr, (int64_t)nb * kSortBins,
                (int32_t *)c->hist, nullptr, nullptr, 0, st);
    hipLaunchKernelGGL(k_sort_scatter, dim3(nb), dim3(T), 0, st, M, c->mtile, c->key[src], c->idx[src],
                       c->key[dst], c->idx[dst], shift, (const int32_t *)c->hist, c->flags);
  }
  c->perm = c->idx[0];
  // gather
  hipLaunchKernelGGL(k_gather, dim3(gb), dim3(T), 0, st, M, c->perm, s->x, s->y, s->z, s->m, s->vpx, s->vpy,
                     s->vpz, s->up, s->h, s->eps, c->pm, c->vu, c->hs, c->es, c->gas, Lp);
  // topology
  hipLaunchKernelGGL(k_topo_init, dim3(1), dim3(256), 0, st, M, c->topo, c->nlevel, c->nparent, c->lvl);
  int64_t maxlev = (c->cap_nodes + 7) / 8;
  int lb = blocks_for(maxlev, T, 4096);
  for (int L = 0; L < kMaxLevel; L++) {
    hipLaunchKernelGGL(k_topo_split, dim3(lb), dim3(T), 0, st, L, c->p.leaf_size, c->lvl, c->topo,
                       c->key[0], c->ctmp, c->ctmpn);
    launch_scan(c, c->ctmpn, 0, c->lvl + 23 + L, c->cap_nodes, c->cscan, nullptr, c->lvl, L, st);
    hipLaunchKernelGGL(k_topo_emit, dim3(lb), dim3(T), 0, st, L, c->lvl, c->topo, c->nlevel, c->nparent,
                       c->ctmp, c->ctmpn, c->cscan, c->cap_nodes, c->flags);
  }
  // moments, deepest level first
  for (int L = kMaxLevel; L >= 0; L--)
    hipLaunchKernelGGL(k_moments, dim3(lb), dim3(T), 0, st, L, c->p.theta, c->lvl, c->topo, c->pm, c->gas,
                       c->key[0], c->root, M, c->nfar, c->nbox, c->nngas, c->leaf_of);
  // groups
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, T, 8192)), dim3(T), 0, st, n, c->gflag, -1);
  hipLaunchKernelGGL(k_group_mark, dim3(blocks_for(c->cap_nodes, T, 8192)), dim3(T), 0, st, n,
                     c->p.group_size, c->lvl, c->topo, c->nparent, c->gflag, nullptr);
  int32_t *flag01 = (int32_t *)c->solve;  // scratch: the solve outputs are written later
  int32_t *pos = flag01 + c->cap_n;
  hipLaunchKernelGGL(k_group_flag, dim3(blocks_for(n, T, 8192)), dim3(T), 0, st, n, c->gflag, flag01);
  launch_scan(c, flag01, n, nullptr, n, pos, c->ngroups, nullptr, 0, st);
  hipLaunchKernelGGL(k_group_compact, dim3(blocks_for(n, T, 8192)), dim3(T), 0, st, n, c->gflag, pos,
                     c->groups, c->cap_nodes, c->flags);
  // walk batches of sibling groups
  const int gbl = blocks_for(c->cap_nodes, T, 8192);
  hipLaunchKernelGGL(k_batch_mark, dim3(gbl), dim3(T), 0, st, c->ngroups, c->groups, c->nparent, c->topo,
                     kWave, c->ctmpn, (const int32_t *)nullptr);
  launch_scan(c, c->ctmpn, 0, c->ngroups, c->cap_nodes, c->cscan, c->nbatches, nullptr, 0, st);
  hipLaunchKernelGGL(k_batch_emit, dim3(gbl), dim3(T), 0, st, c->ngroups, c->ctmpn, c->cscan, c->batches,
                     c->cap_nodes, c->flags);
  // the SPH walks' batches: up to 64 gas sinks each
  if (s->n_gas > 0) {
    hipLaunchKernelGGL(k_batch_mark, dim3(gbl), dim3(T), 0, st, c->ngroups, c->groups, c->nparent, c->topo,
                       kWave, c->ctmpn, (const int32_t *)c->nngas);
    launch_scan(c, c->ctmpn, 0, c->ngroups, c->cap_nodes, c->cscan, c->nsbatches, nullptr, 0, st);
    hipLaunchKernelGGL(k_batch_emit, dim3(gbl), dim3(T), 0, st, c->ngroups, c->ctmpn, c->cscan, c->sbatches,
                       c->cap_nodes, c->flags);
  }
  TSPH_HIP_CHECK(c, hipGetLastError());
  c->n = n;
  c->n_gas = s->n_gas;
  return TSPH_OK;
}

tsph_status tsph_impl_refresh(Ctx *c, hipStream_t st) {
  int64_t maxlev = (c->cap_nodes + 7) / 8;
  int lb = blocks_for(maxlev, 256, 4096);
  for (int L = kMaxLevel; L >= 0; L--)
    hipLaunchKernelGGL(k_refresh, dim3(lb), dim3(256), 0, st, L, c->lvl, c->topo, c->hs, c->es, c->gas,
                       c->nbox, c->pm, c->soft, c->p.soften_cells && c->p.gravity ? c->nsoft : nullptr);
  TSPH_HIP_CHECK(c, hipGetLastError());
  return TSPH_OK;
}
