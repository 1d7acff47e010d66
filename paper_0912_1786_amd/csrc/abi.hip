// abi.hip -- the C ABI of include/tsph.h: context and scratch arena,
// argument validation, the per-step pipeline and the debug exports.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "tsph_internal.h"

using namespace tsph;

tsph_status tsph_impl_refresh(Ctx *c, hipStream_t st);

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxMembers = 65535;  // members are a grid dimension of the per-member reductions

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int64_t node_capacity(int64_t cap_n, int leaf) {
  return 8 * cap_n / (leaf > 0 ? leaf : 1) + 1024;
}

// Offsets of the arena's buffers, in the order tsph_create maps them.  A
// layout with more buffers than the table holds is marked full (an internal
// error reported by both callers) instead of writing past the table.
struct Layout {
  static constexpr int kSlots = 96;
  size_t off[kSlots];
  int k = 0;
  bool full = false;
  size_t total = 0;
  size_t add(size_t bytes) {
    size_t o = total;
    if (k < kSlots) off[k++] = o;
    else full = true;
    total = align_up(total + bytes);
    return o;
  }
};

const char *param_error(const tsph_params *p) {
  if (!p) return "params is NULL";
  if (!(p->theta >= 0.0)) return "theta must be >= 0";
  if (p->leaf_size < 1 || p->leaf_size > 64) return "leaf_size must be in [1, 64]";
  if (p->group_size < 1 || p->group_size > 64) return "group_size must be in [1, 64]";
  if (!(p->eta_h > 0.0) || !(p->eta_eps > 0.0)) return "eta_h and eta_eps must be > 0";
  if (!(p->gamma > 1.0)) return "gamma must be > 1";
  if (!(p->h_tol > 0.0) || p->h_maxit < 1) return "h_tol must be > 0 and h_maxit >= 1";
  if (!(p->kappa >= 0.0)) return "kappa must be >= 0";
  if (p->soft_mode < 0 || p->soft_mode > 2) return "unknown soft_mode";
  if (p->precision != TSPH_FP64 && p->precision != TSPH_FP32_BULK) return "unknown precision";
  if (!(p->alpha >= 0.0) || !(p->beta >= 0.0) || !(p->av_eps2 > 0.0)) return "bad viscosity parameters";
  if (!(p->G > 0.0)) return "G must be > 0";
  if (!(p->eta_dt > 0.0)) return "eta_dt must be > 0";
  if (p->split_leaves < 0) return "split_leaves must be >= 0";
  if (p->max_members < 1 || p->max_members > kMaxMembers) return "max_members must be in [1, 65535]";
  if (p->grav_corr_literal != 0 && p->grav_corr_literal != 1) return "grav_corr_literal must be 0 or 1";
  if (p->soften_cells != 0 && p->soften_cells != 1) return "soften_cells must be 0 or 1";
  if (p->visc_form != TSPH_VISC_MG && p->visc_form != TSPH_VISC_SIGNAL) return "unknown visc_form";
  if (p->entropy != 0 && p->entropy != 1) return "entropy must be 0 or 1";
  if (!(p->xsph_eta >= 0.0 && p->xsph_eta <= 1.0)) return "xsph_eta must be in [0, 1]";
  if (p->h_scheme != TSPH_H_LAGRANGIAN && p->h_scheme != TSPH_H_STANDARD) return "unknown h_scheme";
  if (p->h_weight != TSPH_HW_NUMBER && p->h_weight != TSPH_HW_MASS) return "unknown h_weight";
  if (p->h_weight == TSPH_HW_MASS && p->h_scheme != TSPH_H_LAGRANGIAN)
    return "the mass-density relation is taken with the Lagrangian scheme only";
  if ((p->balsara | p->alpha_switch | p->conduction) & ~1) return "balsara, alpha_switch, conduction must be 0 or 1";
  if (!(p->alpha_min >= 0.0) || !(p->alpha_u_min >= 0.0)) return "alpha_min and alpha_u_min must be >= 0";
  if (p->conduction && p->entropy) return "conduction acts on u: not with the entropy variable";
  if (!(p->period >= 0.0) || !(p->period < INFINITY)) return "period must be finite and >= 0";
  return nullptr;
}

size_t layout_bytes(int64_t N, int64_t M, int64_t S, Layout *L) {
  L->k = 0;
  L->full = false;
  L->total = 0;
  int64_t sort_blocks = (N + kSortTile - 1) / kSortTile + 1 + S;
  int64_t scan_blocks = (std::max<int64_t>(std::max<int64_t>(N, M), sort_blocks * kSortBins) + kScanTile - 1) /
                            kScanTile + 16;
  // particles
  L->add(8 * N);        // 0 key0
  L->add(8 * N);        // 1 key1
  L->add(4 * N);        // 2 idx0
  L->add(4 * N);        // 3 idx1
  L->add(32 * N);       // 4 pm
  L->add(32 * N);       // 5 vu
  L->add(8 * N);        // 6 hs
  L->add(8 * N);        // 7 es
  L->add(N);            // 8 gas
  L->add(4 * N);        // 9 leaf_of
  L->add(32 * N);       // 10 sph
  L->add(8 * N);        // 11 zo
  L->add(16 * N);       // 12 soft
  L->add(8 * kNumSolve * N);  // 13 solve
  L->add(8 * 6 * N);    // 14 acc
  L->add(4 * 3 * N);    // 15 cnt
  L->add(4 * N);        // 16 gflag
  L->add(sizeof(GravRec) * N);  // grec
  L->add(sizeof(SphRec) * N);   // srec
  L->add(sizeof(SphRec32) * N); // srec32
  L->add(32 * N);               // srec2: alpha, alpha_u, Balsara factor, u of the gas
  L->add(16 * N);               // av: alpha, alpha_u in key order
  L->add(8 * kCarryRows * N);   // pdiv: the carry to the next drift
  // nodes
  L->add(sizeof(NodeTopo) * M);  // 17 topo
  L->add(4 * M);        // 18 nlevel
  L->add(4 * M);        // 19 nparent
  L->add(4 * M);        // 20 nngas
  L->add(sizeof(NodeFar) * M);   // 21 nfar
  L->add(sizeof(NodeBox) * M);   // 22 nbox
  L->add(16 * M);                // nsoft
  L->add(8 * 8 * M);    // 23 ctmp
  L->add(4 * M);        // 24 ctmpn
  L->add(4 * M);        // 25 cscan
  L->add(4 * M);        // 26 groups
  L->add(8 * M);        // batches
  L->add(4 * 16);       // nbatches
  L->add(8 * M);        // sbatches
  L->add(4 * 16);       // nsbatches
  const int64_t icap = split_item_cap(M);
  L->add(8 * (size_t)icap * kSplitItemRanges);  // split_rng
  L->add(sizeof(SplitItem) * (size_t)icap);     // split_item
  L->add(32 * 64 * (size_t)icap);               // split_part
  L->add(4 * M);                                // split_head
  L->add(4 * 3 * heavy_batch_cap(M));           // heavy: batches, keys, ordered batches
  // small
  L->add(8 * (S + 1));               // moff
  L->add(8 * S);                     // mgas
  L->add(4 * (S + 1));               // mtile
  L->add(sizeof(DevRoot) * S);       // 27 root
  L->add(8 * 6 * std::max<int64_t>(512, kMemberBlocks * S));  // 28 bbox_part
  L->add(4 * 64);                    // 29 lvl
  L->add(4 * 16);                    // 30 ngroups
  L->add(4 * kSortBins * sort_blocks);  // 31 hist
  L->add(4 * scan_blocks);           // 32 scan_part
  L->add(4 * kWorkCounters);         // 33 work
  L->add(4 * 16);                    // 34 flags
  L->add(4 * 16);                    // 35 noconv
  L->add(8 * 9 * std::max<int64_t>(1024, kMemberBlocks * S));  // 36 red
  L->add(8 * std::max<int64_t>(16, S));                         // 37 dt
  // individual time-steps
  L->add(N);            // bact
  L->add(N);            // bact_s
  L->add(4 * N);        // bcur
  L->add(4 * N);        // bcur_s
  L->add(4 * N);        // bm
  L->add(4 * N);        // bw
  L->add(4 * 16);       // bnext
  L->add(8 * kEwaldValues);  // ewt: Ewald table of a periodic box
  L->add(16 * (kEwaldValues / 3));  // ewt32: the same in single precision
  return L->total;
}

__global__ void k_reset(int32_t *work, int n) {
  if ((int)threadIdx.x < n) work[threadIdx.x] = 0;
}

__global__ void k_fill_dbg(int64_t n, int32_t *a) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = -1;
}

// text of the last tsph_create failure (no context exists to hold it)
char g_create_err[256] = "";

tsph_status create_fail(Ctx *c, tsph_status s, const char *what, hipError_t e) {
  snprintf(g_create_err, sizeof(g_create_err), "tsph_create: %s: %s", what,
           e == hipSuccess ? "failed" : hipGetErrorString(e));
  if (c) {
    if (c->h_flags) (void)hipHostFree(c->h_flags);
    if (c->arena) (void)hipFree(c->arena);
    free(c->h_moff);
    free(c->h_mgas);
    delete c;
  }
  return s;
}

tsph_status set_err(Ctx *c, tsph_status s, const char *msg) {
  if (c) snprintf(c->err, sizeof(c->err), "%s", msg);
  return s;
}

// a context holding several members takes only states of their total size
tsph_status check_members(Ctx *c, const tsph_state *s) {
  if (c->nmem <= 1) return TSPH_OK;
  int64_t ng = 0;
  for (int k = 0; k < c->nmem; k++) ng += c->h_mgas[k];
  if (s->n != c->h_moff[c->nmem] || s->n_gas != ng)
    return set_err(c, TSPH_EINVAL, "n and n_gas must be the members' totals (tsph_set_members)");
  return TSPH_OK;
}

tsph_status check_state(Ctx *c, const tsph_state *s, bool forces) {
  if (!s) return set_err(c, TSPH_EINVAL, "state is NULL");
  if (s->n < 1) return set_err(c, TSPH_EINVAL, "n must be >= 1");
  if (s->n > c->cap_n) return set_err(c, TSPH_ECAPACITY, "n exceeds the context capacity");
  if (s->n_gas < 0 || s->n_gas > s->n) return set_err(c, TSPH_EINVAL, "n_gas must be in [0, n]");
  if (tsph_status r = check_members(c, s)) return r;
  if (!s->x || !s->y || !s->z || !s->m) return set_err(c, TSPH_EINVAL, "x, y, z, m are required");
  if (forces) {
    if (!s->ax || !s->ay || !s->az) return set_err(c, TSPH_EINVAL, "ax, ay, az are required");
    if (!s->vpx || !s->vpy || !s->vpz) return set_err(c, TSPH_EINVAL, "vpx, vpy, vpz are required");
    if (s->n_gas > 0 && c->p.hydro && (!s->up || !s->h || !s->dudt || !s->rho))
      return set_err(c, TSPH_EINVAL, "gas needs up, h, dudt and rho");
    if (c->p.gravity && !s->eps) return set_err(c, TSPH_EINVAL, "eps is required with gravity");
    if (s->n_gas > 0 && c->p.hydro && ((c->p.alpha_switch && !s->alpha) || (c->p.conduction && !s->alpha_u)))
      return set_err(c, TSPH_EINVAL, "alpha_switch needs alpha and conduction needs alpha_u");
  }
  return TSPH_OK;
}

// fields the time-step criteria read, after a force pass with this n
tsph_status check_timestep_state(Ctx *c, const tsph_state *s) {
  if (!s || s->n < 1 || s->n_gas < 0 || s->n_gas > s->n) return set_err(c, TSPH_EINVAL, "bad state sizes");
  if (s->n > c->cap_n) return set_err(c, TSPH_ECAPACITY, "n exceeds the context capacity");
  if (tsph_status r = check_members(c, s)) return r;
  if (!s->ax || !s->ay || !s->az) return set_err(c, TSPH_EINVAL, "ax, ay, az are required");
  if (s->n_gas > 0 && (!s->h || !s->u || !s->dudt || !s->rho))
    return set_err(c, TSPH_EINVAL, "gas needs h, u, dudt and rho");
  if (c->p.alpha_switch && s->n_gas > 0 && !s->alpha) return set_err(c, TSPH_EINVAL, "alpha_switch needs alpha");
  if (c->p.gravity && !s->eps) return set_err(c, TSPH_EINVAL, "eps is required with gravity");
  if (c->pdiv_n != s->n) return set_err(c, TSPH_EINVAL, "no force pass with this n");
  return TSPH_OK;
}

}  // namespace

extern "C" {

#ifndef TSPH_SOURCE_ID
#define TSPH_SOURCE_ID "unknown"
#endif
const char *tsph_version(void) { return "tsph 0.2 (gfx950) sources " TSPH_SOURCE_ID; }

const char *tsph_source_id(void) { return TSPH_SOURCE_ID; }

void tsph_default_params(tsph_params *p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  const double nnei = 50.0;
  const double eta = 0.5 * cbrt(3.0 * nnei / (4.0 * 3.14159265358979323846));
  p->G = 1.0;
  p->theta = 0.5;
  p->quadrupole = 1;
  p->soft_mode = TSPH_SOFT_ADAPTIVE;
  p->eta_h = eta;
  p->eta_eps = eta;
  p->gamma = 5.0 / 3.0;
  p->alpha = 1.0;
  p->beta = 2.0;
  p->av_eps2 = 0.01;
  p->tc92 = 1;
  p->h_maxit = 60;
  p->h_tol = 1e-10;
  p->kappa = 0.02;
  p->leaf_size = 16;
  p->group_size = 64;
  p->precision = TSPH_FP64;
  p->gravity = 1;
  p->hydro = 1;
  p->eta_dt = 0.1;
  p->split_leaves = 256;
  p->max_members = 1;
  p->alpha_min = 0.01;
}

tsph_status tsph_bytes_required(int64_t capacity_n, const tsph_params *p, size_t *bytes) {
  if (!bytes || capacity_n < 1) return TSPH_EINVAL;
  if (param_error(p)) return TSPH_EINVAL;
  Layout L;
  *bytes = layout_bytes(capacity_n, node_capacity(capacity_n, p->leaf_size), p->max_members, &L);
  return L.full ? TSPH_EINVAL : TSPH_OK;
}

tsph_status tsph_create(void **out, int64_t capacity_n, const tsph_params *p) {
  if (!out) return TSPH_EINVAL;
  *out = nullptr;
  if (capacity_n < 1 || capacity_n > (int64_t)1 << 30) {
    snprintf(g_create_err, sizeof(g_create_err), "tsph_create: capacity_n must be in [1, 2^30]");
    return TSPH_EINVAL;
  }
  if (const char *pe = param_error(p)) {
    snprintf(g_create_err, sizeof(g_create_err), "tsph_create: %s", pe);
    return TSPH_EINVAL;
  }
  Ctx *c = new (std::nothrow) Ctx();
  if (!c) return TSPH_ENOMEM;
  memset(c, 0, sizeof(*c));
  c->p = *p;
  c->cap_n = capacity_n;
  c->cap_nodes = node_capacity(capacity_n, p->leaf_size);
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) return create_fail(c, TSPH_EHIP, "hipGetDevice", e);
  e = hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device);
  if (e != hipSuccess) return create_fail(c, TSPH_EHIP, "hipDeviceGetAttribute", e);
  Layout L;
  c->cap_mem = p->max_members;
  c->nmem = 1;
  c->h_moff = (int64_t *)calloc((size_t)c->cap_mem + 1, sizeof(int64_t));
  c->h_mgas = (int64_t *)calloc((size_t)c->cap_mem, sizeof(int64_t));
  if (!c->h_moff || !c->h_mgas) return create_fail(c, TSPH_ENOMEM, "member tables", hipSuccess);
  size_t bytes = layout_bytes(c->cap_n, c->cap_nodes, c->cap_mem, &L);
  if (L.full) return create_fail(c, TSPH_EINVAL, "internal: arena layout exceeds its offset table", hipSuccess);
  e = hipMalloc(&c->arena, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    c->arena = nullptr;
    return create_fail(c, TSPH_ENOMEM, "hipMalloc of the arena", e);
  }
  c->arena_bytes = bytes;
  char *b = (char *)c->arena;
  int k = 0;
#define AT(T) (T)(b + L.off[k++])
  c->key[0] = AT(uint64_t *);
  c->key[1] = AT(uint64_t *);
  c->idx[0] = AT(int32_t *);
  c->idx[1] = AT(int32_t *);
  c->pm = AT(double4 *);
  c->vu = AT(double4 *);
  c->hs = AT(double *);
  c->es = AT(double *);
  c->gas = AT(uint8_t *);
  c->leaf_of = AT(int32_t *);
  c->sph = AT(double4 *);
  c->zo = AT(double *);
  c->soft = AT(double2 *);
  c->solve = AT(double *);
  c->acc = AT(double *);
  c->cnt = AT(int32_t *);
  c->gflag = AT(int32_t *);
  c->grec = AT(GravRec *);
  c->srec = AT(SphRec *);
  c->srec32 = AT(SphRec32 *);
  c->srec2 = AT(double4 *);
  c->av = AT(double2 *);
  c->pdiv = AT(double *);
  c->topo = AT(NodeTopo *);
  c->nlevel = AT(int32_t *);
  c->nparent = AT(int32_t *);
  c->nngas = AT(int32_t *);
  c->nfar = AT(NodeFar *);
  c->nbox = AT(NodeBox *);
  c->nsoft = AT(double2 *);
  c->ctmp = AT(int2 *);
  c->ctmpn = AT(int32_t *);
  c->cscan = AT(int32_t *);
  c->groups = AT(int32_t *);
  c->batches = AT(int2 *);
  c->nbatches = AT(int32_t *);
  c->sbatches = AT(int2 *);
  c->nsbatches = AT(int32_t *);
  c->split_rng = AT(int2 *);
  c->split_item = AT(SplitItem *);
  c->split_part = AT(double4 *);
  c->split_head = AT(int32_t *);
  c->split_cap = split_item_cap(c->cap_nodes);
  c->heavy = AT(int32_t *);
  c->heavy_cap = heavy_batch_cap(c->cap_nodes);
  c->moff = AT(int64_t *);
  c->mgas = AT(int64_t *);
  c->mtile = AT(int32_t *);
  c->root = AT(DevRoot *);
  c->bbox_part = AT(double *);
  c->lvl = AT(int32_t *);
  c->ngroups = AT(int32_t *);
  c->hist = AT(uint32_t *);
  c->scan_part = AT(int32_t *);
  c->work = AT(int32_t *);
  c->flags = AT(uint32_t *);
  c->noconv = AT(int32_t *);
  c->red = AT(double *);
  c->dt = AT(double *);
  c->bact = AT(uint8_t *);
  c->bact_s = AT(uint8_t *);
  c->bcur = AT(int32_t *);
  c->bcur_s = AT(int32_t *);
  c->bm = AT(int32_t *);
  c->bw = AT(int32_t *);
  c->bnext = AT(int32_t *);
  c->ewt = AT(double *);
  c->ewt32 = AT(float4 *);
#undef AT
  if (k != L.k) return create_fail(c, TSPH_EINVAL, "internal: arena layout and mapping disagree", hipSuccess);
  c->perm = c->idx[0];
  e = hipHostMalloc((void **)&c->h_flags, 64, hipHostMallocDefault);
  if (e != hipSuccess) {
    c->h_flags = nullptr;
    return create_fail(c, TSPH_ENOMEM, "hipHostMalloc of the flag block", e);
  }
  c->h_noconv = (int32_t *)(c->h_flags + 4);
  if ((e = hipMemset(c->flags, 0, 64)) != hipSuccess || (e = hipMemset(c->noconv, 0, 64)) != hipSuccess ||
      (e = hipMemset(c->lvl, 0, 256)) != hipSuccess || (e = hipMemset(c->ngroups, 0, 64)) != hipSuccess ||
      (e = hipMemset(c->nsbatches, 0, 64)) != hipSuccess ||
      (e = hipMemset(c->split_item, 0xff, sizeof(SplitItem) * (size_t)c->split_cap)) != hipSuccess ||
      (e = hipMemset(c->split_head, 0xff, 4 * (size_t)c->cap_nodes)) != hipSuccess ||
      (e = hipDeviceSynchronize()) != hipSuccess)
    return create_fail(c, TSPH_EHIP, "clearing the control block", e);
  if (tsph_impl_ewald(c) != TSPH_OK) return create_fail(c, TSPH_EHIP, "the Ewald table", hipErrorUnknown);
  *out = c;
  return TSPH_OK;
}

tsph_status tsph_destroy(void *ctx) {
  Ctx *c = (Ctx *)ctx;
  if (!c) return TSPH_EINVAL;
  (void)hipDeviceSynchronize();
  if (c->dbg_nbr) (void)hipFree(c->dbg_nbr);
  if (c->tev) {
    for (int i = 0; i < 64; i++)
      for (int k = 0; k < 6; k++) (void)hipEventDestroy(c->tev[i][k]);
    free(c->tev);
  }
  if (c->h_flags) (void)hipHostFree(c->h_flags);
  if (c->arena) (void)hipFree(c->arena);
  free(c->h_moff);
  free(c->h_mgas);
  delete c;
  return TSPH_OK;
}

tsph_status tsph_set_members(void *ctx, int32_t count, const int64_t *off, const int64_t *n_gas) {
  Ctx *c = (Ctx *)ctx;
  if (!c) return TSPH_EINVAL;
  if (count < 1 || count > c->cap_mem) return set_err(c, TSPH_ECAPACITY, "count must be in [1, max_members]");
  if (!off || !n_gas) return set_err(c, TSPH_EINVAL, "off and n_gas are required");
  if (off[0] != 0) return set_err(c, TSPH_EINVAL, "off[0] must be 0");
  int64_t tiles = 0;
  std::vector<int32_t> mt((size_t)count + 1);
  for (int k = 0; k < count; k++) {
    const int64_t nk = off[k + 1] - off[k];
    if (nk < 1) return set_err(c, TSPH_EINVAL, "every member needs at least one particle");
    if (n_gas[k] < 0 || n_gas[k] > nk) return set_err(c, TSPH_EINVAL, "n_gas[k] must be in [0, off[k+1] - off[k]]");
    mt[k] = (int32_t)tiles;
    tiles += (nk + kSortTile - 1) / kSortTile;
  }
  mt[count] = (int32_t)tiles;
  if (off[count] > c->cap_n) return set_err(c, TSPH_ECAPACITY, "the members exceed the context capacity");
  if (count > c->cap_nodes / 4) return set_err(c, TSPH_ECAPACITY, "too many members for the node capacity");
  TSPH_HIP_CHECK(c, hipDeviceSynchronize());
  TSPH_HIP_CHECK(c, hipMemcpy(c->moff, off, sizeof(int64_t) * (count + 1), hipMemcpyHostToDevice));
  TSPH_HIP_CHECK(c, hipMemcpy(c->mgas, n_gas, sizeof(int64_t) * count, hipMemcpyHostToDevice));
  TSPH_HIP_CHECK(c, hipMemcpy(c->mtile, mt.data(), sizeof(int32_t) * (count + 1), hipMemcpyHostToDevice));
  memcpy(c->h_moff, off, sizeof(int64_t) * (count + 1));
  memcpy(c->h_mgas, n_gas, sizeof(int64_t) * count);
  c->nmem = count;
  c->sort_tiles = (int32_t)tiles;
  c->pdiv_n = 0;
  return TSPH_OK;
}

tsph_status tsph_set_params(void *ctx, const tsph_params *p) {
  Ctx *c = (Ctx *)ctx;
  if (!c) return TSPH_EINVAL;
  const char *e = param_error(p);
  if (e) return set_err(c, TSPH_EINVAL, e);
  if (node_capacity(c->cap_n, p->leaf_size) > c->cap_nodes)
    return set_err(c, TSPH_ECAPACITY, "a smaller leaf_size needs a new context");
  c->p = *p;
  return tsph_impl_ewald(c);  // a new periodic box side: its table
}

tsph_status tsph_build_tree(void *ctx, const tsph_state *s, void *stream) {
  Ctx *c = (Ctx *)ctx;
  if (!c) return TSPH_EINVAL;
  tsph_status r = check_state(c, s, false);
  if (r != TSPH_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  c->last_stream = st;
  return tsph_impl_build_tree(c, s, st);
}

static constexpr int kTimingRing = 64;

// fold the elapsed times of the oldest recorded slots into the totals
static tsph_status timing_drain(Ctx *c, int64_t upto) {
  while (c->t_done < upto) {
    hipEvent_t *e = c->tev[c->t_done % kTimingRing];
    TSPH_HIP_CHECK(c, hipEventSynchronize(e[5]));
    for (int k = 0; k < 5; k++) {
      float ms = 0.f;
      TSPH_HIP_CHECK(c, hipEventElapsedTime(&ms, e[k], e[k + 1]));
      c->t_ms[k] += ms;
    }
    c->t_done++;
  }
  return TSPH_OK;
}

tsph_status tsph_compute_forces(void *ctx, tsph_state *s, void *stream) {
  Ctx *c = (Ctx *)ctx;
  if (!c) return TSPH_EINVAL;
  tsph_status r = check_state(c, s, true);
  if (r != TSPH_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  c->last_stream = st;
  hipEvent_t *ev = nullptr;
  if (c->timing) {
    if (c->t_calls - c->t_done >= kTimingRing && (r = timing_drain(c, c->t_calls - kTimingRing + 1)) != TSPH_OK)
      return r;
    ev = c->tev[c->t_calls % kTimingRing];
    c->t_calls++;
  }
#define MARK(i) \
  if (ev) TSPH_HIP_CHECK(c, hipEventRecord(ev[i], st));
  MARK(0);
  c->alpha_state = s->alpha;
  c->alpha_u_state = s->alpha_u;
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(kWorkCounters), 0, st, c->work, kWorkCounters);
  if (c->dbg_nbr)
    hipLaunchKernelGGL(k_fill_dbg, dim3(1024), dim3(256), 0, st, (int64_t)3 * c->cap_n * c->dbg_max, c->dbg_nbr);
  if ((r = tsph_impl_build_tree(c, s, st)) != TSPH_OK) return r;
  if (c->blk_on && (r = tsph_impl_gather_active(c, st)) != TSPH_OK) return r;
  MARK(1);
  if ((r = tsph_impl_density(c, st)) != TSPH_OK) return r;
  MARK(2);
  if ((r = tsph_impl_gravity(c, s->pot != nullptr, st)) != TSPH_OK) return r;
  MARK(3);
  if ((r = tsph_impl_sph(c, st)) != TSPH_OK) return r;
  MARK(4);
  if ((r = tsph_impl_finish(c, s, st)) != TSPH_OK) return r;
  c->pdiv_n = s->n;
  MARK(5);
#undef MARK
  return TSPH_OK;
}

tsph_status tsph_timing(void *ctx, int32_t enable) {
  Ctx *c = (Ctx *)ctx;
  if (!c) return TSPH_EINVAL;
  TSPH_HIP_CHECK(c, hipDeviceSynchronize());
  if (c->tev) {
    for (int i = 0; i < kTimingRing; i++)
      for (int k = 0; k < 6; k++) (void)hipEventDestroy(c->tev[i][k]);
    free(c->tev);
    c->tev = nullptr;
  }
  c->timing = 0;
  c->t_calls = c->t_done = 0;
  for (int k = 0; k < 5; k++) c->t_ms[k] = 0.0;
  if (!enable) return TSPH_OK;
  c->tev = (hipEvent_t(*)[6])malloc(sizeof(hipEvent_t[6]) * kTimingRing);
  if (!c->tev) return set_err(c, TSPH_ENOMEM, "timing events");
  for (int i = 0; i < kTimingRing; i++)
    for (int k = 0; k < 6; k++) TSPH_HIP_CHECK(c, hipEventCreate(&c->tev[i][k]));
  c->timing = 1;
  return TSPH_OK;
}

tsph_status tsph_phase_times(void *ctx, double *ms_out, int64_t *calls) {
  Ctx *c = (Ctx *)ctx;
  if (!c || !ms_out) return TSPH_EINVAL;
  if (!c->timing) return set_err(c, TSPH_EINVAL, "timing is not enabled");
  tsph_status r = timing_drain(c, c->t_calls);
  if (r != TSPH_OK) return r;
  for (int k = 0; k < 5; k++) ms_out[k] = c->t_ms[k];
  if (calls) *calls = c->t_done;
  return TSPH_OK;
}

static tsph_status kick_drift_checks(Ctx *c, tsph_state *s, int32_t phase) {
  if (!s || s->n < 1 || s->n_gas < 0 || s->n_gas > s->n) return set_err(c, TSPH_EINVAL, "bad state sizes");
  if (tsph_status r = check_members(c, s)) return r;
  if (!s->x || !s->y || !s->z || !s->vx || !s->vy || !s->vz || !s->ax || !s->ay || !s->az)
    return set_err(c, TSPH_EINVAL, "x, v and a are required");
  if (s->n_gas > 0 && (!s->u || !s->dudt)) return set_err(c, TSPH_EINVAL, "gas needs u and dudt");
  if (phase != TSPH_KD_FIRST && phase != TSPH_KD_SECOND) return set_err(c, TSPH_EINVAL, "unknown phase");
  return TSPH_OK;
}

tsph_status tsph_carry_bytes(int64_t n, size_t *bytes) {
  if (!bytes || n < 1) return TSPH_EINVAL;
  *bytes = sizeof(double) * (kCarryRows * (size_t)n);
  return TSPH_OK;
}

tsph_status tsph_carry_save(void *ctx, int64_t n, void *dst_device, void *stream) {
  Ctx *c = (Ctx *)ctx;
  if (!c) return TSPH_EINVAL;
  if (c->nmem > 1) return set_err(c, TSPH_EINVAL, "the carry covers a context holding one system");
  if (!dst_device) return set_err(c, TSPH_EINVAL, "dst_device is NULL");
  if (n < 1 || n != c->pdiv_n) return set_err(c, TSPH_EINVAL, "no force pass with this n to save");
  hipStream_t st = (hipStream_t)stream;
  double *d = (double *)dst_device;
  for (int k = 0; k < kCarryRows; k++)
    TSPH_HIP_CHECK(c, hipMemcpyAsync(d + k * n, c->pdiv + k * c->cap_n, sizeof(double) * n,
                                     hipMemcpyDeviceToDevice, st));
  return TSPH_OK;
}

tsph_status tsph_carry_load(void *ctx, int64_t n, const void *src_device, void *stream) {
  Ctx *c = (Ctx *)ctx;
  if (!c) return TSPH_EINVAL;
  if (c->nmem > 1) return set_err(c, TSPH_EINVAL, "the carry covers a context holding one system");
  if (!src_device) return set_err(c, TSPH_EINVAL, "src_device is NULL");
  if (n < 1 || n > c->cap_n) return set_err(c, TSPH_ECAPACITY, "n exceeds the context capacity");
  hipStream_t st = (hipStream_t)stream;
  const double *d = (const double *)src_device;
  for (int k = 0; k < kCarryRows; k++)
    TSPH_HIP_CHECK(c, hipMemcpyAsync(c->pdiv + k * c->cap_n, d + k * n, sizeof(double) * n,
                                     hipMemcpyDeviceToDevice, st));
  c->pdiv_n = n;
  return TSPH_OK;
}

tsph_status tsph_kick_drift_dt(void *ctx, tsph_state *s, const double *dt_device, int32_t phase, void *stream) {
  Ctx *c = (Ctx *)ctx;
  if (!c) return TSPH_EINVAL;
  if (!dt_device) return set_err(c, TSPH_EINVAL, "dt_device is NULL");
  tsph_status r = kick_drift_checks(c, s, phase);
  if (r != TSPH_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  c->last_stream = st;
  return tsph_impl_kick_drift(c, s, 0.0, dt_device, phase, st);
}

tsph_status tsph_kick_drift(void *ctx, tsph_state *s, double dt, int32_t phase, void *stream) {
  Ctx *c = (Ctx *)ctx;
  if (!c) return TSPH_EINVAL;
  tsph_status r = kick_drift_checks(c, s, phase);
  if (r != TSPH_OK) return r;
  if (!(dt >= 0.0)) return set_err(c, TSPH_EINVAL, "dt must be >= 0");
  hipStream_t st = (hipStream_t)stream;
  c->last_stream = st;
  return tsph_impl_kick_drift(c, s, dt, nullptr, phase, st);
}

tsph_status tsph_batch_step(void *ctx, tsph_state *s, double *dt_device, void *stream) {
  Ctx *c = (Ctx *)ctx;
  if (!c) return TSPH_EINVAL;
  if (!dt_device) return set_err(c, TSPH_EINVAL, "dt_device is NULL");
  tsph_status r = check_state(c, s, true);
  if (r != TSPH_OK) return r;
  if ((r = kick_drift_checks(c, s, TSPH_KD_FIRST)) != TSPH_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  c->last_stream = st;
  if ((r = check_timestep_state(c, s)) != TSPH_OK) return r;
  if ((r = tsph_impl_timestep(c, s, dt_device, st)) != TSPH_OK) return r;
  if ((r = tsph_impl_kick_drift(c, s, 0.0, dt_device, TSPH_KD_FIRST, st)) != TSPH_OK) return r;
  if ((r = tsph_compute_forces(ctx, s, stream)) != TSPH_OK) return r;
  return tsph_impl_kick_drift(c, s, 0.0, dt_device, TSPH_KD_SECOND, st);
}

tsph_status tsph_timestep(void *ctx, const tsph_state *s, double *dt_device, void *stream) {
  Ctx *c = (Ctx *)ctx;
  if (!c || !dt_device) return TSPH_EINVAL;
  tsph_status r = check_timestep_state(c, s);
  if (r != TSPH_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  c->last_stream = st;
  return tsph_impl_timestep(c, s, dt_device, st);
}

tsph_status tsph_diagnostics(void *ctx, const tsph_state *s, double *out_device, void *stream) {
  Ctx *c = (Ctx *)ctx;
  if (!c || !out_device) return TSPH_EINVAL;
  if (!s || s->n < 1 || !s->x || !s->y || !s->z || !s->vx || !s->vy || !s->vz || !s->m)
    return set_err(c, TSPH_EINVAL, "diagnostics need x, v, m");
  if (tsph_status r = check_members(c, s)) return r;
  hipStream_t st = (hipStream_t)stream;
  c->last_stream = st;
  return tsph_impl_diagnostics(c, s, out_device, st);
}

tsph_status tsph_read_flags(void *ctx, uint32_t *flags, int64_t *n_noconv) {
  Ctx *c = (Ctx *)ctx;
  if (!c) return TSPH_EINVAL;
  // ordered on the context's last stream only: other streams keep running
  hipStream_t st = c->last_stream;
  TSPH_HIP_CHECK(c, hipMemcpyAsync(c->h_flags, c->flags, 4, hipMemcpyDeviceToHost, st));
  TSPH_HIP_CHECK(c, hipMemcpyAsync(c->h_noconv, c->noconv, 4, hipMemcpyDeviceToHost, st));
  TSPH_HIP_CHECK(c, hipMemsetAsync(c->flags, 0, 4, st));
  TSPH_HIP_CHECK(c, hipMemsetAsync(c->noconv, 0, 4, st));
  TSPH_HIP_CHECK(c, hipStreamSynchronize(st));
  if (flags) *flags = c->h_flags[0];
  if (n_noconv) *n_noconv = c->h_noconv[0];
  return TSPH_OK;
}

tsph_status tsph_take_flags_async(void *ctx, uint32_t *dst, void *stream) {
  Ctx *c = (Ctx *)ctx;
  if (!c) return TSPH_EINVAL;
  if (!dst) return set_err(c, TSPH_EINVAL, "dst is NULL");
  hipStream_t st = (hipStream_t)stream;
  c->last_stream = st;
  TSPH_HIP_CHECK(c, hipMemcpyAsync(dst, c->flags, 4, hipMemcpyDefault, st));
  TSPH_HIP_CHECK(c, hipMemcpyAsync(dst + 1, c->noconv, 4, hipMemcpyDefault, st));
  TSPH_HIP_CHECK(c, hipMemsetAsync(c->flags, 0, 4, st));
  TSPH_HIP_CHECK(c, hipMemsetAsync(c->noconv, 0, 4, st));
  return TSPH_OK;
}

tsph_status tsph_debug_lists(void *ctx, int32_t max_per_particle) {
  Ctx *c = (Ctx *)ctx;
  if (!c || max_per_particle < 0) return TSPH_EINVAL;
  TSPH_HIP_CHECK(c, hipDeviceSynchronize());
  if (c->dbg_nbr) {
    TSPH_HIP_CHECK(c, hipFree(c->dbg_nbr));
    c->dbg_nbr = nullptr;
  }
  c->dbg_max = 0;
  if (max_per_particle == 0) return TSPH_OK;
  size_t bytes = (size_t)3 * c->cap_n * max_per_particle * sizeof(int32_t);
  if (hipMalloc(&c->dbg_nbr, bytes) != hipSuccess) {
    (void)hipGetLastError();
    c->dbg_nbr = nullptr;
    return set_err(c, TSPH_ENOMEM, "debug list allocation failed");
  }
  c->dbg_max = max_per_particle;
  return TSPH_OK;
}

tsph_status tsph_debug_export(void *ctx, int32_t what, void *host, size_t cap_bytes, size_t *written) {
  Ctx *c = (Ctx *)ctx;
  if (!c || !host) return TSPH_EINVAL;
  TSPH_HIP_CHECK(c, hipStreamSynchronize(c->last_stream));
  TSPH_HIP_CHECK(c, hipDeviceSynchronize());
  const int64_t n = c->n;
  int32_t lvl[64];
  TSPH_HIP_CHECK(c, hipMemcpy(lvl, c->lvl, sizeof(lvl), hipMemcpyDeviceToHost));
  const int64_t nn = lvl[46];
  int32_t ngr = 0, nbat = 0;
  TSPH_HIP_CHECK(c, hipMemcpy(&ngr, c->ngroups, 4, hipMemcpyDeviceToHost));
  TSPH_HIP_CHECK(c, hipMemcpy(&nbat, c->nbatches, 4, hipMemcpyDeviceToHost));
  size_t need = 0;
  switch (what) {
    case TSPH_DBG_KEYS: need = 8 * n; break;
    case TSPH_DBG_PERM: need = 4 * n; break;
    case TSPH_DBG_NODES: need = 4 * 7 * nn; break;
    case TSPH_DBG_NNODES: need = 8; break;
    case TSPH_DBG_MOMENTS: need = 8 * 16 * nn; break;
    case TSPH_DBG_GROUPS: need = 4 * (size_t)ngr; break;
    case TSPH_DBG_NGROUPS: need = 8; break;
    case TSPH_DBG_COUNTS: need = 4 * 3 * n; break;
    case TSPH_DBG_NBR: need = (size_t)4 * 3 * n * c->dbg_max; break;
    case TSPH_DBG_ROOT: need = 8 * 4; break;
    case TSPH_DBG_SOLVE: need = 8 * (size_t)kNumSolve * n; break;
    case TSPH_DBG_BATCHES: need = 8 * (size_t)nbat; break;
    case TSPH_DBG_NBATCHES: need = 8; break;
    default: return set_err(c, TSPH_EINVAL, "unknown export");
  }
  if (written) *written = need;
  if (cap_bytes < need) return set_err(c, TSPH_EINVAL, "host buffer too small");
  switch (what) {
    case TSPH_DBG_KEYS: TSPH_HIP_CHECK(c, hipMemcpy(host, c->key[0], need, hipMemcpyDeviceToHost)); break;
    case TSPH_DBG_PERM: TSPH_HIP_CHECK(c, hipMemcpy(host, c->perm, need, hipMemcpyDeviceToHost)); break;
    case TSPH_DBG_NNODES: *(int64_t *)host = nn; break;
    case TSPH_DBG_NGROUPS: *(int64_t *)host = ngr; break;
    case TSPH_DBG_NBATCHES: *(int64_t *)host = nbat; break;
    case TSPH_DBG_BATCHES: TSPH_HIP_CHECK(c, hipMemcpy(host, c->batches, need, hipMemcpyDeviceToHost)); break;
    case TSPH_DBG_GROUPS: TSPH_HIP_CHECK(c, hipMemcpy(host, c->groups, need, hipMemcpyDeviceToHost)); break;
    case TSPH_DBG_NODES: {
      std::vector<NodeTopo> t(nn);
      std::vector<int32_t> lev(nn), par(nn), ng(nn);
      TSPH_HIP_CHECK(c, hipMemcpy(t.data(), c->topo, nn * sizeof(NodeTopo), hipMemcpyDeviceToHost));
      TSPH_HIP_CHECK(c, hipMemcpy(lev.data(), c->nlevel, nn * 4, hipMemcpyDeviceToHost));
      TSPH_HIP_CHECK(c, hipMemcpy(par.data(), c->nparent, nn * 4, hipMemcpyDeviceToHost));
      TSPH_HIP_CHECK(c, hipMemcpy(ng.data(), c->nngas, nn * 4, hipMemcpyDeviceToHost));
      int32_t *o = (int32_t *)host;
      for (int64_t k = 0; k < nn; k++) {
        o[0 * nn + k] = lev[k];
        o[1 * nn + k] = t[k].first;
        o[2 * nn + k] = t[k].count;
        o[3 * nn + k] = t[k].child;
        o[4 * nn + k] = t[k].nchild;
        o[5 * nn + k] = par[k];
        o[6 * nn + k] = ng[k];
      }
      break;
    }
    case TSPH_DBG_MOMENTS: {
      std::vector<NodeFar> f(nn);
      std::vector<NodeBox> bx(nn);
      TSPH_HIP_CHECK(c, hipMemcpy(f.data(), c->nfar, nn * sizeof(NodeFar), hipMemcpyDeviceToHost));
      TSPH_HIP_CHECK(c, hipMemcpy(bx.data(), c->nbox, nn * sizeof(NodeBox), hipMemcpyDeviceToHost));
      double *o = (double *)host;
      for (int64_t k = 0; k < nn; k++) {
        double v[16] = {f[k].m, f[k].cx, f[k].cy, f[k].cz, f[k].qxx, f[k].qyy, f[k].qzz, f[k].qxy,
                        f[k].qxz, f[k].qyz, bx[k].lox, bx[k].loy, bx[k].loz, bx[k].hix, bx[k].hiy, bx[k].hiz};
        for (int a = 0; a < 16; a++) o[a * nn + k] = v[a];
      }
      break;
    }
    case TSPH_DBG_COUNTS:
      for (int a = 0; a < 3; a++)
        TSPH_HIP_CHECK(c, hipMemcpy((int32_t *)host + a * n, c->cnt + a * c->cap_n, 4 * n, hipMemcpyDeviceToHost));
      break;
    case TSPH_DBG_NBR:
      if (!c->dbg_nbr) return set_err(c, TSPH_EINVAL, "debug lists are not enabled");
      for (int a = 0; a < 3; a++)
        TSPH_HIP_CHECK(c, hipMemcpy((int32_t *)host + (size_t)a * n * c->dbg_max,
                                    c->dbg_nbr + (size_t)a * c->cap_n * c->dbg_max,
                                    (size_t)4 * n * c->dbg_max, hipMemcpyDeviceToHost));
      break;
    case TSPH_DBG_ROOT: {
      DevRoot r;
      TSPH_HIP_CHECK(c, hipMemcpy(&r, c->root, sizeof(r), hipMemcpyDeviceToHost));
      double *o = (double *)host;
      o[0] = r.x0;
      o[1] = r.y0;
      o[2] = r.z0;
      o[3] = r.side;
      break;
    }
    case TSPH_DBG_SOLVE: {
      std::vector<int32_t> perm(n);
      std::vector<double> tmp(n);
      TSPH_HIP_CHECK(c, hipMemcpy(perm.data(), c->perm, 4 * n, hipMemcpyDeviceToHost));
      double *o = (double *)host;
      for (int a = 0; a < kNumSolve; a++) {
        TSPH_HIP_CHECK(c, hipMemcpy(tmp.data(), c->solve + (size_t)a * c->cap_n, 8 * n, hipMemcpyDeviceToHost));
        for (int64_t p = 0; p < n; p++) o[(size_t)a * n + perm[p]] = tmp[p];
      }
      break;
    }
  }
  return TSPH_OK;
}

tsph_status tsph_debug_handoff_cap(void *ctx, int64_t items) {
  Ctx *c = (Ctx *)ctx;
  if (!c || items < 0) return TSPH_EINVAL;
  c->split_cap_limit = items;
  return TSPH_OK;
}

const char *tsph_last_error(const void *ctx) {
  const Ctx *c = (const Ctx *)ctx;
  if (c) return c->err;
  return g_create_err[0] ? g_create_err : "no context";
}

}  // extern "C"
