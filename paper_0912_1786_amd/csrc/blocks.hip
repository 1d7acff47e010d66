// blocks.hip -- individual power-of-two time-steps with wake-up.
//
// Merlin et al., arXiv:0912.1786: Sect. 4.2.1 (individual time-stepping:
// steps dt_max / 2^n, longer steps only where synchronised, active particles
// re-evaluated, the others lending predicted quantities, wake-up of
// neighbours whose step is too long), Sect. 4.1 (kick-drift-kick with the
// predicted velocity v_n + a_n dt), Sect. 4.2 (the criteria).
//
// Time runs in integer ticks, dt_max = 2^L ticks.  The per-particle kernels
// here are elementwise over caller order and HBM-bound; the force pass of
// the active particles is the ordinary one with chunks of 64 sinks without
// an active sink skipped by the gravity and SPH walks, and the wake-up minima
// are one more SPH-neighbour walk over the active gas (sph.hip, mode 2).
#include <stdio.h>

#include "tsph_internal.h"

namespace tsph {

// dt of a step of k ticks: exact (a power-of-two scaling of dt_max) when k is
// a power of two, k * (dt_max / 2^L) otherwise
__device__ __forceinline__ double tick_dt(int64_t k, double dt_max, int L) {
  if (k > 0 && (k & (k - 1)) == 0) return ldexp(dt_max, (63 - __builtin_clzll((uint64_t)k)) - L);
  return (double)k * ldexp(dt_max, -L);
}

__device__ __forceinline__ double grow(double dt, double divv) {
  double f = 1.0 + (dt / 3.0) * divv;
  if (!(f >= 0.5)) f = 0.5;
  else if (f > 2.0) f = 2.0;
  return f;
}

struct BlkArgs {
  int64_t n, n_gas, cap_n;
  double *x, *y, *z, *vx, *vy, *vz, *u;
  const double *ax, *ay, *az, *dudt;
  double *vpx, *vpy, *vpz, *up, *h, *eps, *alpha, *alpha_u;
  const double *pdiv;
  int32_t *t0, *t1;
  double *vsx, *vsy, *vsz, *us;
  uint8_t *act;
  int32_t *cur, *cur_s;
  const int32_t *bm, *bw, *perm;
  const double *dt_i;
  int32_t *next;  // [0] next system time, [1] active count, [2] woken count
  double dt_max, alpha_min, alpha_u_min, period;
  int32_t L, wake, xsph, t, shift;
};

// the first system time: everything active, predictions = the state
__global__ __launch_bounds__(256) void k_blk_init(BlkArgs A) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  A.t0[i] = 0;
  A.t1[i] = 0;
  A.act[i] = 1;
  A.vpx[i] = A.vx[i];
  A.vpy[i] = A.vy[i];
  A.vpz[i] = A.vz[i];
  if (i < A.n_gas) A.up[i] = A.u[i];
}

__global__ void k_blk_clear(int32_t *next) {
  if (threadIdx.x == 0) {
    next[0] = INT32_MAX;
    next[1] = 0;
    next[2] = 0;
  }
}

// the earliest step end
__global__ __launch_bounds__(256) void k_blk_next(int64_t n, const int32_t *__restrict__ t1, int32_t *next) {
  int32_t v = INT32_MAX;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v = min(v, t1[i]);
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMin(next, v);
}

// Every particle to the system time tn with its half-kicked velocity (gas
// with the X-SPH correction), lengths along the drift as in Sect. 2.1, the
// predicted velocity and energy from the last synchronised state, and the
// active flags (step ends at tn).
__global__ __launch_bounds__(256) void k_blk_drift(BlkArgs A) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  const int tn = A.next[0];
  const bool gas = i < A.n_gas;
  const double d = tick_dt(tn - A.t, A.dt_max, A.L);
  const int64_t cap = A.cap_n;
  double v0 = A.vx[i], v1 = A.vy[i], v2 = A.vz[i];
  if (A.xsph && gas) {
    v0 = v0 + A.pdiv[2 * cap + i];
    v1 = v1 + A.pdiv[3 * cap + i];
    v2 = v2 + A.pdiv[4 * cap + i];
  }
  A.x[i] += d * v0;
  A.y[i] += d * v1;
  A.z[i] += d * v2;
  if (A.period > 0.0) {  // back into the periodic box
    A.x[i] = in_box(A.x[i], A.period);
    A.y[i] = in_box(A.y[i], A.period);
    A.z[i] = in_box(A.z[i], A.period);
  }
  if (A.h && gas && A.h[i] > 0.0) A.h[i] *= grow(d, A.pdiv[i]);
  if (A.eps && A.eps[i] > 0.0) A.eps[i] *= grow(d, A.pdiv[cap + i]);
  const double dp = tick_dt(tn - A.t0[i], A.dt_max, A.L);
  A.vpx[i] = A.vsx[i] + dp * A.ax[i];
  A.vpy[i] = A.vsy[i] + dp * A.ay[i];
  A.vpz[i] = A.vsz[i] + dp * A.az[i];
  if (gas) A.up[i] = A.us[i] + dp * A.dudt[i];
  const bool a = A.t1[i] == tn;
  A.act[i] = a;
  if (a) atomicAdd(&A.next[1], 1);
}

// half kick of particle i by dt/2 with its current rates
__device__ __forceinline__ void half_kick(const BlkArgs &A, int64_t i, double dt) {
  const double hdt = 0.5 * dt;
  A.vx[i] += hdt * A.ax[i];
  A.vy[i] += hdt * A.ay[i];
  A.vz[i] += hdt * A.az[i];
  if (i < A.n_gas) {
    A.u[i] += hdt * A.dudt[i];
    if (A.alpha) A.alpha[i] = fmax(A.alpha[i] + hdt * A.pdiv[5 * A.cap_n + i], A.alpha_min);
    if (A.alpha_u) A.alpha_u[i] = fmax(A.alpha_u[i] + hdt * A.pdiv[6 * A.cap_n + i], A.alpha_u_min);
  }
}

// closing half kick of the active particles (none at the first system time:
// kick = 0), their synchronised v and u, the shift of the tick origin at the
// end of the largest step
__global__ __launch_bounds__(256) void k_blk_close(BlkArgs A, int kick) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= A.n || !A.act[i]) return;
  if (kick) half_kick(A, i, tick_dt(A.t1[i] - A.t0[i], A.dt_max, A.L));
  A.vsx[i] = A.vx[i];
  A.vsy[i] = A.vy[i];
  A.vsz[i] = A.vz[i];
  if (i < A.n_gas) A.us[i] = A.u[i];
  A.t0[i] -= A.shift;
  A.t1[i] -= A.shift;
}

// criterion steps of the active particles (the largest power-of-two
// fraction of dt_max not above the criteria, shortened to divide the current
// tick), the current step of the others, in caller and key order
__global__ __launch_bounds__(256) void k_blk_choose(BlkArgs A) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= A.n) return;
  const int i = A.perm[p];
  int32_t c;
  if (A.act[i]) {
    const double dt = A.dt_i[i];
    int lev = A.L;
    for (int k = 0; k <= A.L; k++)
      if (ldexp(A.dt_max, -k) <= dt) {
        lev = k;
        break;
      }
    c = 1 << (A.L - lev);
    while (A.t % c) c >>= 1;
  } else {
    c = A.t1[i] - A.t0[i];
  }
  A.cur[i] = c;
  A.cur_s[p] = c;
}

// wake-up and the opening half kicks
__global__ __launch_bounds__(256) void k_blk_open(BlkArgs A) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  const bool gas = i < A.n_gas;
  const int64_t f = A.wake;
  if (A.act[i]) {
    int64_t len = A.cur[i];
    if (f > 0 && gas && A.bm[i] != INT32_MAX) {
      // at most f times the shortest step around it: the largest power of
      // two not above that (it divides len, hence the current tick)
      const int64_t cap = f * (int64_t)A.bm[i];
      const int64_t p2 = (int64_t)1 << (63 - __builtin_clzll((uint64_t)cap));
      if (p2 < len) len = p2;
    }
    A.t0[i] = A.t;
    A.t1[i] = A.t + (int32_t)len;
    half_kick(A, i, tick_dt(len, A.dt_max, A.L));
    return;
  }
  if (f > 0 && gas && A.bw[i] != INT32_MAX) {
    const int64_t w = A.bw[i];
    const int64_t t0 = A.t0[i], t1 = A.t1[i];
    if (t1 - t0 > f * w && A.t + w < t1) {
      // woken: the step now ends at t + w, its opening kick redone from the
      // synchronised state for the shorter step
      const double old = tick_dt(t1 - t0, A.dt_max, A.L);
      const int32_t e = A.t + (int32_t)w;
      const double nw = tick_dt(e - t0, A.dt_max, A.L);
      A.vx[i] = A.vsx[i] + 0.5 * nw * A.ax[i];
      A.vy[i] = A.vsy[i] + 0.5 * nw * A.ay[i];
      A.vz[i] = A.vsz[i] + 0.5 * nw * A.az[i];
      A.u[i] = A.us[i] + 0.5 * nw * A.dudt[i];
      if (A.alpha) A.alpha[i] = fmax(A.alpha[i] - 0.5 * (old - nw) * A.pdiv[5 * A.cap_n + i], A.alpha_min);
      if (A.alpha_u)
        A.alpha_u[i] = fmax(A.alpha_u[i] - 0.5 * (old - nw) * A.pdiv[6 * A.cap_n + i], A.alpha_u_min);
      A.t1[i] = e;
      atomicAdd(&A.next[2], 1);
    }
  }
}

__global__ __launch_bounds__(256) void k_gather_act(int64_t n, const int32_t *__restrict__ perm,
                                                    const uint8_t *__restrict__ act, uint8_t *__restrict__ act_s) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p < n) act_s[p] = act[perm[p]];
}

}  // namespace tsph

using namespace tsph;

tsph_status tsph_impl_gather_active(Ctx *c, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_act, dim3(blocks_for(c->n, 256, 1 << 20)), dim3(256), 0, st, c->n, c->perm, c->bact,
                     c->bact_s);
  TSPH_HIP_CHECK(c, hipGetLastError());
  return TSPH_OK;
}

namespace {

tsph_status blk_err(Ctx *c, tsph_status s, const char *msg) {
  snprintf(c->err, sizeof(c->err), "%s", msg);
  return s;
}

tsph_status blk_checks(Ctx *c, const tsph_state *s, const tsph_blocks *b) {
  if (!s || !b) return blk_err(c, TSPH_EINVAL, "state and blocks are required");
  if (c->nmem > 1) return blk_err(c, TSPH_EINVAL, "individual time-steps need a context holding one system");
  if (!(b->dt_max > 0.0) || !(b->dt_max < INFINITY)) return blk_err(c, TSPH_EINVAL, "dt_max must be positive");
  if (b->max_level < 0 || b->max_level > 30) return blk_err(c, TSPH_EINVAL, "max_level must be in [0, 30]");
  if (b->wake < 0 || b->wake > 64 || (b->wake & (b->wake - 1)))
    return blk_err(c, TSPH_EINVAL, "wake must be 0 or a power of two <= 64");
  if (!b->t0 || !b->t1 || !b->vsx || !b->vsy || !b->vsz || (s->n_gas > 0 && !b->us))
    return blk_err(c, TSPH_EINVAL, "t0, t1, vsx, vsy, vsz (and us with gas) are required");
  if (!s->u && s->n_gas > 0) return blk_err(c, TSPH_EINVAL, "gas needs u");
  return TSPH_OK;
}

BlkArgs blk_args(Ctx *c, tsph_state *s, tsph_blocks *b) {
  BlkArgs A;
  A.n = s->n;
  A.n_gas = s->n_gas;
  A.cap_n = c->cap_n;
  A.x = s->x; A.y = s->y; A.z = s->z;
  A.vx = s->vx; A.vy = s->vy; A.vz = s->vz;
  A.u = s->u;
  A.ax = s->ax; A.ay = s->ay; A.az = s->az;
  A.dudt = s->dudt;
  A.vpx = s->vpx; A.vpy = s->vpy; A.vpz = s->vpz; A.up = s->up;
  A.h = s->h;
  A.eps = s->eps;
  A.alpha = c->p.alpha_switch ? s->alpha : nullptr;
  A.alpha_u = c->p.conduction ? s->alpha_u : nullptr;
  A.pdiv = c->pdiv;
  A.t0 = b->t0; A.t1 = b->t1;
  A.vsx = b->vsx; A.vsy = b->vsy; A.vsz = b->vsz; A.us = b->us;
  A.act = c->bact;
  A.cur = c->bcur;
  A.cur_s = c->bcur_s;
  A.bm = c->bm;
  A.bw = c->bw;
  A.perm = c->perm;
  A.dt_i = c->acc + 5 * c->cap_n;
  A.next = c->bnext;
  A.dt_max = b->dt_max;
  A.alpha_min = c->p.alpha_min;
  A.alpha_u_min = c->p.alpha_u_min;
  A.period = c->p.period;
  A.L = b->max_level;
  A.wake = (c->p.hydro && s->n_gas > 0) ? b->wake : 0;
  A.xsph = c->p.xsph_eta > 0.0 ? 1 : 0;
  A.t = (int32_t)b->t;
  A.shift = 0;
  return A;
}

// After the force pass of system time A.t: close the active steps, choose
// the next ones, wake neighbours, open.  Reads the counts back.
tsph_status blk_finish(Ctx *c, tsph_state *s, tsph_blocks *b, BlkArgs &A, int kick, hipStream_t st) {
  const dim3 g(blocks_for(s->n, 256, 1 << 20)), t(256);
  hipLaunchKernelGGL(k_blk_close, g, t, 0, st, A, kick);
  A.t -= A.shift;
  A.shift = 0;
  tsph_status r = tsph_impl_criteria(c, s, st);
  if (r != TSPH_OK) return r;
  hipLaunchKernelGGL(k_blk_choose, g, t, 0, st, A);
  if (A.wake > 0 && (r = tsph_impl_wake(c, st)) != TSPH_OK) return r;
  hipLaunchKernelGGL(k_blk_open, g, t, 0, st, A);
  TSPH_HIP_CHECK(c, hipGetLastError());
  int32_t h[3];
  TSPH_HIP_CHECK(c, hipMemcpyAsync(h, c->bnext, sizeof(h), hipMemcpyDeviceToHost, st));
  TSPH_HIP_CHECK(c, hipStreamSynchronize(st));
  b->t = A.t;
  b->n_active = kick ? h[1] : s->n;
  b->n_woken = h[2];
  return TSPH_OK;
}

}  // namespace

extern "C" {

tsph_status tsph_block_start(void *ctx, tsph_state *s, tsph_blocks *b, void *stream) {
  Ctx *c = (Ctx *)ctx;
  if (!c) return TSPH_EINVAL;
  tsph_status r = blk_checks(c, s, b);
  if (r != TSPH_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  c->last_stream = st;
  b->t = 0;
  BlkArgs A = blk_args(c, s, b);
  const dim3 g(blocks_for(s->n, 256, 1 << 20)), t(256);
  hipLaunchKernelGGL(k_blk_clear, dim3(1), dim3(64), 0, st, c->bnext);
  hipLaunchKernelGGL(k_blk_init, g, t, 0, st, A);
  TSPH_HIP_CHECK(c, hipGetLastError());
  c->blk_on = 0;
  if ((r = tsph_compute_forces(ctx, s, stream)) != TSPH_OK) return r;
  return blk_finish(c, s, b, A, 0, st);
}

tsph_status tsph_block_advance(void *ctx, tsph_state *s, tsph_blocks *b, void *stream) {
  Ctx *c = (Ctx *)ctx;
  if (!c) return TSPH_EINVAL;
  tsph_status r = blk_checks(c, s, b);
  if (r != TSPH_OK) return r;
  if (c->pdiv_n != s->n) return blk_err(c, TSPH_EINVAL, "no tsph_block_start with this n");
  if (b->t < 0 || b->t >= ((int64_t)1 << b->max_level)) return blk_err(c, TSPH_EINVAL, "t out of range");
  hipStream_t st = (hipStream_t)stream;
  c->last_stream = st;
  BlkArgs A = blk_args(c, s, b);
  const dim3 g(blocks_for(s->n, 256, 1 << 20)), t(256);
  hipLaunchKernelGGL(k_blk_clear, dim3(1), dim3(64), 0, st, c->bnext);
  hipLaunchKernelGGL(k_blk_next, dim3(blocks_for(s->n, 256, 1024)), t, 0, st, s->n, b->t1, c->bnext);
  hipLaunchKernelGGL(k_blk_drift, g, t, 0, st, A);
  TSPH_HIP_CHECK(c, hipGetLastError());
  int32_t tn = 0;
  TSPH_HIP_CHECK(c, hipMemcpyAsync(&tn, c->bnext, sizeof(tn), hipMemcpyDeviceToHost, st));
  TSPH_HIP_CHECK(c, hipStreamSynchronize(st));
  if (tn <= b->t || tn > (1 << b->max_level)) return blk_err(c, TSPH_EINVAL, "step ends out of range");
  c->blk_on = 1;
  r = tsph_compute_forces(ctx, s, stream);
  c->blk_on = 0;
  if (r != TSPH_OK) return r;
  A.t = tn;
  A.shift = tn == (1 << b->max_level) ? tn : 0;
  return blk_finish(c, s, b, A, 1, st);
}

}  // extern "C"
