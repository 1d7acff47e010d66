// integrate.hip -- output scatter, kick-drift-kick leapfrog, global
// time-step and FP64 diagnostics.
//
// Merlin et al., arXiv:0912.1786: Sect. 4.1 (KDK with the predicted velocity
// v_n + a_n dt used at the end of the step), Sect. 4.2 (time-step criteria),
// Sect. 2.1 (potential of the softened system, Eqs. Lagrangian, potential).
// All integrator arithmetic is FP64 and elementwise, so these kernels are
// bound by HBM bandwidth.  Reductions run in a fixed tree order and are
// bit-reproducible.
#include <stdio.h>

#include <mutex>

#include "tsph_internal.h"

namespace tsph {

constexpr int kRedBlocks = 1024;       // partial reductions of a single system

struct FinishArgs {
  int64_t n, cap_n;
  const int32_t *perm;
  const uint8_t *gas;
  const uint8_t *act;  // key order: force outputs of these only (NULL: all)
  const double *acc;
  const double4 *sph;
  const double4 *vu;
  const double *hs, *es, *solve;
  double *ax, *ay, *az, *pot, *dudt, *rho, *h, *eps;
  double *pdiv;  // kCarryRows x cap_n, caller order
  double alpha, gamma, xsph_eta;
  int32_t entropy;
  // dissipation switches: key-order alpha, alpha_u; floors
  const double2 *av;
  int32_t alpha_switch, conduction;
  double alpha_min, alpha_u_min;
};

// Key order -> caller order: the lengths, densities and divergences of every
// particle, the forces and rates of the evaluated ones.
__global__ __launch_bounds__(256) void k_finish(FinishArgs A) {
  int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= A.n) return;
  const int i = A.perm[p];
  const bool g = A.gas[p];
  const double4 s = A.sph[p];
  if (A.rho) A.rho[i] = g ? s.y : 0.0;
  if (A.h) A.h[i] = g ? A.hs[p] : 0.0;
  if (A.eps) A.eps[i] = A.es[p];
  A.pdiv[i] = g ? A.solve[kDivv * A.cap_n + p] : 0.0;
  A.pdiv[A.cap_n + i] = A.solve[kDivvE * A.cap_n + p];
  if (A.act && !A.act[p]) return;
  // with the entropic function as energy variable its rate is the viscous
  // heating times (gamma - 1) rho^(1 - gamma) (Sect. 3.4, Eq. SPHentr)
  const double du = !g ? 0.0
                       : (A.entropy ? (A.gamma - 1.0) * pow(s.y, 1.0 - A.gamma) * A.solve[kDuv * A.cap_n + p]
                                    : A.acc[4 * A.cap_n + p]);
  A.ax[i] = A.acc[p];
  A.ay[i] = A.acc[A.cap_n + p];
  A.az[i] = A.acc[2 * A.cap_n + p];
  if (A.pot) A.pot[i] = A.acc[3 * A.cap_n + p];
  if (A.dudt) A.dudt[i] = du;
  // X-SPH velocity correction of the next drift (Sect. 3.5, Eq. xsph)
  A.pdiv[2 * A.cap_n + i] = g ? A.xsph_eta * A.solve[kXsx * A.cap_n + p] : 0.0;
  A.pdiv[3 * A.cap_n + i] = g ? A.xsph_eta * A.solve[kXsy * A.cap_n + p] : 0.0;
  A.pdiv[4 * A.cap_n + i] = g ? A.xsph_eta * A.solve[kXsz * A.cap_n + p] : 0.0;
  // rates of the dissipation coefficients (Sect. 3.3.1, 3.3.2): relaxation to
  // the floor over tau = h / (0.1 v_sig), sources 0.75 f max(0, -div v) and
  // h |lap u| / sqrt(u)
  double da = 0.0, dau = 0.0;
  if (g && (A.alpha_switch || A.conduction)) {
    const double vs = A.solve[kVsig * A.cap_n + p];
    const double tau = vs > 0.0 ? s.x / (0.1 * vs) : INFINITY;
    const double2 al = A.av[p];
    if (A.alpha_switch) {
      const double dv = A.solve[kDivv * A.cap_n + p];
      da = -(al.x - A.alpha_min) / tau + 0.75 * A.solve[kFbal * A.cap_n + p] * (dv < 0.0 ? -dv : 0.0);
    }
    if (A.conduction) {
      const double uu = A.vu[p].w;
      dau = -(al.y - A.alpha_u_min) / tau +
            (uu > 0.0 ? s.x * fabs(A.solve[kLapu * A.cap_n + p]) / sqrt(uu) : 0.0);
    }
  }
  A.pdiv[5 * A.cap_n + i] = da;
  A.pdiv[6 * A.cap_n + i] = dau;
  A.pdiv[7 * A.cap_n + i] = g ? A.solve[kMaxmu * A.cap_n + p] : 0.0;
}

struct CritArgs {
  Members M;
  const double *ax, *ay, *az, *eps, *h, *u, *dudt, *rho, *alpha;
  const double *pdiv;
  int64_t cap_n;
  double *dt_i;  // caller order
  double eta_dt, alpha0, beta, gamma;
  int32_t hydro, entropy;
};

// Time-step criteria of Sect. 4.2 per particle (caller order) from the
// state: acceleration, Courant and internal-energy criteria, one eta.
__global__ __launch_bounds__(256) void k_criteria(CritArgs A) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= A.M.n) return;
  const bool g = member_gas(A.M, member_of(A.M, i), i);
  double dt = INFINITY;
  const double ax = A.ax[i], ay = A.ay[i], az = A.az[i];
  const double amag = sqrt(ax * ax + ay * ay + az * az);
  // min(eps, h) over the lengths the particle has (no softening: h alone)
  double len = (A.eps && A.eps[i] > 0.0) ? A.eps[i] : INFINITY;
  if (g && A.h[i] < len) len = A.h[i];
  if (amag > 0.0 && len < INFINITY) dt = fmin(dt, A.eta_dt * sqrt(len / amag));
  if (g && A.hydro) {
    const double u = A.u[i], hh = A.h[i];
    // with the entropic function A: c^2 = gamma A rho^(gamma - 1) (Sect. 3.4)
    const double c = A.entropy ? sqrt(A.gamma * u * pow(A.rho[i], A.gamma - 1.0))
                               : sqrt(A.gamma * (A.gamma - 1.0) * u);
    const double al = A.alpha ? A.alpha[i] : A.alpha0;
    const double den = hh * fabs(A.pdiv[i]) + c + 1.2 * (al * c + A.beta * A.pdiv[7 * A.cap_n + i]);
    if (den > 0.0) dt = fmin(dt, A.eta_dt * hh / den);
    const double du = A.dudt[i];
    if (du != 0.0) dt = fmin(dt, A.eta_dt * fabs(u / du));
  }
  A.dt_i[i] = dt;
}

// growth factor of a length over a drift of dt, clamped to [1/2, 2]
__device__ __forceinline__ double predict_factor(double dt, double divv) {
  double f = 1.0 + (dt / 3.0) * divv;
  if (!(f >= 0.5)) f = 0.5;
  else if (f > 2.0) f = 2.0;
  return f;
}

// dt: the same for every member, or dt_dev[member] when dt_dev is given
__global__ __launch_bounds__(256) void k_kick_drift(Members M, double dt, int phase, double *x,
                                                    double *y, double *z, double *vx, double *vy, double *vz,
                                                    double *u, const double *__restrict__ ax,
                                                    const double *__restrict__ ay, const double *__restrict__ az,
                                                    const double *__restrict__ dudt, double *vpx, double *vpy,
                                                    double *vpz, double *up, double *h, double *eps,
                                                    const double *__restrict__ pdiv, int64_t cap_n,
                                                    const double *__restrict__ dt_dev, int xsph, double *alpha,
                                                    double *alpha_u, double alpha_min, double alpha_u_min,
                                                    double period) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= M.n) return;
  const int mem = member_of(M, i);
  const bool gas = member_gas(M, mem, i);
  if (dt_dev) {
    dt = dt_dev[mem];
    if (!(dt >= 0.0 && dt < INFINITY)) return;
  }
  const double hdt = 0.5 * dt;
  const double a0 = ax[i], a1 = ay[i], a2 = az[i];
  double v0 = vx[i], v1 = vy[i], v2 = vz[i];
  if (phase == TSPH_KD_FIRST) {
    if (vpx) {
      vpx[i] = v0 + dt * a0;
      vpy[i] = v1 + dt * a1;
      vpz[i] = v2 + dt * a2;
    }
    v0 += hdt * a0;
    v1 += hdt * a1;
    v2 += hdt * a2;
    if (xsph && pdiv && gas) {
      // X-SPH: the gas drifts with v + dv of the last force pass (Eq. xsph)
      x[i] += dt * (v0 + pdiv[2 * cap_n + i]);
      y[i] += dt * (v1 + pdiv[3 * cap_n + i]);
      z[i] += dt * (v2 + pdiv[4 * cap_n + i]);
    } else {
      x[i] += dt * v0;
      y[i] += dt * v1;
      z[i] += dt * v2;
    }
    if (period > 0.0) {  // back into the periodic box
      x[i] = in_box(x[i], period);
      y[i] = in_box(y[i], period);
      z[i] = in_box(z[i], period);
    }
    // lengths along the drift: h n^(1/3) = eta with dn/dt = -n div v gives
    // dh/dt = (h/3) div v (Sect. 2.1); the next solve starts from them
    if (pdiv) {
      if (h && gas && h[i] > 0.0) h[i] *= predict_factor(dt, pdiv[i]);
      if (eps && eps[i] > 0.0) eps[i] *= predict_factor(dt, pdiv[cap_n + i]);
    }
    if (gas) {
      const double du = dudt[i];
      if (up) up[i] = u[i] + dt * du;
      u[i] += hdt * du;
    }
  } else {
    v0 += hdt * a0;
    v1 += hdt * a1;
    v2 += hdt * a2;
    if (gas) u[i] += hdt * dudt[i];
  }
  vx[i] = v0;
  vy[i] = v1;
  vz[i] = v2;
  // the dissipation coefficients follow the half kicks with the rates of the
  // last force pass, kept at or above their floors
  if (pdiv && gas) {
    if (alpha) alpha[i] = fmax(alpha[i] + hdt * pdiv[5 * cap_n + i], alpha_min);
    if (alpha_u) alpha_u[i] = fmax(alpha_u[i] + hdt * pdiv[6 * cap_n + i], alpha_u_min);
  }
}

// grid (blocks per member, members); a in key or caller order (member m
// holds the same range in both)
__global__ __launch_bounds__(256) void k_min_partial(Members M, const double *__restrict__ a,
                                                     double *__restrict__ part) {
  __shared__ double s[256];
  double v = INFINITY;
  const int mem = blockIdx.y;
  const int64_t i1 = member_end(M, mem);
  for (int64_t i = member_begin(M, mem) + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < i1;
       i += (int64_t)gridDim.x * blockDim.x)
    v = fmin(v, a[i]);
  s[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] = fmin(s[threadIdx.x], s[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)mem * gridDim.x + blockIdx.x] = s[0];
}

// one block per member over its nb partial minima
__global__ __launch_bounds__(256) void k_min_final(int nb, const double *__restrict__ part, double *__restrict__ out,
                                                   double *__restrict__ keep) {
  __shared__ double s[256];
  double v = INFINITY;
  part += (int64_t)blockIdx.x * nb;
  for (int i = threadIdx.x; i < nb; i += 256) v = fmin(v, part[i]);
  s[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] = fmin(s[threadIdx.x], s[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (out) out[blockIdx.x] = s[0];
    if (keep) keep[blockIdx.x] = s[0];
  }
}

constexpr int kNDiag = 9;

// grid (blocks per member, members)
__global__ __launch_bounds__(256) void k_diag_partial(Members M, const double *__restrict__ x,
                                                      const double *__restrict__ y, const double *__restrict__ z,
                                                      const double *__restrict__ vx, const double *__restrict__ vy,
                                                      const double *__restrict__ vz, const double *__restrict__ m,
                                                      const double *__restrict__ u, const double *__restrict__ pot,
                                                      double *__restrict__ part, const double *__restrict__ rho,
                                                      double gamma, int entropy) {
  double acc[kNDiag] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int mem = blockIdx.y;
  // member ranges clamped to [0, n): tables the host never read stay in bounds
  const int64_t i0 = max((int64_t)0, min(member_begin(M, mem), M.n));
  const int64_t i1 = max(i0, min(member_end(M, mem), M.n));
  const int64_t gas_end = i0 + (M.count <= 1 ? M.n_gas : M.ngas[mem]);
  for (int64_t i = i0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < i1;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double mi = m[i], a = vx[i], b = vy[i], c = vz[i];
    acc[0] += 0.5 * mi * (a * a + b * b + c * c);
    // u = A rho^(gamma - 1) / (gamma - 1) with the entropy variable (Sect. 3.4)
    if (i < gas_end && u) acc[1] += mi * (entropy ? u[i] * pow(rho[i], gamma - 1.0) / (gamma - 1.0) : u[i]);
    if (pot) acc[2] += 0.5 * mi * pot[i];
    acc[3] += mi * a;
    acc[4] += mi * b;
    acc[5] += mi * c;
    acc[6] += mi * (y[i] * c - z[i] * b);
    acc[7] += mi * (z[i] * a - x[i] * c);
    acc[8] += mi * (x[i] * b - y[i] * a);
  }
  __shared__ double s[kNDiag][256];
  for (int k = 0; k < kNDiag; k++) s[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int k = 0; k < kNDiag; k++) s[k][threadIdx.x] += s[k][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < kNDiag) part[((int64_t)mem * gridDim.x + blockIdx.x) * kNDiag + threadIdx.x] = s[threadIdx.x][0];
}

// one block per member: out[member * 9 + k]
__global__ __launch_bounds__(256) void k_diag_final(int nb, const double *__restrict__ part, double *__restrict__ out) {
  __shared__ double s[256];
  part += (int64_t)blockIdx.x * nb * kNDiag;
  out += (int64_t)blockIdx.x * kNDiag;
  for (int k = 0; k < kNDiag; k++) {
    double v = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) v += part[i * kNDiag + k];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = s[0];
    __syncthreads();
  }
}

}  // namespace tsph

using namespace tsph;

tsph_status tsph_impl_finish(Ctx *c, tsph_state *s, hipStream_t st) {
  FinishArgs A;
  A.n = c->n;
  A.cap_n = c->cap_n;
  A.perm = c->perm;
  A.gas = c->gas;
  A.act = c->blk_on ? c->bact_s : nullptr;
  A.acc = c->acc;
  A.sph = c->sph;
  A.vu = c->vu;
  A.hs = c->hs;
  A.es = c->es;
  A.solve = c->solve;
  A.ax = s->ax;
  A.ay = s->ay;
  A.az = s->az;
  A.pot = s->pot;
  A.dudt = s->dudt;
  A.rho = s->rho;
  A.h = s->h;
  A.eps = s->eps;
  A.pdiv = c->pdiv;
  A.alpha = c->p.alpha;
  A.gamma = c->p.gamma;
  A.xsph_eta = c->p.xsph_eta;
  A.entropy = c->p.entropy;
  A.av = c->av;
  A.alpha_switch = c->p.alpha_switch;
  A.conduction = c->p.conduction;
  A.alpha_min = c->p.alpha_min;
  A.alpha_u_min = c->p.alpha_u_min;
  hipLaunchKernelGGL(k_finish, dim3(blocks_for(c->n, 256, 1 << 20)), dim3(256), 0, st, A);
  TSPH_HIP_CHECK(c, hipGetLastError());
  return TSPH_OK;
}

tsph_status tsph_impl_criteria(Ctx *c, const tsph_state *s, hipStream_t st) {
  CritArgs A;
  A.M = members_of(c, s->n, s->n_gas);
  A.ax = s->ax;
  A.ay = s->ay;
  A.az = s->az;
  A.eps = c->p.gravity ? s->eps : nullptr;
  A.h = s->h;
  A.u = s->u;
  A.dudt = s->dudt;
  A.rho = s->rho;
  A.alpha = c->p.alpha_switch ? s->alpha : nullptr;
  A.pdiv = c->pdiv;
  A.cap_n = c->cap_n;
  A.dt_i = c->acc + 5 * c->cap_n;
  A.eta_dt = c->p.eta_dt;
  A.alpha0 = c->p.alpha;
  A.beta = c->p.beta;
  A.gamma = c->p.gamma;
  A.hydro = c->p.hydro && s->n_gas > 0;
  A.entropy = c->p.entropy;
  hipLaunchKernelGGL(k_criteria, dim3(blocks_for(s->n, 256, 1 << 20)), dim3(256), 0, st, A);
  TSPH_HIP_CHECK(c, hipGetLastError());
  return TSPH_OK;
}

tsph_status tsph_impl_kick_drift(Ctx *c, tsph_state *s, double dt, const double *dt_dev, int phase,
                                 hipStream_t st) {
  hipLaunchKernelGGL(k_kick_drift, dim3(blocks_for(s->n, 256, 1 << 20)), dim3(256), 0, st,
                     members_of(c, s->n, s->n_gas), dt, phase, s->x, s->y, s->z, s->vx, s->vy, s->vz, s->u, s->ax, s->ay, s->az, s->dudt, s->vpx,
                     s->vpy, s->vpz, s->up, s->h, s->eps, c->pdiv_n == s->n ? c->pdiv : nullptr, c->cap_n,
                     dt_dev, c->p.xsph_eta > 0.0 ? 1 : 0, c->p.alpha_switch ? s->alpha : nullptr,
                     c->p.conduction ? s->alpha_u : nullptr, c->p.alpha_min, c->p.alpha_u_min, c->p.period);
  TSPH_HIP_CHECK(c, hipGetLastError());
  return TSPH_OK;
}

tsph_status tsph_impl_timestep(Ctx *c, const tsph_state *s, double *dt_device, hipStream_t st) {
  tsph_status r = tsph_impl_criteria(c, s, st);
  if (r != TSPH_OK) return r;
  // the minimum of each member, in a fixed tree order
  const Members M = members_of(c, s->n, s->n_gas);
  const int rb = M.count > 1 ? kMemberBlocks : kRedBlocks;
  hipLaunchKernelGGL(k_min_partial, dim3(rb, M.count), dim3(256), 0, st, M, c->acc + 5 * c->cap_n, c->red);
  hipLaunchKernelGGL(k_min_final, dim3(M.count), dim3(256), 0, st, rb, c->red, dt_device, c->dt);
  TSPH_HIP_CHECK(c, hipGetLastError());
  return TSPH_OK;
}

// diagnostics of the systems of M: partial sums per block to part, totals to out
static hipError_t launch_diagnostics(const Members &M, const tsph_state *s, double *part, double *out,
                                     hipStream_t st, double gamma = 0.0, int entropy = 0) {
  const int rb = M.count > 1 ? kMemberBlocks : kRedBlocks;
  hipLaunchKernelGGL(k_diag_partial, dim3(rb, M.count), dim3(256), 0, st, M, s->x, s->y, s->z, s->vx, s->vy,
                     s->vz, s->m, s->u, s->pot, part, s->rho, gamma, entropy);
  hipLaunchKernelGGL(k_diag_final, dim3(M.count), dim3(256), 0, st, rb, part, out);
  return hipGetLastError();
}

tsph_status tsph_impl_diagnostics(Ctx *c, const tsph_state *s, double *out, hipStream_t st) {
  if (c->p.entropy && s->n_gas > 0 && !s->rho) return TSPH_EINVAL;
  TSPH_HIP_CHECK(c, launch_diagnostics(members_of(c, s->n, s->n_gas), s, c->red, out, st, c->p.gamma, c->p.entropy));
  return TSPH_OK;
}

// ---------------------------------------------------------------------------
// Diagnostics without a context and without allocation: the partial sums go
// to a static device array (one copy per GPU, held until the process ends).
// In host code `scratch` names a host-side stand-in, so its device address on
// each GPU is taken once with hipGetSymbolAddress and used from then on.
// ---------------------------------------------------------------------------
constexpr int64_t kScratchDoubles = TSPH_NOALLOC_SCRATCH_BYTES / 8;
static_assert(TSPH_NOALLOC_MAX_SYSTEMS * kMemberBlocks * kNDiag <= kScratchDoubles, "scratch too small");
static_assert(kRedBlocks * kNDiag <= kScratchDoubles, "scratch too small");
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices];

// device address of this GPU's scratch array (taken on first use)
hipError_t scratch_for_device(double **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (double *)p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

thread_local char g_noalloc_err[256] = "";
}  // namespace

extern "C" tsph_status tsph_diagnostics_noalloc(const tsph_state *s, int32_t count, const int64_t *off_device,
                                                const int64_t *ngas_device, double *out_device, void *stream) {
  auto fail = [](tsph_status r, const char *msg) {
    snprintf(g_noalloc_err, sizeof(g_noalloc_err), "tsph_diagnostics_noalloc: %s", msg);
    return r;
  };
  if (!s || !out_device) return fail(TSPH_EINVAL, "state and out_device are required");
  if (s->n < 1 || s->n_gas < 0 || s->n_gas > s->n) return fail(TSPH_EINVAL, "bad state sizes");
  if (!s->x || !s->y || !s->z || !s->vx || !s->vy || !s->vz || !s->m)
    return fail(TSPH_EINVAL, "diagnostics need x, v, m");
  if (count < 1) return fail(TSPH_EINVAL, "count must be >= 1");
  if (count > TSPH_NOALLOC_MAX_SYSTEMS) return fail(TSPH_ECAPACITY, "count exceeds TSPH_NOALLOC_MAX_SYSTEMS");
  if (count > 1 && (!off_device || !ngas_device))
    return fail(TSPH_EINVAL, "several systems need off_device and ngas_device");
  double *part = nullptr;
  hipError_t e = scratch_for_device(&part);
  if (e != hipSuccess) return fail(TSPH_EHIP, hipGetErrorString(e));
  const Members M{count > 1 ? off_device : nullptr, count > 1 ? ngas_device : nullptr, count, s->n, s->n_gas};
  e = launch_diagnostics(M, s, part, out_device, (hipStream_t)stream);
  if (e != hipSuccess) return fail(TSPH_EHIP, hipGetErrorString(e));
  return TSPH_OK;
}

extern "C" const char *tsph_noalloc_last_error(void) { return g_noalloc_err; }
