// probe.hip -- machine probes for the roofline denominators: what this
// build's kernels can issue (independent FMA chains in FP32 and FP64,
// compiled like every other kernel here, so without packed FP32) and what
// HBM delivers to a stream triad.  They measure the machine, not the method.
#include <algorithm>

#include "tsph_internal.h"

namespace {

constexpr int kProbeBlocks = 4096;  // 16 workgroups per CU
constexpr int kProbeThreads = 256;
constexpr int kChains = 8;          // independent FMA chains per thread

template <class T>
__global__ __launch_bounds__(kProbeThreads) void k_fma_chains(int64_t iters, double *sink) {
  const int t = blockIdx.x * kProbeThreads + threadIdx.x;
  T v[kChains];
#pragma unroll
  for (int k = 0; k < kChains; k++) v[k] = T(1) + T(1e-7) * T(t + k);
  const T a = T(0.999999), b = T(1e-7);
  for (int64_t i = 0; i < iters; i++) {
#pragma unroll
    for (int k = 0; k < kChains; k++) v[k] = fma(v[k], a, b);
  }
  T s = T(0);
#pragma unroll
  for (int k = 0; k < kChains; k++) s += v[k];
  // never true for these inputs; keeps the chains from being removed
  if (s == T(-1)) sink[0] = (double)s;
}

__global__ __launch_bounds__(kProbeThreads) void k_triad(int64_t n, double *__restrict__ a,
                                                         const double *__restrict__ b,
                                                         const double *__restrict__ c, double s) {
  const int64_t stride = (int64_t)gridDim.x * kProbeThreads;
  for (int64_t i = blockIdx.x * (int64_t)kProbeThreads + threadIdx.x; i < n; i += stride) a[i] = fma(s, c[i], b[i]);
}

}  // namespace

extern "C" tsph_status tsph_probe(int32_t kind, int64_t n, double *a, const double *b, const double *c,
                                  void *stream, double *work) {
  if (!work || !a || n < 1) return TSPH_EINVAL;
  const hipStream_t st = (hipStream_t)stream;
  if (kind == TSPH_PROBE_FMA32 || kind == TSPH_PROBE_FMA64) {
    if (n > (int64_t)1 << 20) return TSPH_EINVAL;
    if (kind == TSPH_PROBE_FMA32)
      hipLaunchKernelGGL(k_fma_chains<float>, dim3(kProbeBlocks), dim3(kProbeThreads), 0, st, n, a);
    else
      hipLaunchKernelGGL(k_fma_chains<double>, dim3(kProbeBlocks), dim3(kProbeThreads), 0, st, n, a);
    *work = 2.0 * kChains * (double)n * kProbeBlocks * kProbeThreads;
  } else if (kind == TSPH_PROBE_TRIAD) {
    if (!b || !c) return TSPH_EINVAL;
    // one element per thread (a grid-stride loop beyond 2^28 elements)
    const int64_t blocks = std::min<int64_t>((n + kProbeThreads - 1) / kProbeThreads, (int64_t)1 << 20);
    hipLaunchKernelGGL(k_triad, dim3((unsigned)blocks), dim3(kProbeThreads), 0, st, n, a, b, c, 0.5);
    *work = 24.0 * (double)n;
  } else {
    return TSPH_EINVAL;
  }
  return hipGetLastError() == hipSuccess ? TSPH_OK : TSPH_EHIP;
}
