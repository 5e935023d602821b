// Pieces of one stochastic-reconfiguration training step (Sec. 3.2,
// Eq. (12) and the update theta <- theta + dtheta that follows it):
//   energy statistics of the configurations' local energies (FP64: mean,
//   centred second moment) and the parameter update with its checks.
// The step itself is composed on the host from the library's entry points
// (nqs_eloc, nqs_grad, nqs_sr_solve) in nqs_vmc_step.
#include "device_common.h"
#include "nqs_internal.h"

namespace nqs {

namespace {

constexpr int kStatThreads = 1024;

// Block-wide sum in a fixed order (one block, kStatThreads threads).
__device__ double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int h = kStatThreads / 2; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// stats[0..2] = Re <E>, Im <E>, <|E - <E>|^2> over the S local energies
// (complex, interleaved); two passes, the mean first.
__global__ __launch_bounds__(kStatThreads) void energy_stats_kernel(const double* __restrict__ e,
                                                                    int64_t S,
                                                                    double* __restrict__ stats) {
  __shared__ double red[kStatThreads];
  double sr = 0.0, si = 0.0;
  for (int64_t i = threadIdx.x; i < S; i += kStatThreads) {
    sr += e[2 * i];
    si += e[2 * i + 1];
  }
  const double mr = block_sum(sr, red) / (double)S;
  const double mi = block_sum(si, red) / (double)S;
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < S; i += kStatThreads) {
    const double dr = e[2 * i] - mr, di = e[2 * i + 1] - mi;
    v = fma(dr, dr, fma(di, di, v));
  }
  const double var = block_sum(v, red) / (double)S;
  if (threadIdx.x == 0) {
    stats[0] = mr;
    stats[1] = mi;
    stats[2] = var;
  }
}

// next = params + dtheta (complex [P]); the imaginary part is dropped for
// real models.  stats[3] = ||dtheta||_2 (of the applied step), stats[4] = 1
// when next holds a NaN or Inf.
__global__ __launch_bounds__(kStatThreads) void params_step_kernel(
    const double* __restrict__ params, const double* __restrict__ dtheta, int64_t P,
    int is_complex, double* __restrict__ next, double* __restrict__ stats) {
  __shared__ double red[kStatThreads];
  double n2 = 0.0, bad = 0.0;
  for (int64_t k = threadIdx.x; k < P; k += kStatThreads) {
    const double dr = dtheta[2 * k], di = is_complex ? dtheta[2 * k + 1] : 0.0;
    const double nr = params[2 * k] + dr, ni = params[2 * k + 1] + di;
    next[2 * k] = nr;
    next[2 * k + 1] = ni;
    n2 = fma(dr, dr, fma(di, di, n2));
    if (!isfinite(nr) || !isfinite(ni)) bad = 1.0;
  }
  const double norm2 = block_sum(n2, red);
  const double anybad = block_sum(bad, red);
  if (threadIdx.x == 0) {
    stats[3] = sqrt(norm2);
    stats[4] = anybad > 0.0 ? 1.0 : 0.0;
  }
}

}  // namespace

hipError_t launch_energy_stats(const double* eloc, int64_t S, double* stats, hipStream_t st) {
  energy_stats_kernel<<<1, kStatThreads, 0, st>>>(eloc, S, stats);
  return hipGetLastError();
}

hipError_t launch_params_step(const double* params, const double* dtheta, int64_t P, int is_complex,
                              double* next, double* stats, hipStream_t st) {
  params_step_kernel<<<1, kStatThreads, 0, st>>>(params, dtheta, P, is_complex, next, stats);
  return hipGetLastError();
}

}  // namespace nqs
