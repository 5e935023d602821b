// Spin structure factor (Sec. 4, the equation defining S(q)):
//   S(q) = (1/N^2) sum_{i,j} <s_i s_j> e^{i q.(r_i - r_j)},  s = +-1/2,
// for every momentum q = 2 pi (kx, ky) / L of the torus.  For one
// configuration the double sum is |F(q)|^2 / N^2 with F(q) = sum_i s_i
// e^{i q.r_i}, so the expectation is the weighted mean of |F(q)|^2 / N^2 over
// the configurations (uniform weights for Monte-Carlo samples, |psi|^2 for an
// exact sum over the Sz = 0 sector).
//
// One wavefront per configuration at a time, one lane per momentum (two for
// N > 64).  The spin row becomes a wave-uniform mask of up spins (one vote),
// so s_i is a scalar for every site; the phases e^{2 pi i m / L} come from a
// small LDS table and each lane steps its phase index m = kx x + ky y (mod L)
// along the row.  Blocks write partial sums (per momentum, and the weight
// sum) to the workspace; a finish kernel adds them in a fixed order.
#include <algorithm>

#include "device_common.h"
#include "nqs_internal.h"

namespace nqs {

namespace {

constexpr int kSqWaves = 4;

template <int L>
__global__ __launch_bounds__(64 * kSqWaves) void sq_kernel(const int8_t* __restrict__ spins,
                                                           int64_t S,
                                                           const double* __restrict__ weights,
                                                           double* __restrict__ part) {
  constexpr int N = L * L, NQL = (N + 63) / 64;
  __shared__ double2 tw[L];
  __shared__ double red[kSqWaves][N + 1];
  if (threadIdx.x < L) {
    double sn, cs;
    sincospi(2.0 * (double)threadIdx.x / L, &sn, &cs);
    tw[threadIdx.x] = make_double2(cs, sn);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int kx[NQL], ky[NQL];
  double acc[NQL];
#pragma unroll
  for (int u = 0; u < NQL; ++u) {
    const int q = (lane + 64 * u) % N;   // lanes past N repeat a momentum, unused
    kx[u] = q % L;
    ky[u] = q / L;
    acc[u] = 0.0;
  }
  double wsum = 0.0;
  for (int64_t s = (int64_t)blockIdx.x * kSqWaves + wv; s < S;
       s += (int64_t)gridDim.x * kSqWaves) {
    const int8_t* row = spins + s * N;
    const uint64_t up0 = __builtin_amdgcn_ballot_w64(lane < N && row[lane] > 0);
    const uint64_t up1 =
        N > 64 ? __builtin_amdgcn_ballot_w64(lane + 64 < N && row[lane + 64] > 0) : 0ull;
    const double ws = weights ? weights[s] : 1.0;
#pragma unroll
    for (int u = 0; u < NQL; ++u) {
      double fr = 0.0, fi = 0.0;
#pragma unroll
      for (int y = 0; y < L; ++y) {
        int m = (ky[u] * y) % L;
#pragma unroll
        for (int x = 0; x < L; ++x) {
          const int i = x + L * y;
          const bool up = i < 64 ? ((up0 >> i) & 1ull) : ((up1 >> (i - 64)) & 1ull);
          const double sg = up ? 0.5 : -0.5;
          const double2 t = tw[m];
          fr = fma(sg, t.x, fr);
          fi = fma(sg, t.y, fi);
          m += kx[u];
          if (m >= L) m -= L;
        }
      }
      acc[u] = fma(ws, fma(fr, fr, fi * fi), acc[u]);
    }
    wsum += ws;
  }
#pragma unroll
  for (int u = 0; u < NQL; ++u)
    if (lane + 64 * u < N) red[wv][lane + 64 * u] = acc[u];
  if (lane == 0) red[wv][N] = wsum;
  __syncthreads();
  for (int idx = threadIdx.x; idx <= N; idx += blockDim.x) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < kSqWaves; ++w) v += red[w][idx];
    part[(size_t)blockIdx.x * (N + 1) + idx] = v;
  }
}

// out[q] = sum_b part[b][q] / (N^2 sum_b part[b][N]), blocks added in order.
__global__ __launch_bounds__(128) void sq_finish_kernel(const double* __restrict__ part, int nblk,
                                                        int N, double* __restrict__ out) {
  __shared__ double wsum;
  const int q = threadIdx.x;
  double v = 0.0;
  if (q <= N)
    for (int b = 0; b < nblk; ++b) v += part[(size_t)b * (N + 1) + q];
  if (q == N) wsum = v;
  __syncthreads();
  if (q < N) out[q] = v / (wsum * (double)N * (double)N);
}

int sq_blocks(const nqs_ctx* c, int64_t S) {
  const int64_t cap = 4 * (int64_t)(c->n_cu > 0 ? c->n_cu : 256);
  return (int)std::max<int64_t>(1, std::min<int64_t>((S + kSqWaves - 1) / kSqWaves, cap));
}

template <int L>
hipError_t run_sq(const nqs_ctx* c, const int8_t* spins, int64_t S, const double* weights,
                  double* out, double* part, hipStream_t st) {
  const int nblk = sq_blocks(c, S);
  sq_kernel<L><<<nblk, 64 * kSqWaves, 0, st>>>(spins, S, weights, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  sq_finish_kernel<<<1, 128, 0, st>>>(part, nblk, L * L, out);
  return hipGetLastError();
}

}  // namespace

size_t sq_workspace_bytes(const nqs_ctx* c, int64_t S) {
  return (size_t)sq_blocks(c, std::max<int64_t>(S, 1)) * (c->N + 1) * sizeof(double);
}

hipError_t launch_sq(const nqs_ctx* c, const int8_t* spins, int64_t S, const double* weights,
                     double* out, void* ws, hipStream_t st) {
  double* part = (double*)ws;
  switch (c->L) {
    case 4: return run_sq<4>(c, spins, S, weights, out, part, st);
    case 6: return run_sq<6>(c, spins, S, weights, out, part, st);
    case 8: return run_sq<8>(c, spins, S, weights, out, part, st);
    case 10: return run_sq<10>(c, spins, S, weights, out, part, st);
    default: return hipErrorNotSupported;
  }
}

}  // namespace nqs
