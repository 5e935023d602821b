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
// so s_i is a scalar for every site.  The transform is separable,
// F(q) = sum_y e^{i ky' y} sum_x s_{x,y} e^{i kx' x} (kx' = 2 pi kx / L), so
// each lane keeps its two rows of L phases in registers: two FMAs per site
// and one complex product per lattice row, independent across rows.  Blocks
// write partial sums (per momentum, and the weight sum) to the workspace; a
// finish kernel adds them in a fixed order.
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
  __shared__ double red[kSqWaves][N + 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double cxr[NQL][L], cxi[NQL][L], cyr[NQL][L], cyi[NQL][L], acc[NQL];
#pragma unroll
  for (int u = 0; u < NQL; ++u) {
    const int q = (lane + 64 * u) % N;   // lanes past N repeat a momentum, unused
    const int kx = q % L, ky = q / L;
#pragma unroll
    for (int v = 0; v < L; ++v) {
      sincospi(2.0 * (double)((kx * v) % L) / L, &cxi[u][v], &cxr[u][v]);
      sincospi(2.0 * (double)((ky * v) % L) / L, &cyi[u][v], &cyr[u][v]);
    }
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
        double rr = 0.0, ri = 0.0;
#pragma unroll
        for (int x = 0; x < L; ++x) {
          const int i = x + L * y;
          const bool up = i < 64 ? ((up0 >> i) & 1ull) : ((up1 >> (i - 64)) & 1ull);
          const double sg = up ? 0.5 : -0.5;
          rr = fma(sg, cxr[u][x], rr);
          ri = fma(sg, cxi[u][x], ri);
        }
        fr = fma(rr, cyr[u][y], fma(-ri, cyi[u][y], fr));
        fi = fma(rr, cyi[u][y], fma(ri, cyr[u][y], fi));
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

// out[q] = sum_b part[b][q] / (N^2 sum_b part[b][N]): one block per momentum;
// thread t adds the partials b = t, t + 256, ... and a fixed tree joins the
// threads, so the result does not depend on timing.  Every block forms the
// weight sum itself.
__global__ __launch_bounds__(256) void sq_finish_kernel(const double* __restrict__ part, int nblk,
                                                        int N, double* __restrict__ out) {
  __shared__ double rv[256], rw[256];
  const int q = blockIdx.x, t = threadIdx.x;
  double v = 0.0, w = 0.0;
  for (int b = t; b < nblk; b += 256) {
    v += part[(size_t)b * (N + 1) + q];
    w += part[(size_t)b * (N + 1) + N];
  }
  rv[t] = v;
  rw[t] = w;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
      rv[t] += rv[t + h];
      rw[t] += rw[t + h];
    }
    __syncthreads();
  }
  if (t == 0) out[q] = rv[0] / (rw[0] * (double)N * (double)N);
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
  sq_finish_kernel<<<L * L, 256, 0, st>>>(part, nblk, L * L, out);
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
