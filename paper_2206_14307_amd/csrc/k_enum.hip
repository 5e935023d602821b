// Enumeration of the Sz = 0 sector (the exact checks of Sec. 3.3 run over
// all of it on the 4x4 lattice): the configurations with N/2 up spins, row r
// being the r-th set of up sites in colex order, i.e. in increasing order of
// the bit mask sum_{i up} 2^i.
//
// Rank r is unranked through the combinatorial number system: the up sites
// c_1 < ... < c_k (k = N/2) are the unique ones with r = sum_i C(c_i, i), so
// from i = k down to 1, c_i is the largest c with C(c, i) <= the remaining
// rank.  One thread per row; the binomials come from a table built on the
// host.
#include "device_common.h"
#include "nqs_internal.h"

namespace nqs {

namespace {

__global__ void enum_sz0_kernel(int N, int64_t count, const uint64_t* __restrict__ binom,
                                int8_t* __restrict__ out) {
  const int64_t r0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r0 >= count) return;
  const int k = N / 2, W = N + 1;
  uint64_t r = (uint64_t)r0, up_lo = 0, up_hi = 0;
  int x = N;                                   // c_i < x
  for (int i = k; i >= 1; --i) {
    int c = x - 1;
    while (binom[c * W + i] > r) --c;        // C(i - 1, i) = 0 ends the scan
    r -= binom[c * W + i];
    if (c < 64) up_lo |= 1ull << c;
    else up_hi |= 1ull << (c - 64);
    x = c;
  }
  int8_t* row = out + r0 * N;
  for (int j = 0; j < N; ++j) {
    const bool up = j < 64 ? ((up_lo >> j) & 1ull) : ((up_hi >> (j - 64)) & 1ull);
    row[j] = up ? (int8_t)1 : (int8_t)-1;
  }
}

}  // namespace

// C(n, i) for 0 <= i <= n <= N, row-major [N+1][N+1]; false if C(N, N/2)
// does not fit in int64.
bool sz0_binomials(int N, std::vector<uint64_t>& b, int64_t& count) {
  const int W = N + 1;
  b.assign((size_t)W * W, 0);
  for (int n = 0; n <= N; ++n) {
    b[(size_t)n * W] = 1;
    for (int i = 1; i <= n; ++i) {
      const uint64_t a = b[(size_t)(n - 1) * W + i - 1], c = i <= n - 1 ? b[(size_t)(n - 1) * W + i] : 0;
      if (a > (uint64_t)INT64_MAX - c) return false;
      b[(size_t)n * W + i] = a + c;
    }
  }
  count = (int64_t)b[(size_t)N * W + N / 2];
  return true;
}

hipError_t launch_enum_sz0(const nqs_ctx* c, int64_t count, int8_t* out, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int64_t blocks = (count + 255) / 256;
  enum_sz0_kernel<<<(unsigned)blocks, 256, 0, st>>>(c->N, count, c->dev.binom, out);
  return hipGetLastError();
}

}  // namespace nqs
