// Three-hop local values and the p = 2 Lanczos step (Sec. 3.3, Eq. (19)
// with p = 2).
//
// e3(s) = (H^3 psi)(s)/psi(s) = H_ss e2(s) + sum_b (J_b/2) psi(s^b)/psi(s) e2(s^b)
// over the bonds b whose spins are antiparallel in s.  The neighbours s^b
// are written out as ordinary configurations (compacted, bond order per
// configuration) so that the library's logpsi / E_loc / two-hop kernels give
// log psi(s^b) and e2(s^b); the combine kernel then forms e3.  The same
// combine forms e2 from the neighbours' E_loc for models without the
// register-resident two-hop kernel.  The moments
// kernel adds <|e2|^2>, Re<conj(e2) e3> and the centred mu4, mu5 to the p = 1
// results, and one thread solves the 3x3 Krylov eigenproblem.
#include "device_common.h"
#include "nqs_internal.h"
#include "hops.h"

namespace nqs {

namespace {

constexpr int kNbWaves = 4;

__device__ __forceinline__ bool bond_anti(const int8_t* srow, const int32_t* bonds, int b, int NB) {
  return b < NB && srow[bonds[2 * b]] != srow[bonds[2 * b + 1]];
}

// cnt[s] = number of antiparallel bonds of configuration s (one wavefront each).
__global__ __launch_bounds__(64 * kNbWaves) void nb_count_kernel(const int8_t* __restrict__ spins,
                                                                 int64_t n, int N, int NB,
                                                                 const int32_t* __restrict__ bonds,
                                                                 int32_t* __restrict__ cnt) {
  const int64_t s = (int64_t)blockIdx.x * kNbWaves + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (s >= n) return;
  const int8_t* srow = spins + s * N;
  int total = 0;
  for (int base = 0; base < NB; base += 64)
    total += __popcll(__ballot(bond_anti(srow, bonds, base + lane, NB)));
  if (lane == 0) cnt[s] = total;
}

// off[0..n]: exclusive prefix sums of cnt, off[n] = total (one block).
__global__ __launch_bounds__(1024) void nb_scan_kernel(const int32_t* __restrict__ cnt, int64_t n,
                                                       int32_t* __restrict__ off) {
  __shared__ int32_t buf[1024];
  const int t = threadIdx.x;
  int32_t carry = 0;
  for (int64_t base = 0; base < n; base += 1024) {
    const int32_t v = base + t < n ? cnt[base + t] : 0;
    buf[t] = v;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
      const int32_t add = t >= d ? buf[t - d] : 0;
      __syncthreads();
      buf[t] += add;
      __syncthreads();
    }
    if (base + t < n) off[base + t] = carry + buf[t] - v;
    carry += buf[1023];
    __syncthreads();
  }
  if (t == 0) off[n] = carry;
}

// Neighbour rows: out[off[s] + k] = s with the spins of its k-th antiparallel
// bond exchanged.
__global__ __launch_bounds__(64 * kNbWaves) void nb_write_kernel(const int8_t* __restrict__ spins,
                                                                 int64_t n, int N, int NB,
                                                                 const int32_t* __restrict__ bonds,
                                                                 const int32_t* __restrict__ off,
                                                                 int8_t* __restrict__ out,
                                                                 int16_t* __restrict__ parent) {
  const int64_t s = (int64_t)blockIdx.x * kNbWaves + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (s >= n) return;
  const int8_t* srow = spins + s * N;
  int64_t pos = off[s];
  for (int base = 0; base < NB; base += 64) {
    const int b = base + lane;
    const bool anti = bond_anti(srow, bonds, b, NB);
    const unsigned long long m = __ballot(anti);
    if (anti) {
      const int64_t k = pos + __popcll(m & ((1ull << lane) - 1ull));
      const int i = bonds[2 * b], j = bonds[2 * b + 1];
      int8_t* row = out + k * N;
      for (int x = 0; x < N; ++x) row[x] = srow[x];
      row[i] = srow[j];
      row[j] = srow[i];
      if (parent) parent[k] = (int16_t)b;
    }
    pos += __popcll(m);
  }
}

// out[s] = H_ss eprev[s] + sum_k (J_k/2) exp(lp_nb[k] - lp[s]) enb[k]; the lanes
// take the bonds, the wavefront sum runs in a fixed order.
__global__ __launch_bounds__(64 * kNbWaves) void hop_combine_kernel(
    const int8_t* __restrict__ spins, int64_t n, int N, int NB, const int32_t* __restrict__ bonds,
    const double* __restrict__ bond_J, const int32_t* __restrict__ off,
    const double* __restrict__ lp, const double* __restrict__ eprev, int eprev_stride,
    const double* __restrict__ lp_nb, const double* __restrict__ enb, int enb_stride,
    double* __restrict__ out, int out_stride, int back) {
  const int64_t s = (int64_t)blockIdx.x * kNbWaves + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (s >= n) return;
  const int8_t* srow = spins + s * N;
  const double lr = lp[2 * s], li = lp[2 * s + 1];
  double diag = 0.0, ar = 0.0, ai = 0.0, jj = 0.0;
  int64_t pos = off[s];
  for (int base = 0; base < NB; base += 64) {
    const int b = base + lane;
    bool anti = false;
    if (b < NB) {
      const int si = srow[bonds[2 * b]], sj = srow[bonds[2 * b + 1]];
      diag += 0.25 * bond_J[b] * (double)(si * sj);
      anti = si != sj;
      if (anti) jj += 0.25 * bond_J[b] * bond_J[b];
    }
    const unsigned long long m = __ballot(anti);
    if (anti) {
      const int64_t k = pos + __popcll(m & ((1ull << lane) - 1ull));
      const double mag = 0.5 * bond_J[b] * exp(lp_nb[2 * k] - lr);
      // psi(s^b) = 0 (a configuration fixed by a symmetry whose character
      // forces a zero): the local value there is undefined, but H^p psi
      // lies in the same symmetry sector and vanishes there too
      if (mag != 0.0) {
        double sn, cs;
        sincos(lp_nb[2 * k + 1] - li, &sn, &cs);
        const double fr = enb ? enb[enb_stride * k] : 1.0, fi = enb ? enb[enb_stride * k + 1] : 0.0;
        ar += mag * (cs * fr - sn * fi);
        ai += mag * (cs * fi + sn * fr);
      }
    }
    pos += __popcll(m);
  }
  diag = wave_sum(diag);
  ar = wave_sum(ar);
  ai = wave_sum(ai);
  jj = back ? wave_sum(jj) : 0.0;
  if (lane == 0) {
    out[out_stride * s] = diag * eprev[eprev_stride * s] + ar + jj;
    out[out_stride * s + 1] = diag * eprev[eprev_stride * s + 1] + ai;
  }
}

// Path sums from the E_loc kernels' partials [S][G/16][6] = (m, den, Q, -):
// log(e^M sum_blocks e^{m - M} (H_ss den + Q)), i.e. log of
// sum_g chi_g psi_s(g s) (H_ss + sum_b (J_b/2) R_gb) without the division by
// psi(s) that E_loc makes (finite where psi(s) vanishes).
__global__ __launch_bounds__(64) void pathsum_finish_kernel(
    const int8_t* __restrict__ spins, int N, int NB, int cbs, const int32_t* __restrict__ bonds,
    const double* __restrict__ bond_J, const double* __restrict__ part, double* __restrict__ out) {
  const int64_t s = blockIdx.x;
  const int lane = threadIdx.x;
  const int8_t* srow = spins + s * N;
  double d = 0.0;
  for (int b = lane; b < NB; b += 64)
    d += 0.25 * bond_J[b] * (double)(srow[bonds[2 * b]] * srow[bonds[2 * b + 1]]);
  d = wave_sum(d);
  const double* ps = part + (size_t)s * cbs * 6;
  double mx = -INFINITY;
  for (int i = lane; i < cbs; i += 64) mx = fmax(mx, ps[6 * i]);
  mx = wave_max(mx);
  double ar = 0.0, ai = 0.0;
  for (int i = lane; i < cbs; i += 64) {
    const double e = exp(ps[6 * i] - mx);
    ar += e * (d * ps[6 * i + 1] + ps[6 * i + 3]);
    ai += e * (d * ps[6 * i + 2] + ps[6 * i + 4]);
  }
  ar = wave_sum(ar);
  ai = wave_sum(ai);
  if (lane == 0) {
    out[2 * s] = mx + 0.5 * log(ar * ar + ai * ai);
    out[2 * s + 1] = atan2(ai, ar);
  }
}

// Lowest eigenpair of a symmetric 3x3 matrix by cyclic Jacobi rotations
// (each rotation zeroes one off-diagonal element; the sweeps converge
// quadratically).  a is destroyed; y receives the unit eigenvector.
__device__ double sym3_lowest(double a[3][3], double y[3]) {
  double V[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
  for (int sweep = 0; sweep < 32; ++sweep) {
    const double offd = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    const double dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (offd == 0.0 || offd <= 1e-34 * dia) break;
    for (int p = 0; p < 2; ++p) {
      for (int q = p + 1; q < 3; ++q) {
        const double apq = a[p][q];
        if (apq == 0.0) continue;
        // tan of the rotation angle: the smaller root of t^2 + 2 th t - 1 = 0
        const double th = (a[q][q] - a[p][p]) / (2.0 * apq);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < 3; ++k) {
          const double kp = a[k][p], kq = a[k][q];
          a[k][p] = c * kp - sn * kq;
          a[k][q] = sn * kp + c * kq;
        }
        for (int k = 0; k < 3; ++k) {
          const double pk = a[p][k], qk = a[q][k];
          a[p][k] = c * pk - sn * qk;
          a[q][k] = sn * pk + c * qk;
        }
        for (int k = 0; k < 3; ++k) {
          const double kp = V[k][p], kq = V[k][q];
          V[k][p] = c * kp - sn * kq;
          V[k][q] = sn * kp + c * kq;
        }
      }
    }
  }
  int lo = 0;
  if (a[1][1] < a[lo][lo]) lo = 1;
  if (a[2][2] < a[lo][lo]) lo = 2;
  for (int k = 0; k < 3; ++k) y[k] = V[k][lo];
  return a[lo][lo];
}

// result[0..13] as written by the p = 1 moments kernel; appends
// result[16..23] = h4 h5 mu4 mu5 e_p2 beta1 beta2 degenerate.
__global__ __launch_bounds__(1024) void moments2_kernel(const double* __restrict__ e1e2,
                                                        const double* __restrict__ e3,
                                                        const double* __restrict__ logpsi,
                                                        int64_t S, int exact,
                                                        double* __restrict__ result) {
  __shared__ double red[16][8];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double mx = -INFINITY;
  if (exact)
    for (int64_t i = tid; i < S; i += 1024) mx = fmax(mx, logpsi[2 * i]);
  mx = wave_max(mx);
  if (lane == 0) red[wv][0] = mx;
  __syncthreads();
  mx = red[0][0];
  for (int q = 1; q < 16; ++q) mx = fmax(mx, red[q][0]);
  __syncthreads();
  const double h1 = result[0];
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};   // sum p, h4, h5, mu4, mu5
  for (int64_t i = tid; i < S; i += 1024) {
    double p = 1.0;
    if (exact) {
      p = exp(2.0 * (logpsi[2 * i] - mx));
      if (p < 1e-300) continue;                 // psi = 0 carries no weight
    }
    const double er = e1e2[4 * i], ei = e1e2[4 * i + 1];
    const double fr = e1e2[4 * i + 2], fi = e1e2[4 * i + 3];
    const double gr = e3[2 * i], gi = e3[2 * i + 1];
    // d2 = e2 - 2 h1 e1 + h1^2, d3 = e3 - 3 h1 e2 + 3 h1^2 e1 - h1^3
    const double d2r = fr - 2.0 * h1 * er + h1 * h1, d2i = fi - 2.0 * h1 * ei;
    const double d3r = gr - 3.0 * h1 * fr + 3.0 * h1 * h1 * er - h1 * h1 * h1;
    const double d3i = gi - 3.0 * h1 * fi + 3.0 * h1 * h1 * ei;
    v[0] += p;
    v[1] += p * (fr * fr + fi * fi);
    v[2] += p * (fr * gr + fi * gi);
    v[3] += p * (d2r * d2r + d2i * d2i);
    v[4] += p * (d2r * d3r + d2i * d3i);
  }
  for (int j = 0; j < 5; ++j) {
    const double x = wave_sum(v[j]);
    if (lane == 0) red[wv][j] = x;
  }
  __syncthreads();
  if (tid != 0) return;
  for (int j = 0; j < 5; ++j) {
    double x = 0.0;
    for (int q = 0; q < 16; ++q) x += red[q][j];
    v[j] = x;
  }
  const double sw = v[0];
  const double h4 = v[1] / sw, h5 = v[2] / sw, mu4 = v[3] / sw, mu5 = v[4] / sw;
  const double vv = result[7], r = result[8], alpha = result[9], ep1 = result[10];
  double ep2 = ep1, b1 = 0.0, b2 = 0.0, degen = 1.0;
  if (result[12] == 0.0) {
    b1 = (alpha / vv) / (1.0 - alpha * h1 / vv);
    const double m4 = mu4 / (vv * vv * vv * vv), m5 = mu5 / (vv * vv * vv * vv * vv);
    const double delta = m4 - r * r - 1.0;
    if (delta > 64.0 * 1.1102230246251565e-16 * fmax(m4, 1.0)) {
      // B = L L^T with L = [[1,0,0],[0,1,0],[1,r,sd]]; C = L^-1 A L^-T
      const double sd = sqrt(delta);
      const double A[3][3] = {{0.0, 1.0, r}, {1.0, r, m4}, {r, m4, m5}};
      const double Li[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {-1.0 / sd, -r / sd, 1.0 / sd}};
      double M[3][3], C[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double x = 0.0;
          for (int k = 0; k < 3; ++k) x += Li[i][k] * A[k][j];
          M[i][j] = x;
        }
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double x = 0.0;
          for (int k = 0; k < 3; ++k) x += M[i][k] * Li[j][k];
          C[i][j] = x;
        }
      for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j) C[i][j] = C[j][i] = 0.5 * (C[i][j] + C[j][i]);
      double y[3];
      const double lam = sym3_lowest(C, y);
      // x = L^-T y: coefficients of K^0, K^1, K^2 with K = (H - h1)/v
      const double x2 = y[2] / sd, x1 = y[1] - r * x2, x0 = y[0] - x2;
      const double c0 = x0 - x1 * h1 / vv + x2 * h1 * h1 / (vv * vv);
      const double c1 = x1 / vv - 2.0 * x2 * h1 / (vv * vv);
      const double c2 = x2 / (vv * vv);
      ep2 = h1 + vv * lam;
      b1 = c1 / c0;
      b2 = c2 / c0;
      degen = 0.0;
    }
  }
  const double out[8] = {h4, h5, mu4, mu5, ep2, b1, b2, degen};
  for (int j = 0; j < 8; ++j) result[16 + j] = out[j];
}

unsigned nb_blocks(int64_t n) { return (unsigned)((n + kNbWaves - 1) / kNbWaves); }

}  // namespace

hipError_t launch_nb_count(const nqs_ctx* c, const int8_t* spins, int64_t n, int32_t* cnt,
                           hipStream_t st) {
  if (n <= 0) return hipSuccess;
  nb_count_kernel<<<nb_blocks(n), 64 * kNbWaves, 0, st>>>(spins, n, c->N, c->NB, c->dev.bonds, cnt);
  return hipGetLastError();
}

hipError_t launch_nb_scan(const int32_t* cnt, int64_t n, int32_t* off, hipStream_t st) {
  nb_scan_kernel<<<1, 1024, 0, st>>>(cnt, n, off);
  return hipGetLastError();
}

hipError_t launch_nb_write(const nqs_ctx* c, const int8_t* spins, int64_t n, const int32_t* off,
                           int8_t* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  nb_write_kernel<<<nb_blocks(n), 64 * kNbWaves, 0, st>>>(spins, n, c->N, c->NB, c->dev.bonds, off,
                                                          out, nullptr);
  return hipGetLastError();
}

hipError_t launch_nb_write_parent(const nqs_ctx* c, const int8_t* spins, int64_t n,
                                  const int32_t* off, int8_t* out, int16_t* parent,
                                  hipStream_t st) {
  if (n <= 0) return hipSuccess;
  nb_write_kernel<<<nb_blocks(n), 64 * kNbWaves, 0, st>>>(spins, n, c->N, c->NB, c->dev.bonds, off,
                                                          out, parent);
  return hipGetLastError();
}

hipError_t launch_pathsum_finish(const nqs_ctx* c, const int8_t* spins, int64_t S,
                                 const double* part, double* out, hipStream_t st) {
  if (S <= 0) return hipSuccess;
  pathsum_finish_kernel<<<(unsigned)S, 64, 0, st>>>(spins, c->N, c->NB, c->G / 16, c->dev.bonds,
                                                    c->dev.bond_J, part, out);
  return hipGetLastError();
}

hipError_t launch_hop_combine(const nqs_ctx* c, const int8_t* spins, int64_t n, const int32_t* off,
                              const double* lp, const double* eprev, int eprev_stride,
                              const double* lp_nb, const double* enb, int enb_stride, double* out,
                              int out_stride, hipStream_t st, int back) {
  if (n <= 0) return hipSuccess;
  hop_combine_kernel<<<nb_blocks(n), 64 * kNbWaves, 0, st>>>(
      spins, n, c->N, c->NB, c->dev.bonds, c->dev.bond_J, off, lp, eprev, eprev_stride, lp_nb, enb,
      enb_stride, out, out_stride, back);
  return hipGetLastError();
}

hipError_t launch_e3_combine(const nqs_ctx* c, const int8_t* spins, int64_t n, const int32_t* off,
                             const double* lp, const double* e1e2, const double* lp_nb,
                             const double* e1e2_nb, double* e3, hipStream_t st) {
  return launch_hop_combine(c, spins, n, off, lp, e1e2 + 2, 4, lp_nb, e1e2_nb + 2, 4, e3, 2, st);
}

hipError_t launch_moments2(const double* e1e2, const double* e3, const double* logpsi, int64_t S,
                           int exact, double* result, hipStream_t st) {
  moments2_kernel<<<1, 1024, 0, st>>>(e1e2, e3, logpsi, S, exact, result);
  return hipGetLastError();
}

}  // namespace nqs
