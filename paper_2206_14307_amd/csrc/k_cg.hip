// Stochastic-reconfiguration step of Eq. (12) solved in parameter space by
// conjugate gradients (Sec. 3.4: the paper solves the system with CG and a
// ridge lambda), matrix-free:
//   A v = O_bar^H (O_bar v) + lambda v,   O_bar = (O - <O>) / sqrt(S),
//   b   = -dtau O_bar^H eps,              eps   = (E_loc - <E>) / sqrt(S),
// without forming O_bar or the P x P matrix.  Centring is applied on the fly:
//   O_bar v   = (O v - (m . v)) / sqrt(S)            (m = <O>, a row vector)
//   O_bar^H u = (O^H u - conj(m) sum_s u_s) / sqrt(S).
// Per iteration two passes over O (HBM-bound for S x P beyond the caches):
//   rows: u_s = sum_k O_sk p_k, a block takes kCgRows rows and one of
//         kRowParts column parts and reuses each loaded p_k for all its
//         rows; the part sums are added in a fixed order;
//   cols: q_k = sum_s conj(O_sk) u_s, a block takes 256 columns and one slab
//         of rows; slab partials are added in a fixed order.
// The CG scalars stay on the device (single-block FP64 kernels).  Iterations
// are queued kCgBatch at a time: a device-side flag set when the residual
// test passes makes the rest of the batch return at once, and the host reads
// the residual once per batch (same iterates and count as a test after every
// iteration).  All sums in FP64.
#include <algorithm>
#include <cmath>

#include "device_common.h"
#include "nqs_internal.h"

namespace nqs {

namespace {

constexpr int kCgRows = 16;      // rows per block of the row GEMV
constexpr int kRowParts = 8;     // most column parts of the complex64 row GEMV
constexpr int kCgThreads = 256;
constexpr int kVecThreads = 1024;
constexpr int kCgBatch = 4;      // CG iterations queued per read of the residual

struct cd {
  double x, y;
};
__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Streaming 16-byte load of O: each pass reads O once, so its lines are
// marked non-temporal and do not displace the reused vectors from the caches
// (a plain streaming read of a 10.6 GB buffer measured 6.6 TB/s this way
// against 6.0 TB/s with ordinary loads).
__device__ __forceinline__ float4 stream_load4(const float* p) {
  const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}

// The kernels of a CG iteration return at once once the solve has stopped
// (stop = the flag cg_step_kernel sets; null outside the iteration), so the
// host can queue several iterations per read of the residual.
__device__ __forceinline__ bool stopped(const double* stop) { return stop != nullptr && *stop != 0.0; }

template <typename RO>
__device__ __forceinline__ cd load_c(const RO* p, size_t i) {
  return {(double)p[2 * i], (double)p[2 * i + 1]};
}

// u[s] = sum_k O[s][k] v[k] for kCgRows rows per block; then
// u[s] = (u[s] - mv) / sqrt(S) with mv = m . v (scal[0..1]) when centre != 0.
template <typename RO>
__global__ __launch_bounds__(kCgThreads) void rows_kernel(const RO* __restrict__ O, int64_t S,
                                                          int64_t P, const double* __restrict__ v,
                                                          const double* __restrict__ mv,
                                                          double inv_sqrt_s,
                                                          double* __restrict__ u,
                                                          const double* __restrict__ stop) {
  if (stopped(stop)) return;
  __shared__ double red[kCgRows][2][kCgThreads / 64];
  const int64_t s0 = (int64_t)blockIdx.x * kCgRows;
  double ar[kCgRows], ai[kCgRows];
#pragma unroll
  for (int r = 0; r < kCgRows; ++r) ar[r] = ai[r] = 0.0;
  for (int64_t k = threadIdx.x; k < P; k += kCgThreads) {
    const double vr = v[2 * k], vi = v[2 * k + 1];
#pragma unroll
    for (int r = 0; r < kCgRows; ++r) {
      if (s0 + r < S) {
        const cd o = load_c(O, (size_t)(s0 + r) * P + k);
        ar[r] = fma(o.x, vr, fma(-o.y, vi, ar[r]));
        ai[r] = fma(o.x, vi, fma(o.y, vr, ai[r]));
      }
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < kCgRows; ++r) {
    const double sr = wave_sum(ar[r]), si = wave_sum(ai[r]);
    if (lane == 0) {
      red[r][0][wv] = sr;
      red[r][1][wv] = si;
    }
  }
  __syncthreads();
  if (threadIdx.x < kCgRows && s0 + threadIdx.x < S) {
    const int r = threadIdx.x;
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int w = 0; w < kCgThreads / 64; ++w) {
      sr += red[r][0][w];
      si += red[r][1][w];
    }
    u[2 * (s0 + r)] = (sr - mv[0]) * inv_sqrt_s;
    u[2 * (s0 + r) + 1] = (si - mv[1]) * inv_sqrt_s;
  }
}

// part[slab][k] = sum_{s in slab} conj(O[s][k]) u[s]  (u = NULL: u = 1).
template <typename RO>
__global__ __launch_bounds__(kCgThreads) void cols_kernel(const RO* __restrict__ O, int64_t S,
                                                          int64_t P, int64_t slab,
                                                          const double* __restrict__ u,
                                                          double* __restrict__ part,
                                                          const double* __restrict__ stop) {
  if (stopped(stop)) return;
  const int64_t k = (int64_t)blockIdx.x * kCgThreads + threadIdx.x;
  const int64_t sb = (int64_t)blockIdx.y * slab, se = std::min<int64_t>(S, sb + slab);
  if (k >= P) return;
  double qr = 0.0, qi = 0.0;
  for (int64_t s = sb; s < se; ++s) {
    const cd o = load_c(O, (size_t)s * P + k);
    const double ur = u ? u[2 * s] : 1.0, ui = u ? u[2 * s + 1] : 0.0;
    qr = fma(o.x, ur, fma(o.y, ui, qr));      // conj(o) u
    qi = fma(o.x, ui, fma(-o.y, ur, qi));
  }
  part[2 * ((size_t)blockIdx.y * P + k)] = qr;
  part[2 * ((size_t)blockIdx.y * P + k) + 1] = qi;
}

// complex64 O: every P here is even (N even, M a multiple of 8), so a row's
// column pairs are 16-byte aligned and one float4 load brings two columns.
// Block (x, y) takes rows x kCgRows .. and column part y of gridDim.y (at
// most kRowParts) and writes its raw partial sums upart[y][s]: many more
// blocks than the device holds at once, so the last round of blocks is a
// small part of the pass.
__global__ __launch_bounds__(kCgThreads) void rows2_kernel(const float* __restrict__ O, int64_t S,
                                                           int64_t P, const double* __restrict__ v,
                                                           double* __restrict__ upart,
                                                           const double* __restrict__ stop) {
  if (stopped(stop)) return;
  __shared__ double red[kCgRows][2][kCgThreads / 64];
  const int64_t s0 = (int64_t)blockIdx.x * kCgRows;
  const int64_t P2 = P / 2;
  const int64_t span = (P2 + gridDim.y - 1) / gridDim.y;
  const int64_t kb = (int64_t)blockIdx.y * span, ke = std::min<int64_t>(P2, kb + span);
  double ar[kCgRows], ai[kCgRows];
#pragma unroll
  for (int r = 0; r < kCgRows; ++r) ar[r] = ai[r] = 0.0;
  for (int64_t k2 = kb + threadIdx.x; k2 < ke; k2 += kCgThreads) {
    const double4 vv = reinterpret_cast<const double4*>(v)[k2];
#pragma unroll
    for (int r = 0; r < kCgRows; ++r) {
      if (s0 + r < S) {
        const float4 o = stream_load4(O + (size_t)(s0 + r) * P * 2 + 4 * k2);
        ar[r] = fma((double)o.x, vv.x, fma(-(double)o.y, vv.y, ar[r]));
        ai[r] = fma((double)o.x, vv.y, fma((double)o.y, vv.x, ai[r]));
        ar[r] = fma((double)o.z, vv.z, fma(-(double)o.w, vv.w, ar[r]));
        ai[r] = fma((double)o.z, vv.w, fma((double)o.w, vv.z, ai[r]));
      }
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < kCgRows; ++r) {
    const double sr = wave_sum(ar[r]), si = wave_sum(ai[r]);
    if (lane == 0) {
      red[r][0][wv] = sr;
      red[r][1][wv] = si;
    }
  }
  __syncthreads();
  if (threadIdx.x < kCgRows && s0 + threadIdx.x < S) {
    const int r = threadIdx.x;
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int w = 0; w < kCgThreads / 64; ++w) {
      sr += red[r][0][w];
      si += red[r][1][w];
    }
    double* dst = upart + 2 * ((size_t)blockIdx.y * S + s0 + r);
    dst[0] = sr;
    dst[1] = si;
  }
}

// u[s] = (sum over the column parts in a fixed order - m . v) / sqrt(S)
__global__ __launch_bounds__(kCgThreads) void rows2_finish_kernel(const double* __restrict__ upart,
                                                                  int parts, int64_t S,
                                                                  const double* __restrict__ mv,
                                                                  double inv_sqrt_s,
                                                                  double* __restrict__ u,
                                                                  const double* __restrict__ stop) {
  if (stopped(stop)) return;
  const int64_t s = (int64_t)blockIdx.x * kCgThreads + threadIdx.x;
  if (s >= S) return;
  double sr = 0.0, si = 0.0;
  for (int y = 0; y < parts; ++y) {
    sr += upart[2 * ((size_t)y * S + s)];
    si += upart[2 * ((size_t)y * S + s) + 1];
  }
  u[2 * s] = (sr - mv[0]) * inv_sqrt_s;
  u[2 * s + 1] = (si - mv[1]) * inv_sqrt_s;
}

// part[slab][k] for the column pair (2 k2, 2 k2 + 1); rows of the slab four at
// a time (independent loads in flight).
__global__ __launch_bounds__(kCgThreads) void cols2_kernel(const float* __restrict__ O, int64_t S,
                                                           int64_t P, int64_t slab,
                                                           const double* __restrict__ u,
                                                           double* __restrict__ part,
                                                           const double* __restrict__ stop) {
  if (stopped(stop)) return;
  const int64_t k2 = (int64_t)blockIdx.x * kCgThreads + threadIdx.x;
  const int64_t sb = (int64_t)blockIdx.y * slab, se = std::min<int64_t>(S, sb + slab);
  if (k2 >= P / 2) return;
  double q0r = 0.0, q0i = 0.0, q1r = 0.0, q1i = 0.0;
  int64_t s = sb;
  for (; s + 4 <= se; s += 4) {
    float4 o[4];
    double2 uu[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      o[j] = stream_load4(O + (size_t)(s + j) * P * 2 + 4 * k2);
      uu[j] = u ? reinterpret_cast<const double2*>(u)[s + j] : make_double2(1.0, 0.0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      q0r = fma((double)o[j].x, uu[j].x, fma((double)o[j].y, uu[j].y, q0r));
      q0i = fma((double)o[j].x, uu[j].y, fma(-(double)o[j].y, uu[j].x, q0i));
      q1r = fma((double)o[j].z, uu[j].x, fma((double)o[j].w, uu[j].y, q1r));
      q1i = fma((double)o[j].z, uu[j].y, fma(-(double)o[j].w, uu[j].x, q1i));
    }
  }
  for (; s < se; ++s) {
    const float4 o = stream_load4(O + (size_t)s * P * 2 + 4 * k2);
    const double2 uu = u ? reinterpret_cast<const double2*>(u)[s] : make_double2(1.0, 0.0);
    q0r = fma((double)o.x, uu.x, fma((double)o.y, uu.y, q0r));
    q0i = fma((double)o.x, uu.y, fma(-(double)o.y, uu.x, q0i));
    q1r = fma((double)o.z, uu.x, fma((double)o.w, uu.y, q1r));
    q1i = fma((double)o.z, uu.y, fma(-(double)o.w, uu.x, q1i));
  }
  double* dst = part + 2 * ((size_t)blockIdx.y * P + 2 * k2);
  dst[0] = q0r;
  dst[1] = q0i;
  dst[2] = q1r;
  dst[3] = q1i;
}

// Fixed-order block-wide sum (kVecThreads threads, one block).
__device__ double vsum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int h = kVecThreads / 2; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Column sums over the slabs: out[k] = sum_slab part[slab][k], then one of
//   mode 0: out = conj(part-sum) / S   (the mean m, from the u = 1 pass)
//   mode 1: out = (part-sum - conj(m) usum) / sqrt(S) * a + lambda * p (A p)
// where usum = scal[2..3] = sum_s u_s and a = 1; b is mode 1 with lambda = 0
// and a = -dtau.
__global__ __launch_bounds__(kCgThreads) void slab_sum_kernel(
    const double* __restrict__ part, int nslab, int64_t P, int mode, double S_or_invsqrt,
    const double* __restrict__ m, const double* __restrict__ usum, double scale, double lambda,
    const double* __restrict__ p, double* __restrict__ out, const double* __restrict__ stop) {
  if (stopped(stop)) return;
  const int64_t k = (int64_t)blockIdx.x * kCgThreads + threadIdx.x;
  if (k >= P) return;
  double qr = 0.0, qi = 0.0;
  for (int j = 0; j < nslab; ++j) {
    qr += part[2 * ((size_t)j * P + k)];
    qi += part[2 * ((size_t)j * P + k) + 1];
  }
  if (mode == 0) {                          // the column kernel conjugates O
    out[2 * k] = qr / S_or_invsqrt;
    out[2 * k + 1] = -qi / S_or_invsqrt;
    return;
  }
  // conj(m_k) * usum
  const double cr = m[2 * k] * usum[0] + m[2 * k + 1] * usum[1];
  const double ci = m[2 * k] * usum[1] - m[2 * k + 1] * usum[0];
  double rr = (qr - cr) * S_or_invsqrt * scale, ri = (qi - ci) * S_or_invsqrt * scale;
  if (p) {
    rr = fma(lambda, p[2 * k], rr);
    ri = fma(lambda, p[2 * k + 1], ri);
  }
  out[2 * k] = rr;
  out[2 * k + 1] = ri;
}

// eps = (E - <E>) / sqrt(S); scal[2..3] = sum_s eps_s (zero up to rounding).
__global__ __launch_bounds__(kVecThreads) void eps_kernel(const double* __restrict__ e, int64_t S,
                                                          double* __restrict__ eps,
                                                          double* __restrict__ scal) {
  __shared__ double red[kVecThreads];
  double sr = 0.0, si = 0.0;
  for (int64_t i = threadIdx.x; i < S; i += kVecThreads) {
    sr += e[2 * i];
    si += e[2 * i + 1];
  }
  const double mr = vsum(sr, red) / (double)S, mi = vsum(si, red) / (double)S;
  const double is = 1.0 / sqrt((double)S);
  double tr = 0.0, ti = 0.0;
  for (int64_t i = threadIdx.x; i < S; i += kVecThreads) {
    const double a = (e[2 * i] - mr) * is, b = (e[2 * i + 1] - mi) * is;
    eps[2 * i] = a;
    eps[2 * i + 1] = b;
    tr += a;
    ti += b;
  }
  tr = vsum(tr, red);
  ti = vsum(ti, red);
  if (threadIdx.x == 0) {
    scal[2] = tr;
    scal[3] = ti;
  }
}

// scal[0..1] = m . v (no conjugation) and scal[2..3] stays; sum of u set by
// usum_kernel.
__global__ __launch_bounds__(kVecThreads) void mdot_kernel(const double* __restrict__ m,
                                                           const double* __restrict__ v, int64_t P,
                                                           double* __restrict__ scal,
                                                           const double* __restrict__ stop) {
  if (stopped(stop)) return;
  __shared__ double red[kVecThreads];
  double sr = 0.0, si = 0.0;
  for (int64_t k = threadIdx.x; k < P; k += kVecThreads) {
    const cd a = {m[2 * k], m[2 * k + 1]}, b = {v[2 * k], v[2 * k + 1]};
    const cd c = cmul(a, b);
    sr += c.x;
    si += c.y;
  }
  sr = vsum(sr, red);
  si = vsum(si, red);
  if (threadIdx.x == 0) {
    scal[0] = sr;
    scal[1] = si;
  }
}

// scal[2..3] = sum_s u_s.
__global__ __launch_bounds__(kVecThreads) void usum_kernel(const double* __restrict__ u, int64_t S,
                                                           double* __restrict__ scal,
                                                           const double* __restrict__ stop) {
  if (stopped(stop)) return;
  __shared__ double red[kVecThreads];
  double sr = 0.0, si = 0.0;
  for (int64_t i = threadIdx.x; i < S; i += kVecThreads) {
    sr += u[2 * i];
    si += u[2 * i + 1];
  }
  sr = vsum(sr, red);
  si = vsum(si, red);
  if (threadIdx.x == 0) {
    scal[2] = sr;
    scal[3] = si;
  }
}

// CG start: x = 0, r = p = b; cg[0] = r^H r, cg[1] = b^H b.
__global__ __launch_bounds__(kVecThreads) void cg_init_kernel(const double* __restrict__ b,
                                                              int64_t P, double* __restrict__ x,
                                                              double* __restrict__ r,
                                                              double* __restrict__ p,
                                                              double* __restrict__ cg) {
  __shared__ double red[kVecThreads];
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < P; k += kVecThreads) {
    const double br = b[2 * k], bi = b[2 * k + 1];
    x[2 * k] = x[2 * k + 1] = 0.0;
    r[2 * k] = p[2 * k] = br;
    r[2 * k + 1] = p[2 * k + 1] = bi;
    s = fma(br, br, fma(bi, bi, s));
  }
  s = vsum(s, red);
  if (threadIdx.x == 0) {
    cg[0] = s;
    cg[1] = s;
    cg[2] = 0.0;
    cg[3] = 0.0;
    cg[4] = 0.0;
  }
}

// One CG update given q = A p: alpha = rr / (p^H q), x += alpha p,
// r -= alpha q, beta = rr' / rr, p = r + beta p.  cg[0] = rr', cg[2] = 1
// if p^H q <= 0 (A not positive definite along p); cg[4] counts the
// iterations and cg[3] = 1 stops the solve (not positive definite, or
// rr' <= thr2 = tol^2 b^H b).
__global__ __launch_bounds__(kVecThreads) void cg_step_kernel(double* __restrict__ x,
                                                              double* __restrict__ r,
                                                              double* __restrict__ p,
                                                              const double* __restrict__ q,
                                                              int64_t P, double* __restrict__ cg,
                                                              double thr2) {
  if (cg[3] != 0.0) return;
  __shared__ double red[kVecThreads];
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < P; k += kVecThreads)
    s = fma(p[2 * k], q[2 * k], fma(p[2 * k + 1], q[2 * k + 1], s));   // Re p^H q
  const double pq = vsum(s, red);
  const double rr = cg[0];
  if (!(pq > 0.0)) {
    if (threadIdx.x == 0) {
      cg[2] = 1.0;
      cg[3] = 1.0;
      cg[4] += 1.0;
    }
    return;
  }
  const double alpha = rr / pq;
  double t = 0.0;
  for (int64_t k = threadIdx.x; k < P; k += kVecThreads) {
    x[2 * k] = fma(alpha, p[2 * k], x[2 * k]);
    x[2 * k + 1] = fma(alpha, p[2 * k + 1], x[2 * k + 1]);
    const double nr = fma(-alpha, q[2 * k], r[2 * k]);
    const double ni = fma(-alpha, q[2 * k + 1], r[2 * k + 1]);
    r[2 * k] = nr;
    r[2 * k + 1] = ni;
    t = fma(nr, nr, fma(ni, ni, t));
  }
  const double rr2 = vsum(t, red);
  const double beta = rr2 / rr;
  for (int64_t k = threadIdx.x; k < P; k += kVecThreads) {
    p[2 * k] = fma(beta, p[2 * k], r[2 * k]);
    p[2 * k + 1] = fma(beta, p[2 * k + 1], r[2 * k + 1]);
  }
  if (threadIdx.x == 0) {
    cg[0] = rr2;
    cg[4] += 1.0;
    if (!(rr2 > thr2)) cg[3] = 1.0;
  }
}

struct CgLayout {
  int64_t nslab, slab;
  size_t m, eps, u, b, r, p, q, part, upart, scal, cg, bytes;
};

CgLayout cg_layout(const nqs_ctx* c, int64_t S) {
  CgLayout L;
  const int64_t P = c->P;
  // column blocks of the pass that runs (pairs of columns per thread for
  // complex64 O), then enough slabs for about 8 blocks per CU: a streaming
  // pass needs many loads in flight; slabs of >= 64 rows
  const int64_t ctiles = ((P % 2 == 0 ? P / 2 : P) + kCgThreads - 1) / kCgThreads;
  const int64_t want = std::max<int64_t>(1, 8 * 256 / ctiles);
  L.nslab = std::max<int64_t>(1, std::min<int64_t>(want, (S + 63) / 64));
  L.slab = (S + L.nslab - 1) / L.nslab;
  auto al = [](size_t v) { return (v + 255) / 256 * 256; };
  size_t off = 0;
  L.m = off; off += al((size_t)P * 16);
  L.eps = off; off += al((size_t)S * 16);
  L.u = off; off += al((size_t)S * 16);
  L.b = off; off += al((size_t)P * 16);
  L.r = off; off += al((size_t)P * 16);
  L.p = off; off += al((size_t)P * 16);
  L.q = off; off += al((size_t)P * 16);
  L.part = off; off += al((size_t)L.nslab * P * 16);
  L.upart = off; off += al((size_t)kRowParts * S * 16);
  L.scal = off; off += al(8 * 8);
  L.cg = off; off += al(8 * 8);
  L.bytes = off;
  return L;
}

template <typename RO>
hipError_t cols_to(const RO* O, int64_t S, int64_t P, const CgLayout& L, const double* u,
                   double* part, const double* stop, hipStream_t st) {
  if constexpr (sizeof(RO) == 4) {
    const dim3 grid((unsigned)((P / 2 + kCgThreads - 1) / kCgThreads), (unsigned)L.nslab);
    cols2_kernel<<<grid, kCgThreads, 0, st>>>(O, S, P, L.slab, u, part, stop);
  } else {
    const dim3 grid((unsigned)((P + kCgThreads - 1) / kCgThreads), (unsigned)L.nslab);
    cols_kernel<RO><<<grid, kCgThreads, 0, st>>>(O, S, P, L.slab, u, part, stop);
  }
  return hipGetLastError();
}

template <typename RO>
hipError_t cg_run(nqs_ctx* c, const RO* O, const double* eloc, int64_t S, double lambda,
                  double dtau, double tol, int max_iter, double* x, char* ws, int* iters,
                  double* resid, int* not_pd, hipStream_t st) {
  const int64_t P = c->P;
  const CgLayout L = cg_layout(c, S);
  double* m = (double*)(ws + L.m);
  double* eps = (double*)(ws + L.eps);
  double* u = (double*)(ws + L.u);
  double* b = (double*)(ws + L.b);
  double* r = (double*)(ws + L.r);
  double* p = (double*)(ws + L.p);
  double* q = (double*)(ws + L.q);
  double* part = (double*)(ws + L.part);
  double* upart = (double*)(ws + L.upart);
  double* scal = (double*)(ws + L.scal);
  double* cg = (double*)(ws + L.cg);
  const unsigned ptiles = (unsigned)((P + kCgThreads - 1) / kCgThreads);
  const double is = 1.0 / std::sqrt((double)S);
  hipError_t e;
  // mean m = <O>
  if ((e = cols_to(O, S, P, L, nullptr, part, nullptr, st)) != hipSuccess) return e;
  slab_sum_kernel<<<ptiles, kCgThreads, 0, st>>>(part, (int)L.nslab, P, 0, (double)S, nullptr,
                                                 nullptr, 1.0, 0.0, nullptr, m, nullptr);
  // eps and b = -dtau O_bar^H eps
  eps_kernel<<<1, kVecThreads, 0, st>>>(eloc, S, eps, scal);
  if ((e = cols_to(O, S, P, L, eps, part, nullptr, st)) != hipSuccess) return e;
  slab_sum_kernel<<<ptiles, kCgThreads, 0, st>>>(part, (int)L.nslab, P, 1, is, m, scal + 2, -dtau,
                                                 0.0, nullptr, b, nullptr);
  cg_init_kernel<<<1, kVecThreads, 0, st>>>(b, P, x, r, p, cg);
  double h[5];
  if ((e = hipMemcpyAsync(h, cg, 40, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  const double bb = h[1];
  const double thr2 = tol * tol * bb;
  // iterations are queued kCgBatch at a time; those after the stop return at
  // once, so the iterates and the count equal a check after every iteration
  int issued = 0;
  if (bb > 0.0 && h[0] > thr2) {
    const double* stop = cg + 3;
    while (issued < max_iter) {
      const int nb = std::min(kCgBatch, max_iter - issued);
      for (int j = 0; j < nb; ++j) {
        // q = A p
        mdot_kernel<<<1, kVecThreads, 0, st>>>(m, p, P, scal, stop);
        if constexpr (sizeof(RO) == 4) {
          // column parts of at least four sweeps of the block over column pairs
          const int parts = (int)std::max<int64_t>(
              1, std::min<int64_t>(kRowParts, P / 2 / (4 * kCgThreads)));
          const dim3 rgrid((unsigned)((S + kCgRows - 1) / kCgRows), (unsigned)parts);
          rows2_kernel<<<rgrid, kCgThreads, 0, st>>>(O, S, P, p, upart, stop);
          rows2_finish_kernel<<<(unsigned)((S + kCgThreads - 1) / kCgThreads), kCgThreads, 0,
                                st>>>(upart, parts, S, scal, is, u, stop);
        } else {
          rows_kernel<RO><<<(unsigned)((S + kCgRows - 1) / kCgRows), kCgThreads, 0, st>>>(
              O, S, P, p, scal, is, u, stop);
        }
        usum_kernel<<<1, kVecThreads, 0, st>>>(u, S, scal, stop);
        if ((e = cols_to(O, S, P, L, u, part, stop, st)) != hipSuccess) return e;
        slab_sum_kernel<<<ptiles, kCgThreads, 0, st>>>(part, (int)L.nslab, P, 1, is, m, scal + 2,
                                                       1.0, lambda, p, q, stop);
        cg_step_kernel<<<1, kVecThreads, 0, st>>>(x, r, p, q, P, cg, thr2);
      }
      issued += nb;
      if ((e = hipGetLastError()) != hipSuccess) return e;
      if ((e = hipMemcpyAsync(h, cg, 40, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
      if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
      if (h[3] != 0.0) break;
    }
  }
  const int it = (int)h[4];
  if (h[2] != 0.0) *not_pd = 1;
  const double rr = h[0];
  *iters = it;
  *resid = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
  return hipSuccess;
}

}  // namespace

size_t cg_workspace_bytes(const nqs_ctx* c, int64_t S) {
  return cg_layout(c, std::max<int64_t>(S, 1)).bytes;
}

extern "C" nqs_status nqs_sr_solve_cg(nqs_ctx* c, const void* O, const double* eloc, int64_t S,
                                      double lambda, double dtau, double tol, int max_iter,
                                      double* dtheta_out, int* iters_out, double* resid_out,
                                      void* ws, size_t ws_bytes, hipStream_t st) {
  if (!c) return NQS_ERR_ARG;
  auto fail = [&](nqs_status s, const std::string& msg) {
    c->last_error = msg;
    return s;
  };
  if (S < 1 || !O || !eloc || !dtheta_out) return fail(NQS_ERR_ARG, "sr_solve_cg: bad arguments");
  if (c->P % 2 != 0) return fail(NQS_ERR_ARG, "sr_solve_cg: P must be even");
  if (!(lambda >= 0.0) || !std::isfinite(lambda) || !std::isfinite(dtau) || !(tol >= 0.0) ||
      max_iter < 0)
    return fail(NQS_ERR_ARG, "sr_solve_cg: lambda >= 0, dtau finite, tol >= 0, max_iter >= 0");
  const size_t need = cg_workspace_bytes(c, S);
  if (!ws || ws_bytes < need)
    return fail(NQS_ERR_ARG, "sr_solve_cg: workspace too small: need " + std::to_string(need));
  int iters = 0, not_pd = 0;
  double resid = 0.0;
  prof_begin(c, K_CG, st);
  const hipError_t e =
      c->prec == NQS_FP64
          ? cg_run<double>(c, (const double*)O, eloc, S, lambda, dtau, tol, max_iter, dtheta_out,
                           (char*)ws, &iters, &resid, &not_pd, st)
          : cg_run<float>(c, (const float*)O, eloc, S, lambda, dtau, tol, max_iter, dtheta_out,
                          (char*)ws, &iters, &resid, &not_pd, st);
  prof_end(c, K_CG, st);
  if (iters_out) *iters_out = iters;
  if (resid_out) *resid_out = resid;
  if (e != hipSuccess) return fail(NQS_ERR_DEVICE, std::string("sr_solve_cg: ") + hipGetErrorString(e));
  if (not_pd) return fail(NQS_ERR_NOT_PD, "sr_solve_cg: p^H A p <= 0");
  if (!(resid <= tol))
    return fail(NQS_WARN_NOT_CONVERGED, "sr_solve_cg: relative residual " + std::to_string(resid) +
                                            " above tol after " + std::to_string(iters) +
                                            " iterations");
  return NQS_OK;
}

}  // namespace nqs
