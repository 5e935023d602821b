// Local energies (Sec. 3.2, Eq. (10)), two-hop H^2 terms and FP64 moments
// for the p = 1 Lanczos step (Sec. 3.3).
//
// Exchanging the antiparallel spins of bond b = (i, j) changes image g at
// the two sites of the bond's pre-image beta = g^-1(b) (a bond of the same
// kind, orientation flip), so theta_h -> theta_h + s D_h,beta with
// s = -2 sigma_i (sign-folded with the orientation) and
//   psi_s(g sigma^b) / psi_s(g sigma) = exp(s A_beta) prod_h cosh(D_h,beta)
//                                        * prod_h (1 + s tanh(theta_h) tanh(D_h,beta)).
// The first two factors and J_b/2 are the table F[k][beta][s]; the product
// runs on the VALU with no transcendental functions (8 operations per
// factor).  E_loc = diag + sum_b (J_b/2) sum_{k,g} w_kg R_kgb with the
// normalised image weights w of the log-sum-exp.
//
// Two exchanges b1 then b2 (b2 antiparallel in sigma^b1) give
// cosh(theta + s1 D1 + s2 D2) / (cosh theta cosh D1 cosh D2)
//   = 1 + t T1 + t T2 + T1 T2 = a + T2 (t + T1),  a = 1 + t T1,
// with sign-folded T1 = s1 tanh D1, T2 = s2 tanh D2, which yields
// e2 = (H^2 psi)/psi = diag e1 + sum_b1 (J_b1/2) [diag(sigma^b1) psi(sigma^b1)/psi
//      + sum_b2 (J_b2/2) psi(sigma^b1b2)/psi].
//
// Wave layout: one wavefront per (sample, 32-image tile); lane = (image,
// half of the bond list), so the bond loop is uniform across the wave and
// every lane streams its own image row of tanh(theta) against the gathered
// T rows.  Reductions are deterministic (fixed order, no float atomics).
#include "device_common.h"
#include "nqs_internal.h"
#include "pair_list.h"

namespace nqs {

namespace {

constexpr int kWavesPerBlock = 4;
constexpr int kMaxBonds = 4 * kMaxN;

// Antiparallel bond list of a spin row into LDS; returns the count.
__device__ __forceinline__ int build_anti_list(const int8_t* srow, const int32_t* bonds, int NB,
                                               int16_t* list, int lane) {
  int n = 0;
  for (int base = 0; base < NB; base += 64) {
    const int b = base + lane;
    bool anti = false;
    if (b < NB) anti = srow[bonds[2 * b]] != srow[bonds[2 * b + 1]];
    const unsigned long long m = __ballot(anti);
    const int pos = __popcll(m & ((1ull << lane) - 1ull));
    if (anti) list[n + pos] = (int16_t)b;
    n += __popcll(m);
  }
  wave_sync_lds();
  return n;
}

__device__ __forceinline__ double diag_of(const int8_t* srow, const int32_t* bonds,
                                          const double* bond_J, int NB, int lane) {
  double d = 0.0;
  for (int b = lane; b < NB; b += 64)
    d += 0.25 * bond_J[b] * (double)(srow[bonds[2 * b]] * srow[bonds[2 * b + 1]]);
  return wave_sum(d);
}

template <typename R, int NBD>
__global__ __launch_bounds__(256) void eloc_bonds_kernel(
    const int8_t* __restrict__ spins, int64_t S, int N, int G, int NB, int K, int M, int n_htiles,
    const int32_t* __restrict__ bonds, const int32_t* __restrict__ bmap,
    const R* __restrict__ t, const R* __restrict__ w, const R* __restrict__ Tpm,
    const R* __restrict__ F, double* __restrict__ partial) {
  __shared__ int16_t lists[kWavesPerBlock][kMaxBonds];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int ntiles = G / 32;
  const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + wv;
  if (wave >= S * ntiles) return;
  const int64_t s = wave / ntiles;
  const int tile = (int)(wave % ntiles);
  const int g = tile * 32 + (lane & 31);
  const int half = lane >> 5;
  const int8_t* srow = spins + s * N;
  int16_t* list = lists[wv];
  const int nc = build_anti_list(srow, bonds, NB, list, lane);
  wave_sync_lds();

  const int KM = K * M, tpr = M / 8;
  const R* tg = t + (((size_t)s * n_htiles) * G + g) * 16;   // + ht * G * 16
  const size_t tstride = (size_t)G * 16;
  double accr = 0.0, acci = 0.0;
  for (int i0 = half; i0 < nc; i0 += 2 * NBD) {
    const R* Trow[NBD];
    int fidx[NBD];
    R valid[NBD];
#pragma unroll
    for (int n = 0; n < NBD; ++n) {
      const int ii = i0 + 2 * n;
      valid[n] = ii < nc ? R(1) : R(0);
      const int b = ii < nc ? list[ii] : list[0];
      const int v = bmap[(size_t)g * NB + b];
      const int beta = v >> 1;
      const int s_b = -(int)srow[bonds[2 * b]];
      const int sp = (v & 1) ? -s_b : s_b;
      const int sidx = sp > 0 ? 0 : 1;
      Trow[n] = Tpm + ((size_t)beta * 2 + sidx) * KM * 2;
      fidx[n] = beta * 2 + sidx;
    }
    for (int k = 0; k < K; ++k) {
      R pr[NBD], pi[NBD];
#pragma unroll
      for (int n = 0; n < NBD; ++n) {
        const R* f = F + ((size_t)k * NB * 2 + fidx[n]) * 2;
        pr[n] = f[0];
        pi[n] = f[1];
      }
      for (int tt = 0; tt < tpr; ++tt) {
        const int ht = k * tpr + tt;
        const R* tp = tg + ht * tstride;
        R tv[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) tv[e] = tp[e];
#pragma unroll
        for (int n = 0; n < NBD; ++n) {
          const R* Tp = Trow[n] + (size_t)ht * 16;
          R Tv[16];
#pragma unroll
          for (int e = 0; e < 16; ++e) Tv[e] = Tp[e];
#pragma unroll
          for (int e = 0; e < 8; ++e)
            mul_one_plus(pr[n], pi[n], tv[2 * e], tv[2 * e + 1], Tv[2 * e], Tv[2 * e + 1]);
        }
      }
      const R* wk = w + (((size_t)s * K + k) * G + g) * 2;
      const R wr = wk[0], wi = wk[1];
#pragma unroll
      for (int n = 0; n < NBD; ++n) {
        accr += (double)(valid[n] * (wr * pr[n] - wi * pi[n]));
        acci += (double)(valid[n] * (wr * pi[n] + wi * pr[n]));
      }
    }
  }
  accr = wave_sum(accr);
  acci = wave_sum(acci);
  if (lane == 0) {
    partial[2 * wave] = accr;
    partial[2 * wave + 1] = acci;
  }
}

__global__ __launch_bounds__(64) void eloc_finish_kernel(const int8_t* __restrict__ spins, int N,
                                                         int NB, int ntiles,
                                                         const int32_t* __restrict__ bonds,
                                                         const double* __restrict__ bond_J,
                                                         const double* __restrict__ partial,
                                                         double* __restrict__ out, int stride) {
  const int64_t s = blockIdx.x;
  const int lane = threadIdx.x;
  const double d = diag_of(spins + s * N, bonds, bond_J, NB, lane);
  double pr = 0.0, pi = 0.0;
  for (int i = lane; i < ntiles; i += 64) {
    pr += partial[2 * (s * ntiles + i)];
    pi += partial[2 * (s * ntiles + i) + 1];
  }
  pr = wave_sum(pr);
  pi = wave_sum(pi);
  if (lane == 0) {
    out[(size_t)s * stride] = d + pr;
    out[(size_t)s * stride + 1] = pi;
  }
}

// One wavefront per (sample, first-hop slot, 32-image tile).
template <typename R, int NBD>
__global__ __launch_bounds__(256) void twohop_kernel(
    const int8_t* __restrict__ spins, int64_t S, int N, int G, int NB, int K, int M, int n_htiles,
    const int32_t* __restrict__ bonds, const double* __restrict__ bond_J,
    const int32_t* __restrict__ bmap, const R* __restrict__ t, const R* __restrict__ w,
    const R* __restrict__ Tpm, const R* __restrict__ F, double* __restrict__ partial2) {
  __shared__ int16_t lists[kWavesPerBlock][2][kMaxBonds];
  __shared__ int8_t rows[kWavesPerBlock][kMaxN];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int ntiles = G / 32;
  const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + wv;
  if (wave >= S * NB * ntiles) return;
  const int64_t s = wave / ((int64_t)NB * ntiles);
  const int slot = (int)((wave / ntiles) % NB);
  const int tile = (int)(wave % ntiles);
  const int8_t* srow = spins + s * N;
  int16_t* l1 = lists[wv][0];
  int16_t* l2 = lists[wv][1];
  const int nc = build_anti_list(srow, bonds, NB, l1, lane);
  if (slot >= nc) return;                               // wave-uniform
  const int b1 = l1[slot];
  const int i1 = bonds[2 * b1], j1 = bonds[2 * b1 + 1];
  int8_t* row2 = rows[wv];
  for (int i = lane; i < N; i += 64) row2[i] = srow[i];
  wave_sync_lds();
  if (lane == 0) {
    row2[i1] = srow[j1];
    row2[j1] = srow[i1];
  }
  wave_sync_lds();
  const int nc2 = build_pair_list(row2, bonds, NB, l2, lane, b1, i1, j1);
  const double diag2 = diag_of(row2, bonds, bond_J, NB, lane);
  wave_sync_lds();

  const int g = tile * 32 + (lane & 31);
  const int half = lane >> 5;
  const int KM = K * M, tpr = M / 8;
  const R* tg = t + (((size_t)s * n_htiles) * G + g) * 16;
  const size_t tstride = (size_t)G * 16;

  const int v1 = bmap[(size_t)g * NB + b1];
  const int beta1 = v1 >> 1;
  const int s1b = -(int)srow[i1];
  const int s1 = (v1 & 1) ? -s1b : s1b;
  const int s1idx = s1 > 0 ? 0 : 1;
  const R* T1row = Tpm + ((size_t)beta1 * 2 + s1idx) * KM * 2;

  double accr = 0.0, acci = 0.0;
  // first hop alone (only one half of the wave, to count each image once)
  for (int k = 0; k < K; ++k) {
    const R* f1 = F + ((size_t)k * NB * 2 + beta1 * 2 + s1idx) * 2;
    R pr = f1[0], pi = f1[1];
    for (int tt = 0; tt < tpr; ++tt) {
      const int ht = k * tpr + tt;
      const R* tp = tg + ht * tstride;
      const R* Tp = T1row + (size_t)ht * 16;
#pragma unroll
      for (int e = 0; e < 8; ++e) mul_one_plus(pr, pi, tp[2 * e], tp[2 * e + 1], Tp[2 * e], Tp[2 * e + 1]);
    }
    const R* wk = w + (((size_t)s * K + k) * G + g) * 2;
    const R wr = wk[0], wi = wk[1];
    if (half == 0) {
      accr += diag2 * (double)(wr * pr - wi * pi);
      acci += diag2 * (double)(wr * pi + wi * pr);
      // b1 exchanged back: s^{b1 b1} = s, ratio 1 in every image
      const double jj = 0.25 * bond_J[b1] * bond_J[b1];
      accr += jj * (double)wr;
      acci += jj * (double)wi;
    }
  }
  // second hop
  for (int i0 = half; i0 < nc2; i0 += 2 * NBD) {
    const R* Trow[NBD];
    int fidx[NBD];
    R valid[NBD];
#pragma unroll
    for (int n = 0; n < NBD; ++n) {
      const int ii = i0 + 2 * n;
      const int e = ii < nc2 ? l2[ii] : l2[0];
      valid[n] = ii < nc2 ? ((e & kPairTwice) ? R(2) : R(1)) : R(0);
      const int b = e & kPairBond;
      const int v = bmap[(size_t)g * NB + b];
      const int beta = v >> 1;
      const int s_b = -(int)row2[bonds[2 * b]];
      const int sp = (v & 1) ? -s_b : s_b;
      const int sidx = sp > 0 ? 0 : 1;
      Trow[n] = Tpm + ((size_t)beta * 2 + sidx) * KM * 2;
      fidx[n] = beta * 2 + sidx;
    }
    for (int k = 0; k < K; ++k) {
      const R* f1 = F + ((size_t)k * NB * 2 + beta1 * 2 + s1idx) * 2;
      R pr[NBD], pi[NBD];
#pragma unroll
      for (int n = 0; n < NBD; ++n) {
        const R* f = F + ((size_t)k * NB * 2 + fidx[n]) * 2;
        pr[n] = f[0] * f1[0] - f[1] * f1[1];
        pi[n] = f[0] * f1[1] + f[1] * f1[0];
      }
      for (int tt = 0; tt < tpr; ++tt) {
        const int ht = k * tpr + tt;
        const R* tp = tg + ht * tstride;
        const R* T1p = T1row + (size_t)ht * 16;
        R ar[8], ai[8], br[8], bi[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const R tr = tp[2 * e], ti = tp[2 * e + 1];
          const R Ur = T1p[2 * e], Ui = T1p[2 * e + 1];
          ar[e] = fmaf_t(tr, Ur, fmaf_t(-ti, Ui, R(1)));
          ai[e] = fmaf_t(tr, Ui, ti * Ur);
          br[e] = tr + Ur;
          bi[e] = ti + Ui;
        }
#pragma unroll
        for (int n = 0; n < NBD; ++n) {
          const R* Tp = Trow[n] + (size_t)ht * 16;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const R Vr = Tp[2 * e], Vi = Tp[2 * e + 1];
            const R fr = fmaf_t(Vr, br[e], fmaf_t(-Vi, bi[e], ar[e]));
            const R fi = fmaf_t(Vr, bi[e], fmaf_t(Vi, br[e], ai[e]));
            const R nr = fmaf_t(pr[n], fr, -(pi[n] * fi));
            pi[n] = fmaf_t(pr[n], fi, pi[n] * fr);
            pr[n] = nr;
          }
        }
      }
      const R* wk = w + (((size_t)s * K + k) * G + g) * 2;
      const R wr = wk[0], wi = wk[1];
#pragma unroll
      for (int n = 0; n < NBD; ++n) {
        accr += (double)(valid[n] * (wr * pr[n] - wi * pi[n]));
        acci += (double)(valid[n] * (wr * pi[n] + wi * pr[n]));
      }
    }
  }
  accr = wave_sum(accr);
  acci = wave_sum(acci);
  if (lane == 0) {
    const size_t o = ((size_t)s * NB + slot) * ntiles + tile;
    partial2[2 * o] = accr;
    partial2[2 * o + 1] = acci;
  }
}

// e2 = diag e1 + sum over (first-hop slot, tile) partials; e1e2 holds e1 on entry.
__global__ __launch_bounds__(64) void twohop_finish_kernel(const int8_t* __restrict__ spins, int N,
                                                           int NB, int ntiles,
                                                           const int32_t* __restrict__ bonds,
                                                           const double* __restrict__ bond_J,
                                                           const double* __restrict__ partial2,
                                                           double* __restrict__ e1e2) {
  __shared__ int16_t list[kMaxBonds];
  const int64_t s = blockIdx.x;
  const int lane = threadIdx.x;
  const int8_t* srow = spins + s * N;
  const int nc = build_anti_list(srow, bonds, NB, list, lane);
  const double d = diag_of(srow, bonds, bond_J, NB, lane);
  double pr = 0.0, pi = 0.0;
  const int n = nc * ntiles;
  for (int i = lane; i < n; i += 64) {
    const size_t o = ((size_t)s * NB + i / ntiles) * ntiles + (i % ntiles);
    pr += partial2[2 * o];
    pi += partial2[2 * o + 1];
  }
  pr = wave_sum(pr);
  pi = wave_sum(pi);
  if (lane == 0) {
    const double e1r = e1e2[4 * s], e1i = e1e2[4 * s + 1];
    e1e2[4 * s + 2] = d * e1r + pr;
    e1e2[4 * s + 3] = d * e1i + pi;
  }
}

// Two-pass FP64 moments in one workgroup (fixed summation order).
// result: h1 h1_im h2 h2_alt h3 c2 c3 v r alpha e_p1 h1_err degenerate n
__global__ __launch_bounds__(1024) void moments_kernel(const double* __restrict__ e1e2,
                                                       const double* __restrict__ logpsi, int64_t S,
                                                       int exact, double* __restrict__ result) {
  __shared__ double red[16][8];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  auto block_sum = [&](double* v, int nv) {
    for (int j = 0; j < nv; ++j) {
      double x = wave_sum(v[j]);
      if (lane == 0) red[wv][j] = x;
    }
    __syncthreads();
    for (int j = 0; j < nv; ++j) {
      double x = 0.0;
      for (int q = 0; q < 16; ++q) x += red[q][j];
      v[j] = x;
    }
    __syncthreads();
  };
  double mx = -INFINITY;
  if (exact)
    for (int64_t i = tid; i < S; i += 1024) mx = fmax(mx, logpsi[2 * i]);
  mx = wave_max(mx);
  if (lane == 0) red[wv][0] = mx;
  __syncthreads();
  mx = red[0][0];
  for (int q = 1; q < 16; ++q) mx = fmax(mx, red[q][0]);
  __syncthreads();
  auto weight = [&](int64_t i) -> double {
    if (!exact) return 1.0;
    const double p = exp(2.0 * (logpsi[2 * i] - mx));
    return p < 1e-300 ? 0.0 : p;   // psi = 0 configurations carry no weight
  };
  double v1[4] = {0.0, 0.0, 0.0, 0.0};   // sum p, sum p e1 (re, im), count
  for (int64_t i = tid; i < S; i += 1024) {
    const double p = weight(i);
    if (p == 0.0) continue;
    v1[0] += p;
    v1[1] += p * e1e2[4 * i];
    v1[2] += p * e1e2[4 * i + 1];
    v1[3] += 1.0;
  }
  block_sum(v1, 4);
  const double sw = v1[0];
  const double h1 = v1[1] / sw, h1i = v1[2] / sw;
  double v2[6] = {0, 0, 0, 0, 0, 0};     // h2, c2, h2_alt, h3, c3
  for (int64_t i = tid; i < S; i += 1024) {
    const double p = weight(i);
    if (p == 0.0) continue;
    const double er = e1e2[4 * i], ei = e1e2[4 * i + 1];
    const double fr = e1e2[4 * i + 2], fi = e1e2[4 * i + 3];
    const double dr = er - h1;
    v2[0] += p * (er * er + ei * ei);
    v2[1] += p * (dr * dr + ei * ei);
    v2[2] += p * fr;
    v2[3] += p * (er * fr + ei * fi);
    const double gr = fr - 2.0 * h1 * er + h1 * h1, gi = fi - 2.0 * h1 * ei;
    v2[4] += p * (dr * gr + ei * gi);
  }
  block_sum(v2, 5);
  if (tid == 0) {
    const double h2 = v2[0] / sw, c2 = v2[1] / sw, h2a = v2[2] / sw, h3 = v2[3] / sw,
                 c3 = v2[4] / sw;
    double v = 0.0, r = 0.0, alpha = 0.0, ep1 = h1, degen = 1.0;
    const double tiny = 8.0 * 1.1102230246251565e-16 * fmax(fabs(h1), 1.0);
    if (c2 > tiny * tiny) {
      v = sqrt(c2);
      r = c3 / (v * v * v);
      const double root = sqrt(0.25 * r * r + 1.0);
      alpha = r <= 0.0 ? 0.5 * r - root : -1.0 / (0.5 * r + root);
      ep1 = h1 + v * alpha;
      degen = 0.0;
    }
    const double out[14] = {h1, h1i, h2, h2a, h3, c2, c3, v, r, alpha, ep1,
                            sqrt(c2 / v1[3]), degen, v1[3]};
    for (int j = 0; j < 14; ++j) result[j] = out[j];
  }
}

template <typename R>
hipError_t eloc_typed(const nqs_ctx* c, const int8_t* spins, int64_t S, const void* t,
                      const void* w, double* partial, hipStream_t st) {
  const int64_t waves = S * (c->G / 32);
  const int64_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
  eloc_bonds_kernel<R, 4><<<(unsigned)blocks, 64 * kWavesPerBlock, 0, st>>>(
      spins, S, c->N, c->G, c->NB, c->K, c->M, c->n_htiles, c->dev.bonds, c->dev.bmap,
      (const R*)t, (const R*)w, (const R*)c->par.Tpm, (const R*)c->par.F, partial);
  return hipGetLastError();
}

template <typename R>
hipError_t twohop_typed(const nqs_ctx* c, const int8_t* spins, int64_t S, const void* t,
                        const void* w, double* partial2, hipStream_t st) {
  const int64_t waves = S * c->NB * (c->G / 32);
  const int64_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
  twohop_kernel<R, 4><<<(unsigned)blocks, 64 * kWavesPerBlock, 0, st>>>(
      spins, S, c->N, c->G, c->NB, c->K, c->M, c->n_htiles, c->dev.bonds, c->dev.bond_J,
      c->dev.bmap, (const R*)t, (const R*)w, (const R*)c->par.Tpm, (const R*)c->par.F, partial2);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_eloc_bonds(const nqs_ctx* c, const int8_t* spins, int64_t S, const void* t,
                             const void* w, double* partial, hipStream_t st) {
  if (S <= 0) return hipSuccess;
  const hipError_t e = launch_eloc_bonds_reg(c, spins, S, t, w, partial, st);
  if (e != hipErrorNotSupported) return e;
  return c->prec == NQS_FP64 ? eloc_typed<double>(c, spins, S, t, w, partial, st)
                             : eloc_typed<float>(c, spins, S, t, w, partial, st);
}

hipError_t launch_eloc_finish(const nqs_ctx* c, const int8_t* spins, int64_t S,
                              const double* partial, double* eloc_out, int eloc_stride,
                              hipStream_t st) {
  if (S <= 0) return hipSuccess;
  eloc_finish_kernel<<<(unsigned)S, 64, 0, st>>>(spins, c->N, c->NB, c->G / 32, c->dev.bonds,
                                                 c->dev.bond_J, partial, eloc_out, eloc_stride);
  return hipGetLastError();
}

hipError_t launch_twohop(const nqs_ctx* c, const int8_t* spins, int64_t S, const void* t,
                         const void* w, double* partial2, hipStream_t st) {
  if (S <= 0) return hipSuccess;
  const hipError_t e = launch_twohop_reg(c, spins, S, t, w, partial2, st);
  if (e != hipErrorNotSupported) return e;
  return c->prec == NQS_FP64 ? twohop_typed<double>(c, spins, S, t, w, partial2, st)
                             : twohop_typed<float>(c, spins, S, t, w, partial2, st);
}

hipError_t launch_twohop_finish(const nqs_ctx* c, const int8_t* spins, int64_t S,
                                const double* partial2, double* e1e2, hipStream_t st) {
  if (S <= 0) return hipSuccess;
  twohop_finish_kernel<<<(unsigned)S, 64, 0, st>>>(spins, c->N, c->NB, c->G / 32, c->dev.bonds,
                                                   c->dev.bond_J, partial2, e1e2);
  return hipGetLastError();
}

hipError_t launch_moments(const double* e1e2, const double* logpsi, int64_t S, int exact,
                          double* partial, int nblocks, double* result, hipStream_t st) {
  (void)partial;
  (void)nblocks;
  moments_kernel<<<1, 1024, 0, st>>>(e1e2, logpsi, S, exact, result);
  return hipGetLastError();
}

}  // namespace nqs
