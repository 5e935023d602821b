// Fused log psi + E_loc (Sec. 3.1 Eqs. (2), (6); Sec. 3.2 Eq. (10)) for
// models whose hidden layer fits in registers (K*M <= 128).
//
// One wavefront per (sample, 16-image column block): the theta contraction
// runs on 16x16 MFMA exactly as in k_theta.hip, the log 2cosh / tanh
// epilogue leaves tanh(theta) in the MFMA output layout -- lane (q, c) holds
// hidden units 8 ht + 2q, 8 ht + 2q + 1 of image c -- and never goes to HBM.
// Each bond-exchange product prod_h (s + t_h T_h) (sign folding as in
// k_eloc_reg.hip) is split four ways over the q lanes of an image and joined
// with two cross-lane complex multiplications.
//
// The normalisation of the image weights is wave-local: with m the largest
// Re L over the wave's images, u_kg = chi_g exp(L_kg - m), the wave emits
// (m, sum u, sum_b (J_b/2) sum u R) and a per-sample finish kernel combines
// the column blocks: log psi = M + log sum e^{m-M} den,
// E_loc = diag + sum e^{m-M} Q / sum e^{m-M} den.
//
// Persistent workgroups of 16 wavefronts keep the +tanh(D) bond table and
// the W fragments in LDS for the whole launch.
#include "theta_common.h"

namespace nqs {

namespace {

constexpr int kFusedWaves = 8;

template <int N, int PREC, int K, int M>
struct FusedCfg {
  using T = ThetaTraits<PREC>;
  using R = typename T::R;
  static constexpr int NB = 4 * N;
  static constexpr int KM = K * M;
  static constexpr int NHT = KM / 8;
  static constexpr int NK = nk_of<N, PREC>();
  static constexpr int ST = 2 * KM + (sizeof(R) == 4 ? 4 : 2);
  static constexpr size_t LDS = (size_t)NB * ST * sizeof(R) +
                                (size_t)NHT * NK * 64 * sizeof(typename T::AFrag) +
                                (size_t)kFusedWaves * NB * 2;
};

__device__ __forceinline__ int fused_list(const int8_t* srow, const int32_t* bonds, int NB,
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

template <typename R>
__device__ __forceinline__ void step_sp(R& pr, R& pi, R s, R tr, R ti, R Tr, R Ti) {
  const R a = fmaf_t(tr, Tr, fmaf_t(-ti, Ti, s));
  const R b = fmaf_t(tr, Ti, ti * Tr);
  const R nr = fmaf_t(pr, a, -(pi * b));
  pi = fmaf_t(pr, b, pi * a);
  pr = nr;
}

// complex product over the four q lanes of one image (xor 16, xor 32)
template <typename R>
__device__ __forceinline__ void qprod(R& pr, R& pi) {
#pragma unroll
  for (int o = 16; o <= 32; o <<= 1) {
    const R orr = __shfl_xor(pr, o, 64), oi = __shfl_xor(pi, o, 64);
    const R nr = pr * orr - pi * oi;
    pi = pr * oi + pi * orr;
    pr = nr;
  }
}

template <int N, int PREC, int K, int M>
__global__ __launch_bounds__(64 * kFusedWaves) void eloc_fused_kernel(
    const int8_t* __restrict__ spins, int64_t S, const uint8_t* __restrict__ perm, int G,
    const typename ThetaTraits<PREC>::AFrag* __restrict__ wfrag,
    const typename ThetaTraits<PREC>::R* __restrict__ bias,
    const typename ThetaTraits<PREC>::R* __restrict__ avec, const int32_t* __restrict__ bonds,
    const int32_t* __restrict__ bmap, const double* __restrict__ chi,
    const typename ThetaTraits<PREC>::R* __restrict__ Tpm,
    const typename ThetaTraits<PREC>::R* __restrict__ F, double* __restrict__ part) {
  using Cfg = FusedCfg<N, PREC, K, M>;
  using T = ThetaTraits<PREC>;
  using R = typename T::R;
  using AF = typename T::AFrag;
  constexpr int NB = Cfg::NB, KM = Cfg::KM, NHT = Cfg::NHT, NK = Cfg::NK, ST = Cfg::ST;
  constexpr int TPR = M / 8;
  __shared__ __align__(16) R Tl[NB * ST];
  __shared__ __align__(16) AF Wl[NHT * NK * 64];
  __shared__ int16_t lists[kFusedWaves][NB];

  for (int idx = threadIdx.x; idx < NB * KM; idx += blockDim.x) {
    const int beta = idx / KM, h = idx % KM;
    const R* src = Tpm + ((size_t)beta * 2 * KM + h) * 2;
    Tl[beta * ST + 2 * h] = src[0];
    Tl[beta * ST + 2 * h + 1] = src[1];
  }
  for (int idx = threadIdx.x; idx < NHT * NK * 64; idx += blockDim.x) Wl[idx] = wfrag[idx];
  __syncthreads();

  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int q = lane >> 4, c = lane & 15;
  const int cbs = G / 16;
  const int64_t n_items = S * cbs;
  const int64_t stride = (int64_t)gridDim.x * kFusedWaves;
  int16_t* list = lists[wv];

  for (int64_t item = (int64_t)blockIdx.x * kFusedWaves + wv; item < n_items; item += stride) {
    const int64_t s = item / cbs;
    const int g = (int)(item % cbs) * 16 + c;
    const int8_t* srow = spins + s * N;
    const uint8_t* prow = perm + (size_t)g * N;
    typename T::BFrag bx[NK];
    load_bfrag<N, PREC>(srow, prow, q, bx);
    const int nc = fused_list(srow, bonds, NB, list, lane);

    // ---- theta on MFMA + epilogue: tanh(theta) stays in registers
    R tr[NHT * 2], ti[NHT * 2];
    double Lr[K], Li[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      R pr = R(1), pi = R(0);
      int pe = 0;
      double sax = 0.0;
#pragma unroll
      for (int tt = 0; tt < TPR; ++tt) {
        const int ht = k * TPR + tt;
        typename T::Acc acc = typename T::Acc{0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) acc = mfma(Wl[(ht * NK + kk) * 64 + lane], bx[kk], acc);
        const int h0 = 8 * ht + 2 * q;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const R x = (R)acc[2 * u] + bias[2 * (h0 + u)];
          const R y = (R)acc[2 * u + 1] + bias[2 * (h0 + u) + 1];
          logcosh_step<R, true>(x, y, pr, pi, sax, tr[2 * ht + u], ti[2 * ht + u]);
        }
        if ((tt & 7) == 7) renorm(pr, pi, pe);
      }
      renorm(pr, pi, pe);
      int E = pe;
#pragma unroll
      for (int o = 16; o <= 32; o <<= 1) {
        const R orr = __shfl_xor(pr, o, 64), oi = __shfl_xor(pi, o, 64);
        const R nr = pr * orr - pi * oi;
        pi = pr * oi + pi * orr;
        pr = nr;
        E += __shfl_xor(E, o, 64);
        sax += __shfl_xor(sax, o, 64);
      }
      double axr = 0.0, axi = 0.0;
      const R* ak = avec + (size_t)k * N * 2;
#pragma unroll
      for (int jj = 0; jj < N / 4; ++jj) {
        const int j = 4 * jj + q;
        const double xj = 0.5 * (double)srow[prow[j]];
        axr += xj * (double)ak[2 * j];
        axi += xj * (double)ak[2 * j + 1];
      }
      axr += __shfl_xor(axr, 16, 64);
      axi += __shfl_xor(axi, 16, 64);
      axr += __shfl_xor(axr, 32, 64);
      axi += __shfl_xor(axi, 32, 64);
      Lr[k] = axr + sax + (double)(R(0.5) * log_t(pr * pr + pi * pi)) +
              (double)E * 0.69314718055994530942;
      Li[k] = axi + (double)atan2_t(pi, pr);
    }
    double mloc = Lr[0];
#pragma unroll
    for (int k = 1; k < K; ++k) mloc = fmax(mloc, Lr[k]);
    const double m = wave_max(mloc);
    const R ch = (R)chi[g];
    R ur[K], ui[K];
    double denr = 0.0, deni = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const R e = ch * exp_t((R)(Lr[k] - m));
      R sn, cs;
      sincos_t((R)Li[k], &sn, &cs);
      ur[k] = e * cs;
      ui[k] = e * sn;
      denr += (double)ur[k];
      deni += (double)ui[k];
    }

    // ---- bond exchanges, two bonds per pass
    double Qr = 0.0, Qi = 0.0;
    for (int i0 = 0; i0 < nc; i0 += 2) {
      int beta[2], sidx[2];
      R sgn[2], valid[2];
#pragma unroll
      for (int n = 0; n < 2; ++n) {
        const int ii = i0 + n;
        valid[n] = ii < nc ? R(1) : R(0);
        const int b = list[ii < nc ? ii : i0];
        const int v = bmap[(size_t)g * NB + b];
        beta[n] = v >> 1;
        const int s_b = -(int)srow[bonds[2 * b]];
        const int sp = (v & 1) ? -s_b : s_b;
        sgn[n] = (R)sp;
        sidx[n] = sp > 0 ? 0 : 1;
      }
      const R* T0 = Tl + beta[0] * ST + 4 * q;
      const R* T1 = Tl + beta[1] * ST + 4 * q;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        R a0r = 1, a0i = 0, b0r = 1, b0i = 0, a1r = 1, a1i = 0, b1r = 1, b1i = 0;
#pragma unroll
        for (int tt = 0; tt < TPR; ++tt) {
          const int ht = k * TPR + tt;
          if constexpr (sizeof(R) == 4) {
            const float4 x0 = *reinterpret_cast<const float4*>(T0 + 16 * ht);
            const float4 x1 = *reinterpret_cast<const float4*>(T1 + 16 * ht);
            step_sp<R>(a0r, a0i, sgn[0], tr[2 * ht], ti[2 * ht], x0.x, x0.y);
            step_sp<R>(b0r, b0i, sgn[0], tr[2 * ht + 1], ti[2 * ht + 1], x0.z, x0.w);
            step_sp<R>(a1r, a1i, sgn[1], tr[2 * ht], ti[2 * ht], x1.x, x1.y);
            step_sp<R>(b1r, b1i, sgn[1], tr[2 * ht + 1], ti[2 * ht + 1], x1.z, x1.w);
          } else {
            const double2 x0 = *reinterpret_cast<const double2*>(T0 + 16 * ht);
            const double2 y0 = *reinterpret_cast<const double2*>(T0 + 16 * ht + 2);
            const double2 x1 = *reinterpret_cast<const double2*>(T1 + 16 * ht);
            const double2 y1 = *reinterpret_cast<const double2*>(T1 + 16 * ht + 2);
            step_sp<R>(a0r, a0i, sgn[0], tr[2 * ht], ti[2 * ht], x0.x, x0.y);
            step_sp<R>(b0r, b0i, sgn[0], tr[2 * ht + 1], ti[2 * ht + 1], y0.x, y0.y);
            step_sp<R>(a1r, a1i, sgn[1], tr[2 * ht], ti[2 * ht], x1.x, x1.y);
            step_sp<R>(b1r, b1i, sgn[1], tr[2 * ht + 1], ti[2 * ht + 1], y1.x, y1.y);
          }
        }
        R p0r = a0r * b0r - a0i * b0i, p0i = a0r * b0i + a0i * b0r;
        R p1r = a1r * b1r - a1i * b1i, p1i = a1r * b1i + a1i * b1r;
        qprod(p0r, p0i);
        qprod(p1r, p1i);
        if (q == 0) {
          const R* f0 = F + (((size_t)k * NB + beta[0]) * 2 + sidx[0]) * 2;
          const R* f1 = F + (((size_t)k * NB + beta[1]) * 2 + sidx[1]) * 2;
          const R g0r = f0[0] * ur[k] - f0[1] * ui[k], g0i = f0[0] * ui[k] + f0[1] * ur[k];
          const R g1r = f1[0] * ur[k] - f1[1] * ui[k], g1i = f1[0] * ui[k] + f1[1] * ur[k];
          Qr += (double)(valid[0] * (g0r * p0r - g0i * p0i)) +
                (double)(valid[1] * (g1r * p1r - g1i * p1i));
          Qi += (double)(valid[0] * (g0r * p0i + g0i * p0r)) +
                (double)(valid[1] * (g1r * p1i + g1i * p1r));
        }
      }
    }
    if (q != 0) {
      denr = 0.0;
      deni = 0.0;
    }
    Qr = wave_sum(Qr);
    Qi = wave_sum(Qi);
    denr = wave_sum(denr);
    deni = wave_sum(deni);
    if (lane == 0) {
      double* o = part + item * 6;
      o[0] = m;
      o[1] = denr;
      o[2] = deni;
      o[3] = Qr;
      o[4] = Qi;
      o[5] = 0.0;
    }
    wave_sync_lds();
  }
}

// Per sample: combine the column blocks into log psi and E_loc.
__global__ __launch_bounds__(64) void fused_finish_kernel(
    const int8_t* __restrict__ spins, int N, int NB, int cbs, const int32_t* __restrict__ bonds,
    const double* __restrict__ bond_J, const double* __restrict__ part, double* __restrict__ logpsi,
    double* __restrict__ eloc, int eloc_stride) {
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
  double dr = 0, di = 0, qr = 0, qi = 0;
  for (int i = lane; i < cbs; i += 64) {
    const double e = exp(ps[6 * i] - mx);
    dr += e * ps[6 * i + 1];
    di += e * ps[6 * i + 2];
    qr += e * ps[6 * i + 3];
    qi += e * ps[6 * i + 4];
  }
  dr = wave_sum(dr);
  di = wave_sum(di);
  qr = wave_sum(qr);
  qi = wave_sum(qi);
  if (lane == 0) {
    const double den2 = dr * dr + di * di;
    if (logpsi) {
      logpsi[2 * s] = mx + 0.5 * log(den2);
      logpsi[2 * s + 1] = atan2(di, dr);
    }
    eloc[(size_t)s * eloc_stride] = d + (qr * dr + qi * di) / den2;
    eloc[(size_t)s * eloc_stride + 1] = (qi * dr - qr * di) / den2;
  }
}

template <int N, int PREC, int K, int M>
hipError_t run(const nqs_ctx* c, const int8_t* spins, int64_t S, double* part, double* logpsi,
               double* eloc, int eloc_stride, hipStream_t st) {
  using T = ThetaTraits<PREC>;
  using R = typename T::R;
  const int cbs = c->G / 16;
  const int64_t items = S * cbs;
  int64_t blocks = (items + kFusedWaves - 1) / kFusedWaves;
  blocks = std::min<int64_t>(blocks, c->n_cu > 0 ? c->n_cu : 256);
  eloc_fused_kernel<N, PREC, K, M><<<(unsigned)blocks, 64 * kFusedWaves, 0, st>>>(
      spins, S, c->dev.perm, c->G, (const typename T::AFrag*)c->par.wfrag, (const R*)c->par.bias,
      (const R*)c->par.avec, c->dev.bonds, c->dev.bmap, c->dev.chi, (const R*)c->par.Tpm,
      (const R*)c->par.F, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  fused_finish_kernel<<<(unsigned)S, 64, 0, st>>>(spins, c->N, c->NB, cbs, c->dev.bonds,
                                                  c->dev.bond_J, part, logpsi, eloc, eloc_stride);
  return hipGetLastError();
}

constexpr size_t kLdsLimit = 160 * 1024;

template <int N, int PREC, int K, int M>
hipError_t run_if_fits(const nqs_ctx* c, const int8_t* spins, int64_t S, double* part,
                       double* logpsi, double* eloc, int es, hipStream_t st) {
  if constexpr (FusedCfg<N, PREC, K, M>::LDS <= kLdsLimit)
    return run<N, PREC, K, M>(c, spins, S, part, logpsi, eloc, es, st);
  else
    return hipErrorNotSupported;
}

template <int N, int K, int M>
hipError_t run_prec(const nqs_ctx* c, const int8_t* spins, int64_t S, double* part,
                    double* logpsi, double* eloc, int es, hipStream_t st) {
  switch (c->prec) {
    case NQS_FP64: return run_if_fits<N, NQS_FP64, K, M>(c, spins, S, part, logpsi, eloc, es, st);
    case NQS_FP32: return run_if_fits<N, NQS_FP32, K, M>(c, spins, S, part, logpsi, eloc, es, st);
    default: return run_if_fits<N, NQS_BF16X2, K, M>(c, spins, S, part, logpsi, eloc, es, st);
  }
}

template <int N, int K, int M>
bool fits(int prec) {
  switch (prec) {
    case NQS_FP64: return FusedCfg<N, NQS_FP64, K, M>::LDS <= kLdsLimit;
    case NQS_FP32: return FusedCfg<N, NQS_FP32, K, M>::LDS <= kLdsLimit;
    default: return FusedCfg<N, NQS_BF16X2, K, M>::LDS <= kLdsLimit;
  }
}

}  // namespace

bool eloc_fused_supported(const nqs_ctx* c) {
  const int N = c->N, K = c->K, M = c->M, p = c->prec;
  if (N == 16 && K == 1 && M == 16) return fits<16, 1, 16>(p);
  if (N == 16 && K == 2 && M == 8) return fits<16, 2, 8>(p);
  if (N == 36 && K == 1 && M == 72) return fits<36, 1, 72>(p);
  if (N == 36 && K == 2 && M == 16) return fits<36, 2, 16>(p);
  if (N == 36 && K == 1 && M == 16) return fits<36, 1, 16>(p);
  return false;
}

hipError_t launch_eloc_fused(const nqs_ctx* c, const int8_t* spins, int64_t S, double* part,
                             double* logpsi, double* eloc, int eloc_stride, hipStream_t st) {
  if (S <= 0) return hipSuccess;
  const int N = c->N, K = c->K, M = c->M;
  if (N == 16 && K == 1 && M == 16) return run_prec<16, 1, 16>(c, spins, S, part, logpsi, eloc, eloc_stride, st);
  if (N == 16 && K == 2 && M == 8) return run_prec<16, 2, 8>(c, spins, S, part, logpsi, eloc, eloc_stride, st);
  if (N == 36 && K == 1 && M == 72) return run_prec<36, 1, 72>(c, spins, S, part, logpsi, eloc, eloc_stride, st);
  if (N == 36 && K == 2 && M == 16) return run_prec<36, 2, 16>(c, spins, S, part, logpsi, eloc, eloc_stride, st);
  if (N == 36 && K == 1 && M == 16) return run_prec<36, 1, 16>(c, spins, S, part, logpsi, eloc, eloc_stride, st);
  return hipErrorNotSupported;
}

}  // namespace nqs
