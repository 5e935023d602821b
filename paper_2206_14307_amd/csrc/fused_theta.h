// Theta of one (sample, 16-image column block) on MFMA with the log 2cosh /
// tanh epilogue (Sec. 3.1, Eq. (2)), shared by the fused E_loc and gradient
// kernels.  Lane (q, c) = (lane / 16, lane % 16) handles image c of the block;
// the W fragments are ordered so that every lane receives Re and Im theta of
// hidden units 8 ht + 2q and 8 ht + 2q + 1 (ht = hidden tile).
//
// Per RBM k the block returns, for the lane's image,
//   L_k = Er_k + log P_k + i Ai_k   (log psi_s of the image, up to i arg P_k)
// with Er_k = Re a.x + sum_h |Re theta_h| + E ln 2 in FP64, P_k the product
// of the c_h of the epilogue renormalised to |P_k| in [1/16, 4) (its exponent
// E moved into Er_k) and Ai_k = Im a.x; tanh(theta) of the lane's hidden
// units stays in tr / ti.  All four q lanes of an image end with the same
// Er, P and Ai.
#pragma once

#include "theta_common.h"

namespace nqs {

template <int N, int PREC, int K, int M>
__device__ __forceinline__ void theta_block(
    const typename ThetaTraits<PREC>::AFrag* Wl, const typename ThetaTraits<PREC>::BFrag* bx,
    const typename ThetaTraits<PREC>::R* bias, const typename ThetaTraits<PREC>::R* avec,
    const int8_t* srow,
    const uint8_t* prow, int lane, typename ThetaTraits<PREC>::R* tr,
    typename ThetaTraits<PREC>::R* ti, double* Er, typename ThetaTraits<PREC>::R* Pr,
    typename ThetaTraits<PREC>::R* Pi, typename ThetaTraits<PREC>::R* Ai,
    const float* axp = nullptr) {
  using T = ThetaTraits<PREC>;
  using R = typename T::R;
  constexpr int NK = nk_of<N, PREC>();
  constexpr int TPR = M / 8;
  const int q = lane >> 4;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    R pr = R(1), pi = R(0);
    int pe = 0;
    uint32_t par = 0u;
    double sax = 0.0;
#pragma unroll
    for (int tt = 0; tt < TPR; ++tt) {
      const int ht = k * TPR + tt;
      const int h0 = 8 * ht + 2 * q;
      typename T::Acc acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = bias[2 * h0 + v];   // start from the biases
#pragma unroll
      for (int kk = 0; kk < NK; ++kk) acc = mfma(Wl[(ht * NK + kk) * 64 + lane], bx[kk], acc);
      const R ax0 = logcosh_step<R, true>((R)acc[0], (R)acc[1], pr, pi, par, tr[2 * ht],
                                          ti[2 * ht]);
      const R ax1 = logcosh_step<R, true>((R)acc[2], (R)acc[3], pr, pi, par, tr[2 * ht + 1],
                                          ti[2 * ht + 1]);
      sax += (double)(ax0 + ax1);
      if ((tt & 7) == 7) renorm(pr, pi, pe);
    }
    renorm(pr, pi, pe);
    apply_parity(pr, pi, par);
    // a . (g sigma): FP32 / FP64 fragments hold x_j for j = q mod 4
    R xr = R(0), xi = R(0);
    const R* ak = avec + (size_t)k * N * 2;
    if constexpr (PREC == kPrecF32S3) {
      // the caller's partial sums over the lane's sites 4i + q
      xr = axp[2 * k];
      xi = axp[2 * k + 1];
    } else if constexpr (!bf16_mfma(PREC)) {
#pragma unroll
      for (int kk = 0; kk < NK; ++kk) {
        xr = fmaf_t(bx[kk], ak[2 * (4 * kk + q)], xr);
        xi = fmaf_t(bx[kk], ak[2 * (4 * kk + q) + 1], xi);
      }
    } else {
#pragma unroll
      for (int jj = 0; jj < N / 4; ++jj) {
        const int j = 4 * jj + q;
        const R xj = R(0.5) * (R)srow[prow[j]];
        xr = fmaf_t(xj, ak[2 * j], xr);
        xi = fmaf_t(xj, ak[2 * j + 1], xi);
      }
    }
    allprod_rows(pr, pi);
    const int E = allreduce_rows(pe, [](int u, int v) { return u + v; });
    sax = allreduce_rows(sax, [](double u, double v) { return u + v; });
    xr = allreduce_rows(xr, [](R u, R v) { return u + v; });
    xi = allreduce_rows(xi, [](R u, R v) { return u + v; });
    Er[k] = (double)xr + sax + (double)E * 0.69314718055994530942;
    Pr[k] = pr;
    Pi[k] = pi;
    Ai[k] = xi;
  }
}

}  // namespace nqs
