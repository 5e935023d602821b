// Shared pieces of the theta contraction: MFMA operand types per precision,
// the B-operand (gathered image) fragments, and the log 2cosh / tanh
// epilogue of one hidden unit (see k_theta.hip for the derivation).
#pragma once

#include "device_common.h"
#include "nqs_internal.h"

namespace nqs {

template <int PREC> struct ThetaTraits;
template <> struct ThetaTraits<NQS_FP64> {
  using R = double;
  using Acc = f64x4;
  using BFrag = double;
  using AFrag = double;
};
template <> struct ThetaTraits<NQS_FP32> {
  using R = float;
  using Acc = f32x4;
  using BFrag = float;
  using AFrag = float;
};
template <> struct ThetaTraits<NQS_BF16X2> {
  using R = float;
  using Acc = f32x4;
  using BFrag = bf16x8;
  using AFrag = bf16x8;
};

template <int N, int PREC> constexpr int nk_of() {
  return PREC == NQS_BF16X2 ? (2 * N + 31) / 32 : N / 4;
}

__device__ __forceinline__ f64x4 mfma(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Working-precision transcendentals.  FP64 uses the accurate library forms.
// FP32 uses the hardware exp2 / log2 / rcp instructions and the sincos below:
// Cody-Waite reduction y = k pi/2 + r, |r| <= pi/4 (pi/2 split into an exact
// float head and a tail), then the Taylor series of sin to r^9 and of cos to
// r^10, whose truncation errors are below 3e-9 on |r| <= pi/4; the quadrant
// k mod 4 rotates (sin r, cos r).  It is accurate to a few ulp for the
// moderate arguments of Im(theta) and, unlike a table-driven library form,
// keeps register pressure low inside the fused kernels.
__device__ __forceinline__ double exp_t(double v) { return exp(v); }
__device__ __forceinline__ float exp_t(float v) { return __expf(v); }
__device__ __forceinline__ void sincos_t(double v, double* s, double* c) { sincos(v, s, c); }
__device__ __forceinline__ void sincos_t(float v, float* s, float* c) {
  const float k = rintf(v * 0.636619772367581343f);             // 2/pi
  float r = fmaf(-k, 1.57079637050628662109375f, v);            // float(pi/2)
  r = fmaf(-k, -4.37113900018624283e-8f, r);                    // pi/2 - float(pi/2)
  const float r2 = r * r;
  const float sp = fmaf(r2, fmaf(r2, fmaf(r2, fmaf(r2, 2.75573192e-6f, -1.98412698e-4f),
                                          8.33333333e-3f), -1.66666667e-1f), 0.0f);
  const float sn = fmaf(r, sp, r);
  const float cs = fmaf(r2, fmaf(r2, fmaf(r2, fmaf(r2, fmaf(r2, -2.75573192e-7f, 2.48015873e-5f),
                                                   -1.38888889e-3f), 4.16666667e-2f), -0.5f),
                        1.0f);
  const int qd = ((int)k) & 3;
  const float s0 = (qd & 1) ? cs : sn;
  const float c0 = (qd & 1) ? sn : cs;
  *s = (qd & 2) ? -s0 : s0;
  *c = ((qd + 1) & 2) ? -c0 : c0;
}
__device__ __forceinline__ double rcp_t(double v) { return 1.0 / v; }
// hardware reciprocal (1 ulp)
__device__ __forceinline__ float rcp_t(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double log_t(double v) { return log(v); }
__device__ __forceinline__ float log_t(float v) { return __logf(v); }
__device__ __forceinline__ double atan2_t(double y, double x) { return atan2(y, x); }
__device__ __forceinline__ float atan2_t(float y, float x) { return atan2f(y, x); }

// Build the B-operand fragments of one 16-image column block.
template <int N, int PREC>
__device__ __forceinline__ void load_bfrag(const int8_t* srow, const uint8_t* prow, int q,
                                           typename ThetaTraits<PREC>::BFrag* bx) {
  constexpr int NK = nk_of<N, PREC>();
  if constexpr (PREC == NQS_BF16X2) {
#pragma unroll
    for (int kk = 0; kk < NK; ++kk) {
      bf16x8 v;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int kap = 32 * kk + 8 * q + e;
        float x = 0.f;
        if (kap < 2 * N) x = 0.5f * (float)srow[prow[kap < N ? kap : kap - N]];
        v[e] = (__bf16)x;
      }
      bx[kk] = v;
    }
  } else {
    using R = typename ThetaTraits<PREC>::R;
#pragma unroll
    for (int kk = 0; kk < NK; ++kk) bx[kk] = R(0.5) * (R)srow[prow[4 * kk + q]];
  }
}

// One hidden unit of the epilogue: with x = Re theta, y = Im theta,
// e = exp(-2|x|), c = (1+e) cos y + i sgn(x)(1-e) sin y = 2cosh(theta) e^{-|x|};
// multiplies c into (pr, pi), adds |x| to sax and, if wanted, returns
// tanh(theta) = (sgn(x)(1-e^2) + i 4 e sin y cos y) / |c|^2.
template <typename R, bool WANT_T>
__device__ __forceinline__ void logcosh_step(R x, R y, R& pr, R& pi, double& sax, R& tr, R& ti) {
  const R ax = x < R(0) ? -x : x;
  const R sg = x < R(0) ? R(-1) : R(1);
  const R e = exp_t(R(-2) * ax);
  R sy, cy;
  sincos_t(y, &sy, &cy);
  const R cr = (R(1) + e) * cy;
  const R ci = sg * (R(1) - e) * sy;
  const R nr = pr * cr - pi * ci;
  pi = pr * ci + pi * cr;
  pr = nr;
  sax += (double)ax;
  if constexpr (WANT_T) {
    const R d = fmaf_t(R(2) * e, cy * cy - sy * sy, fmaf_t(e, e, R(1)));
    const R inv = rcp_t(d);
    tr = sg * (R(1) - e * e) * inv;
    ti = R(4) * e * sy * cy * inv;
  }
}

// Keep a running complex product in range: scale by a power of two.
template <typename R>
__device__ __forceinline__ void renorm(R& pr, R& pi, int& pe) {
  const R m = fmax(fabs(pr), fabs(pi));
  if (m > R(0)) {
    int ex;
    frexp(m, &ex);
    pr = ldexp(pr, -ex);
    pi = ldexp(pi, -ex);
    pe += ex;
  }
}

}  // namespace nqs
