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

// Internal precision tag: FP32 theta on BF16 MFMA from an exact three-term
// BF16 split of W, K axis [W_hi | W_mid | W_lo | 0] against [x | x | x | 0].
// x = +-1/2 is exact in BF16 and W_hi + W_mid + W_lo == W (split3 of the
// FP32 W), so the products are the exact FP32 products and only the FP32
// accumulation rounds -- the numerics of the FP32 MFMA form.
constexpr int kPrecF32X3 = 16;
template <> struct ThetaTraits<kPrecF32X3> {
  using R = float;
  using Acc = f32x4;
  using BFrag = bf16x8;
  using AFrag = bf16x8;
};
// Internal precision tag: the same three-term split with the K slots grouped
// by site.  Lane group q (lanes 16q .. 16q+15) owns sites 4i + q, i < N/4; its
// slots, taken eight per MFMA, are hi and mid of each of its sites in turn,
// then lo of each, then zeros.  A lane then needs x of only N/4 sites (as for
// the 16x16x4 FP32 MFMA) instead of one per slot, and the MFMA count per tile
// is ceil(3 N/4 / 8) (4 at N = 36, against 9 FP32 MFMAs of twice the cycles).
constexpr int kPrecF32S3 = 17;
template <> struct ThetaTraits<kPrecF32S3> {
  using R = float;
  using Acc = f32x4;
  using BFrag = bf16x8;
  using AFrag = bf16x8;
};
// theta runs on 16x16x32 BF16 MFMA; copies of x along the K axis
__host__ __device__ constexpr bool bf16_mfma(int prec) {
  return prec == NQS_BF16X2 || prec == kPrecF32X3 || prec == kPrecF32S3;
}
__host__ __device__ constexpr int x_copies(int prec) { return prec == kPrecF32X3 ? 3 : 2; }

template <int N, int PREC> constexpr int nk_of() {
  if constexpr (PREC == kPrecF32S3) return (3 * (N / 4) + 7) / 8;
  return bf16_mfma(PREC) ? (x_copies(PREC) * N + 31) / 32 : N / 4;
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

// Working-precision transcendentals.  FP64 uses the accurate library forms;
// FP32 uses the hardware exp2 / log2 / rcp instructions and the sine and
// cosine below.
//
// sincos_pi: Cody-Waite reduction by multiples of pi (pi split into the float
// nearest to it and the remainder), y = k pi + r with |r| <= pi/2, then
// sin r = r + r^3 P(r^2) and cos r = 1 + r^2 Q(r^2) with near-minimax P, Q
// fitted on [-pi/2, pi/2] (gen_sincos_coeffs.py; approximation errors 1.7e-8
// and 5e-9, below FP32 rounding).  It returns sin r and cos r, which are
// (-1)^k sin y and (-1)^k cos y; bit 0 of par is toggled by k.  k is rounded
// by adding 1.5 * 2^23, which leaves it in the low mantissa bits, so its
// parity costs one XOR.
__device__ __forceinline__ double exp_t(double v) { return exp(v); }
__device__ __forceinline__ float exp_t(float v) { return __expf(v); }
__device__ __forceinline__ void sincos_pi(float y, float& sn, float& cs, uint32_t& par) {
  const float t = fmaf(y, 0.318309886183790672f, 12582912.0f);   // 1/pi, 1.5 * 2^23
  const float kf = t - 12582912.0f;
  float r = fmaf(-kf, 3.14159274101257324f, y);                   // float(pi)
  r = fmaf(-kf, -8.742278013e-8f, r);                             // pi - float(pi)
  par ^= __float_as_uint(t);
  const float z = r * r;
  const float p = fmaf(fmaf(fmaf(2.600053676e-6f, z, -1.980661473e-4f), z, 8.333017118e-3f), z,
                       -1.666665673e-1f);
  sn = fmaf(r * z, p, r);
  const float qq = fmaf(fmaf(fmaf(fmaf(-2.607709746e-7f, z, 2.476188638e-5f), z,
                                  -1.388840377e-3f), z, 4.166664183e-2f), z, -0.5f);
  cs = fmaf(z, qq, 1.0f);
}
__device__ __forceinline__ void sincos_pi(double y, double& sn, double& cs, uint32_t&) {
  sincos(y, &sn, &cs);
}
__device__ __forceinline__ void sincos_t(double v, double* s, double* c) { sincos(v, s, c); }
__device__ __forceinline__ void sincos_t(float v, float* s, float* c) {
  uint32_t par = 0;
  float sn, cs;
  sincos_pi(v, sn, cs, par);
  *s = (par & 1u) ? -sn : sn;
  *c = (par & 1u) ? -cs : cs;
}
__device__ __forceinline__ double rcp_t(double v) { return 1.0 / v; }
// hardware reciprocal (1 ulp)
__device__ __forceinline__ float rcp_t(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double log_t(double v) { return log(v); }
__device__ __forceinline__ float log_t(float v) { return __logf(v); }
__device__ __forceinline__ double atan2_t(double y, double x) { return atan2(y, x); }
__device__ __forceinline__ float atan2_t(float y, float x) { return atan2f(y, x); }

// Down spins of one configuration as bit masks (bit j set: spin j is down),
// from a vote of the wavefront's lanes over the spin row; x_j = -+1/2 of a
// gathered image is then a shift of the mask.  All 64 lanes must be active.
struct SpinBits {
  uint64_t lo, hi;
};
template <int N>
__device__ __forceinline__ SpinBits spin_bits(const int8_t* srow) {
  const int lane = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
  SpinBits m;
  m.lo = __builtin_amdgcn_ballot_w64(lane < N && srow[lane] < 0);
  m.hi = N > 64 ? __builtin_amdgcn_ballot_w64(lane + 64 < N && srow[lane + 64] < 0) : 0ull;
  return m;
}
// FP32 bit pattern of x = +1/2 (spin up) or -1/2 (down) at site p.
template <int N>
__device__ __forceinline__ uint32_t x_bits(const SpinBits& m, int p) {
  if constexpr (N <= 64) {
    return 0x3F000000u | ((uint32_t)(m.lo >> p) << 31);
  } else {
    const uint64_t w = p < 64 ? m.lo : m.hi;
    return 0x3F000000u | ((uint32_t)(w >> (p & 63)) << 31);
  }
}

// Build the B-operand fragments of one 16-image column block: lane (q, c)
// holds sites 4 kk + q of image c (FP32 / FP64), or for the BF16 forms the K
// positions 32 kk + 8 q + e of [x | x | 0] (split BF16) or [x | x | x | 0].
template <int N, int PREC>
__device__ __forceinline__ SpinBits load_bfrag(const int8_t* srow, const uint8_t* prow, int q,
                                               typename ThetaTraits<PREC>::BFrag* bx) {
  constexpr int NK = nk_of<N, PREC>();
  constexpr int XC = x_copies(PREC);
  const SpinBits m = spin_bits<N>(srow);
  if constexpr (bf16_mfma(PREC)) {
#pragma unroll
    for (int kk = 0; kk < NK; ++kk) {
      uint32_t w[4];
#pragma unroll
      for (int e2 = 0; e2 < 4; ++e2) {
        uint32_t half[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int kap = 32 * kk + 8 * q + 2 * e2 + h;
          half[h] = kap < XC * N ? x_bits<N>(m, prow[kap % N]) : 0u;
        }
        w[e2] = (half[0] >> 16) | (half[1] & 0xffff0000u);   // two BF16, low element first
      }
      bx[kk] = __builtin_bit_cast(bf16x8, w);
    }
  } else {
    using R = typename ThetaTraits<PREC>::R;
#pragma unroll
    for (int kk = 0; kk < NK; ++kk) bx[kk] = (R)__uint_as_float(x_bits<N>(m, prow[4 * kk + q]));
  }
  return m;
}

// B-operand fragments of the site-grouped three-term form (kPrecF32S3) for
// lane (q, c), image c: dword d of MFMA m covers flat slots 8m + 2d and
// 8m + 2d + 1 of lane group q, i.e. (x_i, x_i) for the hi / mid pair of its
// site i, or (x_i, x_i+1) in the lo run.  Also returns, per site 4i + q of the
// lane, x as FP32 (xv) and as a BF16 pair (dx: the same BF16 value in both
// halves), and the spin bits of the row.  N must be a multiple of 4.
template <int N>
__device__ __forceinline__ SpinBits load_bfrag_s3(const int8_t* srow, const uint8_t* prow, int q,
                                                  bf16x8* bx, float* xv, uint32_t* dx) {
  static_assert(N % 4 == 0, "site-grouped fragments need N divisible by 4");
  constexpr int NI = N / 4, NM = nk_of<N, kPrecF32S3>();
  const SpinBits m = spin_bits<N>(srow);
  uint32_t bits[NI];
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    bits[i] = x_bits<N>(m, prow[4 * i + q]);
    xv[i] = __uint_as_float(bits[i]);
    dx[i] = __builtin_amdgcn_perm(bits[i], bits[i], 0x03020302u);
  }
#pragma unroll
  for (int mm = 0; mm < NM; ++mm) {
    uint32_t w[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const int f = 8 * mm + 2 * d;
      if (f < 2 * NI) {
        w[d] = dx[f / 2];
      } else if (f < 3 * NI) {
        const int i = f - 2 * NI;
        w[d] = i + 1 < NI ? pack_hi16(bits[i], bits[i + 1]) : bits[i] >> 16;
      } else {
        w[d] = 0u;
      }
    }
    bx[mm] = __builtin_bit_cast(bf16x8, w);
  }
  return m;
}

// The same fragments gathered byte by byte from the spin row (measured faster
// in the wide E_loc kernel, whose fragments live across long chunk loops).
template <int N, int PREC>
__device__ __forceinline__ void load_bfrag_gather(const int8_t* srow, const uint8_t* prow, int q,
                                                  typename ThetaTraits<PREC>::BFrag* bx) {
  constexpr int NK = nk_of<N, PREC>();
  if constexpr (bf16_mfma(PREC)) {
#pragma unroll
    for (int kk = 0; kk < NK; ++kk) {
      bf16x8 v;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int kap = 32 * kk + 8 * q + e;
        float x = 0.f;
        if (kap < x_copies(PREC) * N) x = 0.5f * (float)srow[prow[kap % N]];
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

// One hidden unit of the epilogue.  With x = Re theta, y = Im theta = k pi + r
// and e = exp(-2|x|):
//   2 cosh(theta) = e^{|x|} (-1)^k c,  c = (1+e) cos r + i sgn(x) (1-e) sin r,
//   tanh(theta)   = (sgn(x)(1-e^2) + i 4 e sin r cos r) / |c|^2
// (both terms of e^{theta} + e^{-theta} change sign together when y moves by
// pi, and tanh has period i pi).  Multiplies c into (pr, pi), toggles bit 0 of
// par by k, returns |x| and, if wanted, tanh(theta).
template <typename R, bool WANT_T>
__device__ __forceinline__ R logcosh_step(R x, R y, R& pr, R& pi, uint32_t& par, R& tr, R& ti) {
  const R ax = fabs(x);
  const R e = exp_t(R(-2) * ax);
  R sn, cs;
  sincos_pi(y, sn, cs, par);
  const R cr = fmaf_t(e, cs, cs);
  const R cu = fmaf_t(-e, sn, sn);
  const R ci = x < R(0) ? -cu : cu;
  const R nr = fmaf_t(pr, cr, -(pi * ci));
  pi = fmaf_t(pr, ci, pi * cr);
  pr = nr;
  if constexpr (WANT_T) {
    const R d = fmaf_t(e + e, fmaf_t(cs, cs, -(sn * sn)), fmaf_t(e, e, R(1)));   // |c|^2
    const R inv = rcp_t(d);
    const R tu = fmaf_t(-e, e, R(1)) * inv;
    tr = x < R(0) ? -tu : tu;
    ti = (R(4) * e) * (sn * cs) * inv;
  }
  return ax;
}

// tanh(x + i y) alone, by the identity above (tanh has period i pi, so the
// reduced angle r suffices): (sgn(x)(1 - e^2) + i 4 e sin r cos r) / |c|^2.
__device__ __forceinline__ void tanh_c(float x, float y, float& tr, float& ti) {
  const float e = exp_t(-2.f * fabsf(x));
  float sn, cs;
  uint32_t par = 0u;
  sincos_pi(y, sn, cs, par);
  const float d = fmaf(e + e, fmaf(cs, cs, -(sn * sn)), fmaf(e, e, 1.f));   // |c|^2
  const float inv = rcp_t(d);
  const float tu = fmaf(-e, e, 1.f) * inv;
  tr = x < 0.f ? -tu : tu;
  ti = (4.f * e) * (sn * cs) * inv;
}

// Apply the collected (-1)^k of the epilogue to a product.
template <typename R>
__device__ __forceinline__ void apply_parity(R& pr, R& pi, uint32_t par) {
  pr = (par & 1u) ? -pr : pr;
  pi = (par & 1u) ? -pi : pi;
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
