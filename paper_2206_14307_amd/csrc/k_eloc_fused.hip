// Fused log psi + E_loc (Sec. 3.1 Eqs. (2), (6); Sec. 3.2 Eq. (10)) for
// models whose hidden layer fits in registers (K*M <= 128).
//
// One wavefront per (sample, 16-image column block): the theta contraction
// runs on 16x16 MFMA exactly as in k_theta.hip, the log 2cosh / tanh
// epilogue leaves tanh(theta) in the MFMA output layout -- lane (q, c) holds
// hidden units 8 ht + 2q, 8 ht + 2q + 1 of image c -- and never goes to HBM.
// Each bond-exchange product F_s prod_h (s + t_h T_h) (sign folding as in
// k_eloc_reg.hip) is split into eight streams, two per q lane of an image;
// each stream starts from a tabulated value (the bond prefactor F_s sits in
// stream 0) and the four q lanes are joined by gfx950 row swaps
// (v_permlane16_swap / v_permlane32_swap), which serve the two bonds of a
// pass at once.  When the parameters allow it (range check at parameter
// upload) the factors are taken in the reciprocal form T_h (t_h + s / T_h):
// the streams start from the product of their T_h and multiply t_h + s U_h,
// 6 VALU operations per factor instead of 8.
//
// The normalisation of the image weights is wave-local: with m a shift common
// to the wave's images, u_kg = chi_g exp(L_kg - m), the wave emits
// (m, sum u, sum_b (J_b/2) sum u R) and a per-sample finish kernel combines
// the column blocks: log psi = M + log sum e^{m-M} den,
// E_loc = diag + sum e^{m-M} Q / sum e^{m-M} den.
//
// Persistent workgroups keep the bond rows and the W fragments in LDS for the
// whole launch; the rows are placed (host side) so that the 16 images of a q
// row read distinct LDS bank groups.
#include "fused_theta.h"

namespace nqs {

namespace {

constexpr int kFusedWaves = 8;

template <int N, int PREC, int K, int M, bool RECIP>
struct FusedCfg {
  using T = ThetaTraits<PREC>;
  using R = typename T::R;
  static constexpr int NB = 4 * N;
  static constexpr int KM = K * M;
  static constexpr int NHT = KM / 8;
  static constexpr int NK = nk_of<N, PREC>();
  // LDS row of bond beta: tanh(D) (direct) or 1/tanh(D) (reciprocal) per
  // hidden unit, then 18 K stream start values, at a host-chosen offset
  static constexpr int ROW = 2 * KM + 18 * K;
  static constexpr int CAP = fused_cap16(NB, fused_row16(K, M, (int)sizeof(R))) * 16 /
                             (int)sizeof(R);
  static constexpr size_t LDS = (size_t)CAP * sizeof(R) +
                                (size_t)NHT * NK * 64 * sizeof(typename T::AFrag) +
                                (size_t)kFusedWaves * NB * 2;
};

// Anti-aligned bonds of the sample: entry b | 0x8000 when s_b = -sigma_p = -1
// for bond (p, q).
__device__ __forceinline__ int fused_list(const int8_t* srow, const int32_t* bonds, int NB,
                                          uint16_t* list, int lane) {
  int n = 0;
  for (int base = 0; base < NB; base += 64) {
    const int b = base + lane;
    bool anti = false;
    int sp = 0;
    if (b < NB) {
      sp = srow[bonds[2 * b]];
      anti = sp != srow[bonds[2 * b + 1]];
    }
    const unsigned long long m = __ballot(anti);
    const int pos = __popcll(m & ((1ull << lane) - 1ull));
    if (anti) list[n + pos] = (uint16_t)(b | (sp > 0 ? 0x8000 : 0));
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

// p *= (t + s U), the reciprocal form of the same factor up to T
template <typename R>
__device__ __forceinline__ void step_rc(R& pr, R& pi, R s, R tr, R ti, R Ur, R Ui) {
  const R a = fmaf_t(s, Ur, tr);
  const R b = fmaf_t(s, Ui, ti);
  const R nr = fmaf_t(pr, a, -(pi * b));
  pi = fmaf_t(pr, b, pi * a);
  pr = nr;
}

// Complex products over the four q rows of two bonds at once: on entry p
// holds bond 0's and o bond 1's per-row partial products; on exit p holds the
// full product of bond 0 in rows 0, 2 and of bond 1 in rows 1, 3.
template <typename R>
__device__ __forceinline__ void qprod_pair(R& pr, R& pi, R orr, R oi) {
  swap16(pr, orr);
  swap16(pi, oi);
  R vr = pr * orr - pi * oi, vi = pr * oi + pi * orr;
  R wr = vr, wi = vi;
  swap32(vr, wr);
  swap32(vi, wi);
  pr = vr * wr - vi * wi;
  pi = vr * wi + vi * wr;
}

template <int N, int PREC, int K, int M, bool RECIP>
__global__ __launch_bounds__(64 * kFusedWaves) void eloc_fused_kernel(
    const int8_t* __restrict__ spins, int64_t S, const uint8_t* __restrict__ perm, int G,
    const typename ThetaTraits<PREC>::AFrag* __restrict__ wfrag,
    const typename ThetaTraits<PREC>::R* __restrict__ bias,
    const typename ThetaTraits<PREC>::R* __restrict__ avec, const int32_t* __restrict__ bonds,
    const int32_t* __restrict__ fmap, const int32_t* __restrict__ frow,
    const double* __restrict__ chi,
    const typename ThetaTraits<PREC>::R* __restrict__ Ttab, double* __restrict__ part) {
  using Cfg = FusedCfg<N, PREC, K, M, RECIP>;
  using T = ThetaTraits<PREC>;
  using R = typename T::R;
  using AF = typename T::AFrag;
  constexpr int NB = Cfg::NB, KM = Cfg::KM, NHT = Cfg::NHT, NK = Cfg::NK;
  constexpr int ROW = Cfg::ROW;
  constexpr int TPR = M / 8;
  __shared__ __align__(16) R Tl[Cfg::CAP];
  __shared__ __align__(16) AF Wl[NHT * NK * 64];
  __shared__ uint16_t lists[kFusedWaves][NB];

  for (int idx = threadIdx.x; idx < NB * ROW; idx += blockDim.x) {
    const int beta = idx / ROW, j = idx % ROW;
    Tl[frow[beta] + j] = Ttab[(size_t)beta * ROW + j];
  }
  for (int idx = threadIdx.x; idx < NHT * NK * 64; idx += blockDim.x) Wl[idx] = wfrag[idx];
  __syncthreads();

  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int q = lane >> 4, c = lane & 15;
  const int cbs = G / 16;
  const int64_t n_items = S * cbs;
  const int64_t stride = (int64_t)gridDim.x * kFusedWaves;
  uint16_t* list = lists[wv];

  for (int64_t item = (int64_t)blockIdx.x * kFusedWaves + wv; item < n_items; item += stride) {
    const int64_t s = item / cbs;
    const int g = (int)(item % cbs) * 16 + c;
    const int8_t* srow = spins + s * N;
    const uint8_t* prow = perm + (size_t)g * N;
    typename T::BFrag bx[NK];
    float axp[2 * K];   // site-grouped form: this lane's partial sums of a . x
    if constexpr (PREC == kPrecF32S3) {
      float xv[N / 4];
      uint32_t dx[N / 4];
      load_bfrag_s3<N>(srow, prow, q, bx, xv, dx);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        float xr = 0.f, xi = 0.f;
#pragma unroll
        for (int i = 0; i < N / 4; ++i) {
          xr = fmaf(xv[i], avec[2 * (k * N + 4 * i + q)], xr);
          xi = fmaf(xv[i], avec[2 * (k * N + 4 * i + q) + 1], xi);
        }
        axp[2 * k] = xr;
        axp[2 * k + 1] = xi;
      }
    } else {
      load_bfrag<N, PREC>(srow, prow, q, bx);
    }
    const int nc = fused_list(srow, bonds, NB, list, lane);

    // ---- theta on MFMA + epilogue: tanh(theta) stays in registers
    R tr[NHT * 2], ti[NHT * 2];
    double Er[K];
    R Pr_[K], Pi_[K], Ai_[K];
    theta_block<N, PREC, K, M>(Wl, bx, bias, avec, srow, prow, lane, tr, ti, Er, Pr_, Pi_, Ai_,
                               axp);
    // u_kg = chi_g exp(L_kg - m) = chi_g e^{Er - m} P e^{i Im a.x}; any common
    // shift m works, the largest Er keeps every u below 4 in magnitude
    double mloc = Er[0];
#pragma unroll
    for (int k = 1; k < K; ++k) mloc = fmax(mloc, Er[k]);
    const double m = wave_max(mloc);
    const R ch = (R)chi[g];
    R ur[K], ui[K];
    double denr = 0.0, deni = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const R e = ch * exp_t((R)(Er[k] - m));
      R sn, cs;
      sincos_t(Ai_[k], &sn, &cs);
      const R zr = Pr_[k] * cs - Pi_[k] * sn, zi = Pr_[k] * sn + Pi_[k] * cs;
      ur[k] = e * zr;
      ui[k] = e * zi;
      denr += (double)ur[k];
      deni += (double)ui[k];
    }

    // ---- bond exchanges, two bonds per pass; the next pass's map entries
    // are loaded one pass ahead
    double Qr[K], Qi[K];
#pragma unroll
    for (int k = 0; k < K; ++k) Qr[k] = Qi[k] = 0.0;
    const int32_t* bm = fmap + (size_t)g * NB;
    int en[2] = {0, 0}, vn[2] = {0, 0};
    if (nc > 0) {
#pragma unroll
      for (int n = 0; n < 2; ++n) {
        en[n] = list[n < nc ? n : 0];
        vn[n] = bm[en[n] & 0x7fff];
      }
    }
    for (int i0 = 0; i0 < nc; i0 += 2) {
      const int e0 = en[0], e1 = en[1], v0 = vn[0], v1 = vn[1];
      if (i0 + 2 < nc) {
#pragma unroll
        for (int n = 0; n < 2; ++n) {
          en[n] = list[i0 + 2 + n < nc ? i0 + 2 + n : i0 + 2];
          vn[n] = bm[en[n] & 0x7fff];
        }
      }
      // s = s_b, flipped when the image bond runs against its table orientation
      const R sg0 = ((e0 >> 15) ^ (v0 & 1)) ? R(-1) : R(1);
      const R sg1 = ((e1 >> 15) ^ (v1 & 1)) ? R(-1) : R(1);
      const R* row0 = Tl + (v0 >> 1);
      const R* row1 = Tl + (v1 >> 1);
      const R* T0 = row0 + 4 * q;
      const R* T1 = row1 + 4 * q;
      const bool valid1 = i0 + 1 < nc;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        // stream starts: (a re, a im, b re, b im) of lane q; stream 0 (q = 0,
        // a) carries F_s, whose s = -1 value is stored after the others
        const R* s0 = row0 + 2 * KM + 16 * k + 4 * q;
        const R* s1 = row1 + 2 * KM + 16 * k + 4 * q;
        const R* n0 = (q == 0 && sg0 < R(0)) ? row0 + 2 * KM + 16 * K + 2 * k : s0;
        const R* n1 = (q == 0 && sg1 < R(0)) ? row1 + 2 * KM + 16 * K + 2 * k : s1;
        R a0r = n0[0], a0i = n0[1], b0r = s0[2], b0i = s0[3];
        R a1r = n1[0], a1i = n1[1], b1r = s1[2], b1i = s1[3];
#pragma unroll
        for (int tt = 0; tt < TPR; ++tt) {
          const int ht = k * TPR + tt;
          R x0[4], x1[4];
          if constexpr (sizeof(R) == 4) {
            const float4 u0 = *reinterpret_cast<const float4*>(T0 + 16 * ht);
            const float4 u1 = *reinterpret_cast<const float4*>(T1 + 16 * ht);
            x0[0] = u0.x; x0[1] = u0.y; x0[2] = u0.z; x0[3] = u0.w;
            x1[0] = u1.x; x1[1] = u1.y; x1[2] = u1.z; x1[3] = u1.w;
          } else {
            const double2 u0 = *reinterpret_cast<const double2*>(T0 + 16 * ht);
            const double2 w0 = *reinterpret_cast<const double2*>(T0 + 16 * ht + 2);
            const double2 u1 = *reinterpret_cast<const double2*>(T1 + 16 * ht);
            const double2 w1 = *reinterpret_cast<const double2*>(T1 + 16 * ht + 2);
            x0[0] = u0.x; x0[1] = u0.y; x0[2] = w0.x; x0[3] = w0.y;
            x1[0] = u1.x; x1[1] = u1.y; x1[2] = w1.x; x1[3] = w1.y;
          }
          if constexpr (RECIP) {
            step_rc<R>(a0r, a0i, sg0, tr[2 * ht], ti[2 * ht], x0[0], x0[1]);
            step_rc<R>(b0r, b0i, sg0, tr[2 * ht + 1], ti[2 * ht + 1], x0[2], x0[3]);
            step_rc<R>(a1r, a1i, sg1, tr[2 * ht], ti[2 * ht], x1[0], x1[1]);
            step_rc<R>(b1r, b1i, sg1, tr[2 * ht + 1], ti[2 * ht + 1], x1[2], x1[3]);
          } else {
            step_sp<R>(a0r, a0i, sg0, tr[2 * ht], ti[2 * ht], x0[0], x0[1]);
            step_sp<R>(b0r, b0i, sg0, tr[2 * ht + 1], ti[2 * ht + 1], x0[2], x0[3]);
            step_sp<R>(a1r, a1i, sg1, tr[2 * ht], ti[2 * ht], x1[0], x1[1]);
            step_sp<R>(b1r, b1i, sg1, tr[2 * ht + 1], ti[2 * ht + 1], x1[2], x1[3]);
          }
        }
        R p0r = a0r * b0r - a0i * b0i, p0i = a0r * b0i + a0i * b0r;
        const R p1r = a1r * b1r - a1i * b1i, p1i = a1r * b1i + a1i * b1r;
        qprod_pair(p0r, p0i, p1r, p1i);
        // rows 0, 2: bond 0; rows 1, 3: bond 1 (absent on an odd tail)
        const bool use = !(q & 1) || valid1;
        Qr[k] += use ? (double)p0r : 0.0;
        Qi[k] += use ? (double)p0i : 0.0;
      }
    }
    // every bond was summed twice (rows 0 and 2, or 1 and 3)
    double qr = 0.0, qi = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      qr += (double)ur[k] * Qr[k] - (double)ui[k] * Qi[k];
      qi += (double)ur[k] * Qi[k] + (double)ui[k] * Qr[k];
    }
    qr *= 0.5;
    qi *= 0.5;
    if (q != 0) {
      denr = 0.0;
      deni = 0.0;
    }
    qr = wave_sum(qr);
    qi = wave_sum(qi);
    denr = wave_sum(denr);
    deni = wave_sum(deni);
    if (lane == 0) {
      double* o = part + item * 6;
      o[0] = m;
      o[1] = denr;
      o[2] = deni;
      o[3] = qr;
      o[4] = qi;
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

template <int N, int PREC, int K, int M, bool RECIP>
hipError_t run(const nqs_ctx* c, const int8_t* spins, int64_t S, double* part, double* logpsi,
               double* eloc, int eloc_stride, hipStream_t st) {
  using T = ThetaTraits<PREC>;
  using R = typename T::R;
  const int cbs = c->G / 16;
  const int64_t items = S * cbs;
  int64_t blocks = (items + kFusedWaves - 1) / kFusedWaves;
  blocks = std::min<int64_t>(blocks, c->n_cu > 0 ? c->n_cu : 256);
  eloc_fused_kernel<N, PREC, K, M, RECIP><<<(unsigned)blocks, 64 * kFusedWaves, 0, st>>>(
      spins, S, c->dev.perm, c->G,
      (const typename T::AFrag*)(PREC == kPrecF32X3   ? c->par.wfrag3
                                 : PREC == kPrecF32S3 ? c->par.wfrag_s3
                                                      : c->par.wfrag),
      (const R*)c->par.bias,
      (const R*)c->par.avec, c->dev.bonds, c->dev.fmap, c->dev.frow, c->dev.chi,
      (const R*)(RECIP ? c->par.Urec : c->par.Tdir), part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  fused_finish_kernel<<<(unsigned)S, 64, 0, st>>>(spins, c->N, c->NB, cbs, c->dev.bonds,
                                                  c->dev.bond_J, part, logpsi, eloc, eloc_stride);
  return hipGetLastError();
}

constexpr size_t kLdsLimit = 160 * 1024;

// The direct form decides whether a model runs fused at all (the workspace
// depends on that, not on the parameters); the reciprocal form runs when its
// range check passed for the current parameters and its table fits in LDS.
template <int N, int PREC, int K, int M>
hipError_t run_if_fits(const nqs_ctx* c, const int8_t* spins, int64_t S, double* part,
                       double* logpsi, double* eloc, int es, hipStream_t st) {
  if constexpr (FusedCfg<N, PREC, K, M, false>::LDS > kLdsLimit) {
    return hipErrorNotSupported;
  } else {
    if constexpr (FusedCfg<N, PREC, K, M, true>::LDS <= kLdsLimit)
      if (c->par.recip_ok && !c->direct_only)
        return run<N, PREC, K, M, true>(c, spins, S, part, logpsi, eloc, es, st);
    return run<N, PREC, K, M, false>(c, spins, S, part, logpsi, eloc, es, st);
  }
}

template <int N, int K, int M>
hipError_t run_prec(const nqs_ctx* c, const int8_t* spins, int64_t S, double* part,
                    double* logpsi, double* eloc, int es, hipStream_t st) {
  switch (c->prec) {
    case NQS_FP64: return run_if_fits<N, NQS_FP64, K, M>(c, spins, S, part, logpsi, eloc, es, st);
    case NQS_FP32:
      // theta from the three-term BF16 split of W (site-grouped) where its
      // fragments fit in LDS
      if constexpr (N % 4 == 0 && FusedCfg<N, kPrecF32S3, K, M, false>::LDS <= kLdsLimit)
        return run_if_fits<N, kPrecF32S3, K, M>(c, spins, S, part, logpsi, eloc, es, st);
      else if constexpr (FusedCfg<N, kPrecF32X3, K, M, false>::LDS <= kLdsLimit)
        return run_if_fits<N, kPrecF32X3, K, M>(c, spins, S, part, logpsi, eloc, es, st);
      else
        return run_if_fits<N, NQS_FP32, K, M>(c, spins, S, part, logpsi, eloc, es, st);
    default: return run_if_fits<N, NQS_BF16X2, K, M>(c, spins, S, part, logpsi, eloc, es, st);
  }
}

template <int N, int K, int M>
bool fits(int prec) {
  switch (prec) {
    case NQS_FP64: return FusedCfg<N, NQS_FP64, K, M, false>::LDS <= kLdsLimit;
    case NQS_FP32: return FusedCfg<N, NQS_FP32, K, M, false>::LDS <= kLdsLimit;
    default: return FusedCfg<N, NQS_BF16X2, K, M, false>::LDS <= kLdsLimit;
  }
}

}  // namespace

hipError_t launch_fused_finish(const nqs_ctx* c, const int8_t* spins, int64_t S,
                               const double* part, double* logpsi, double* eloc, int eloc_stride,
                               hipStream_t st) {
  if (S <= 0) return hipSuccess;
  fused_finish_kernel<<<(unsigned)S, 64, 0, st>>>(spins, c->N, c->NB, c->G / 16, c->dev.bonds,
                                                  c->dev.bond_J, part, logpsi, eloc, eloc_stride);
  return hipGetLastError();
}

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
