// theta GEMM + log 2cosh epilogue + log-sum-exp over symmetry images.
//
// For every configuration sigma and symmetry image g (Sec. 3.1, Eq. (6)),
// theta_h = sum_j W_hj (g sigma)_j + b_h (Eq. (2)) is one dense contraction
// (samples x images) x N x (K M), run on MFMA: the A operand is W with its
// real and imaginary rows interleaved (row 2h = Re W_h, row 2h+1 = Im W_h),
// the B operand is the gathered image x = sigma[perm_g(.)] = +-1/2, built in
// registers from the spin row and the permutation table.  One 16x16 output
// tile covers 8 hidden units x 16 images; lane (q = l/16, c = l%16) receives
// Re/Im theta of hidden units 8 ht + 2q, 8 ht + 2q + 1 for image c, so the
// epilogue is lane-local.
//
// Epilogue (theta_common.h): with x = Re theta, y = Im theta = k pi + r,
// e = exp(-2|x|),
//   2 cosh(theta) = exp(|x|) (-1)^k c,  c = (1+e) cos r + i sgn(x) (1-e) sin r,
//   tanh(theta)   = (sgn(x)(1-e^2) + i 4 e sin r cos r) / |c|^2,
// so sum_h log 2cosh(theta_h) = sum_h |x_h| + log((-1)^{sum k} prod_h c_h), with
// the product kept as (mantissa, binary exponent) -- one log/atan2 per (RBM,
// image) instead of one per hidden unit.  The accumulators start from the
// biases; sum |x| is added in FP64 once per tile (two units per lane).
//
// After the last tile of an RBM the four lane groups q (different hidden
// units of one image) are joined with shuffles; a.(g sigma) comes from the B
// fragments already in registers (FP32 / FP64: lane q holds x_j for
// j = q mod 4).  Lane group q then finishes column block q mod CB, so each
// lane evaluates one log and one atan2.
#include "theta_common.h"

namespace nqs {

namespace {

template <int N, int PREC, int CB, bool WANT_T>
__global__ __launch_bounds__(256) void theta_kernel(
    const int8_t* __restrict__ spins, int64_t S, const uint8_t* __restrict__ perm, int G,
    const typename ThetaTraits<PREC>::AFrag* __restrict__ wfrag,
    const typename ThetaTraits<PREC>::R* __restrict__ bias,
    const typename ThetaTraits<PREC>::R* __restrict__ avec, int K, int M, int n_htiles,
    double* __restrict__ Lout, typename ThetaTraits<PREC>::R* __restrict__ t_out) {
  using T = ThetaTraits<PREC>;
  using R = typename T::R;
  constexpr int NK = nk_of<N, PREC>();
  const int lane = threadIdx.x & 63;
  const int q = lane >> 4, c = lane & 15;
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int cb_per_s = G / 16;
  const int64_t total_cb = S * cb_per_s;

  typename T::BFrag bx[CB][NK];
  int64_t s_of[CB];
  int g_of[CB];
  bool live[CB];
#pragma unroll
  for (int b = 0; b < CB; ++b) {
    const int64_t cbi = wave * CB + b;
    live[b] = cbi < total_cb;
    const int64_t cbc = live[b] ? cbi : 0;
    s_of[b] = cbc / cb_per_s;
    g_of[b] = (int)(cbc % cb_per_s) * 16 + c;
    load_bfrag<N, PREC>(spins + s_of[b] * N, perm + (size_t)g_of[b] * N, q, bx[b]);
  }
  if (!live[0]) return;  // whole wave idle (live[0] is wave-uniform)

  const int tiles_per_rbm = M / 8;
  for (int k = 0; k < K; ++k) {
    R pr[CB], pi[CB];
    int pe[CB];
    uint32_t par[CB];
    double sax[CB];
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      pr[b] = R(1);
      pi[b] = R(0);
      pe[b] = 0;
      par[b] = 0u;
      sax[b] = 0.0;
    }
    for (int tt = 0; tt < tiles_per_rbm; ++tt) {
      const int ht = k * tiles_per_rbm + tt;
      const int h0 = 8 * ht + 2 * q;
      typename T::Acc b0;
#pragma unroll
      for (int v = 0; v < 4; ++v) b0[v] = bias[2 * h0 + v];
      typename T::Acc acc[CB];
#pragma unroll
      for (int b = 0; b < CB; ++b) acc[b] = b0;
      const typename T::AFrag* ap = wfrag + (size_t)ht * NK * 64 + lane;
#pragma unroll
      for (int kk = 0; kk < NK; ++kk) {
        const typename T::AFrag a = ap[kk * 64];
#pragma unroll
        for (int b = 0; b < CB; ++b) acc[b] = mfma(a, bx[b][kk], acc[b]);
      }
#pragma unroll
      for (int b = 0; b < CB; ++b) {
        R tv[4];
        const R ax0 = logcosh_step<R, WANT_T>((R)acc[b][0], (R)acc[b][1], pr[b], pi[b], par[b],
                                              tv[0], tv[1]);
        const R ax1 = logcosh_step<R, WANT_T>((R)acc[b][2], (R)acc[b][3], pr[b], pi[b], par[b],
                                              tv[2], tv[3]);
        sax[b] += (double)(ax0 + ax1);
        if constexpr (WANT_T) {
          if (live[b]) {
            R* dst = t_out + ((((size_t)s_of[b] * n_htiles + ht) * G + g_of[b]) * 8 + 2 * q) * 2;
#pragma unroll
            for (int v = 0; v < 4; ++v) dst[v] = tv[v];
          }
        }
      }
      if ((tt & 7) == 7) {
#pragma unroll
        for (int b = 0; b < CB; ++b) renorm(pr[b], pi[b], pe[b]);
      }
    }

    // a . (g sigma), per lane over its sites, for every column block
    R axr[CB], axi[CB];
#pragma unroll
    for (int b = 0; b < CB; ++b) axr[b] = axi[b] = R(0);
    const R* ak = avec + (size_t)k * N * 2;
    if constexpr (PREC != NQS_BF16X2) {
#pragma unroll
      for (int kk = 0; kk < NK; ++kk) {
        const R ar = ak[2 * (4 * kk + q)], ai = ak[2 * (4 * kk + q) + 1];
#pragma unroll
        for (int b = 0; b < CB; ++b) {
          axr[b] = fmaf_t(bx[b][kk], ar, axr[b]);
          axi[b] = fmaf_t(bx[b][kk], ai, axi[b]);
        }
      }
    } else {
#pragma unroll
      for (int b = 0; b < CB; ++b) {
        const int8_t* srow = spins + s_of[b] * N;
        const uint8_t* prow = perm + (size_t)g_of[b] * N;
        for (int j = q; j < N; j += 4) {
          const R xj = R(0.5) * (R)srow[prow[j]];
          axr[b] = fmaf_t(xj, ak[2 * j], axr[b]);
          axi[b] = fmaf_t(xj, ak[2 * j + 1], axi[b]);
        }
      }
    }

    // join the four lane groups; lane group q keeps column block q mod CB
    double Lre = 0.0, Lim = 0.0, Ps = 1.0, Qs = 0.0;
    int64_t s_sel = 0;
    int g_sel = 0;
    bool live_sel = false;
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      renorm(pr[b], pi[b], pe[b]);
      apply_parity(pr[b], pi[b], par[b]);
      double Pr = (double)pr[b], Pi = (double)pi[b];
      int E = pe[b];
      double sx = sax[b];
      R xr = axr[b], xi = axi[b];
#pragma unroll
      for (int o = 16; o <= 32; o <<= 1) {
        const double orr = __shfl_xor(Pr, o, 64), oi = __shfl_xor(Pi, o, 64);
        const double nr = Pr * orr - Pi * oi;
        Pi = Pr * oi + Pi * orr;
        Pr = nr;
        E += __shfl_xor(E, o, 64);
        sx += __shfl_xor(sx, o, 64);
        xr += __shfl_xor(xr, o, 64);
        xi += __shfl_xor(xi, o, 64);
      }
      if ((q & (CB - 1)) == b) {
        Lre = (double)xr + sx + (double)E * 0.69314718055994530942;
        Lim = (double)xi;
        Ps = Pr;
        Qs = Pi;
        s_sel = s_of[b];
        g_sel = g_of[b];
        live_sel = live[b];
      }
    }
    if (q < CB && live_sel) {
      double* o = Lout + (((size_t)s_sel * K + k) * G + g_sel) * 2;
      o[0] = Lre + log(sqrt(Ps * Ps + Qs * Qs));
      o[1] = Lim + atan2(Qs, Ps);
    }
  }
}

// Per-sample log-sum-exp over (k, g): log psi = m + log sum chi_g exp(L - m);
// the normalised image weights w = chi_g exp(L - log psi) feed E_loc and O_k.
template <typename R>
__global__ __launch_bounds__(256) void lse_kernel(const double* __restrict__ L, int KG, int G,
                                                  const double* __restrict__ chi,
                                                  double* __restrict__ logpsi, R* __restrict__ w) {
  const int64_t s = blockIdx.x;
  const double* Ls = L + (size_t)s * KG * 2;
  __shared__ double red[2][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double m = -INFINITY;
  for (int i = threadIdx.x; i < KG; i += blockDim.x) m = fmax(m, Ls[2 * i]);
  m = wave_max(m);
  if (lane == 0) red[0][wv] = m;
  __syncthreads();
  m = fmax(fmax(red[0][0], red[0][1]), fmax(red[0][2], red[0][3]));
  __syncthreads();
  double sr = 0.0, si = 0.0;
  for (int i = threadIdx.x; i < KG; i += blockDim.x) {
    const double ch = chi[i % G];
    const double e = ch * exp(Ls[2 * i] - m);
    double sn, cs;
    sincos(Ls[2 * i + 1], &sn, &cs);
    sr += e * cs;
    si += e * sn;
  }
  sr = wave_sum(sr);
  si = wave_sum(si);
  if (lane == 0) {
    red[0][wv] = sr;
    red[1][wv] = si;
  }
  __syncthreads();
  sr = red[0][0] + red[0][1] + red[0][2] + red[0][3];
  si = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  const double lre = m + 0.5 * log(sr * sr + si * si);
  const double lim = atan2(si, sr);
  if (threadIdx.x == 0) {
    logpsi[2 * s] = lre;
    logpsi[2 * s + 1] = lim;
  }
  if (w) {
    R* ws = w + (size_t)s * KG * 2;
    for (int i = threadIdx.x; i < KG; i += blockDim.x) {
      const double ch = chi[i % G];
      const double e = ch * exp(Ls[2 * i] - lre);
      double sn, cs;
      sincos(Ls[2 * i + 1] - lim, &sn, &cs);
      ws[2 * i] = (R)(e * cs);
      ws[2 * i + 1] = (R)(e * sn);
    }
  }
}

template <int N, int PREC>
hipError_t theta_for(const nqs_ctx* c, const int8_t* spins, int64_t S, double* Lout, void* t_out,
                     hipStream_t st) {
  using T = ThetaTraits<PREC>;
  using R = typename T::R;
  constexpr int CB = N <= 36 ? 4 : 2;
  const int64_t total_cb = S * (c->G / 16);
  const int64_t waves = (total_cb + CB - 1) / CB;
  const int64_t blocks = (waves + 3) / 4;
  if (t_out)
    theta_kernel<N, PREC, CB, true><<<(unsigned)blocks, 256, 0, st>>>(
        spins, S, c->dev.perm, c->G, (const typename T::AFrag*)c->par.wfrag,
        (const R*)c->par.bias, (const R*)c->par.avec, c->K, c->M, c->n_htiles, Lout, (R*)t_out);
  else
    theta_kernel<N, PREC, CB, false><<<(unsigned)blocks, 256, 0, st>>>(
        spins, S, c->dev.perm, c->G, (const typename T::AFrag*)c->par.wfrag,
        (const R*)c->par.bias, (const R*)c->par.avec, c->K, c->M, c->n_htiles, Lout, nullptr);
  return hipGetLastError();
}

template <int N>
hipError_t theta_prec(const nqs_ctx* c, const int8_t* spins, int64_t S, double* Lout, void* t_out,
                      hipStream_t st) {
  switch (c->prec) {
    case NQS_FP64: return theta_for<N, NQS_FP64>(c, spins, S, Lout, t_out, st);
    case NQS_FP32: return theta_for<N, NQS_FP32>(c, spins, S, Lout, t_out, st);
    default: return theta_for<N, NQS_BF16X2>(c, spins, S, Lout, t_out, st);
  }
}

}  // namespace

hipError_t launch_theta(const nqs_ctx* c, const int8_t* spins, int64_t S, double* Lout,
                        void* t_out, hipStream_t st) {
  switch (c->L) {
    case 4: return theta_prec<16>(c, spins, S, Lout, t_out, st);
    case 6: return theta_prec<36>(c, spins, S, Lout, t_out, st);
    case 8: return theta_prec<64>(c, spins, S, Lout, t_out, st);
    default: return theta_prec<100>(c, spins, S, Lout, t_out, st);
  }
}

hipError_t launch_lse(const nqs_ctx* c, const double* L, int64_t S, double* logpsi_out,
                      void* w_out, hipStream_t st) {
  if (S <= 0) return hipSuccess;
  if (c->prec == NQS_FP64)
    lse_kernel<double><<<(unsigned)S, 256, 0, st>>>(L, c->K * c->G, c->G, c->dev.chi, logpsi_out,
                                                    (double*)w_out);
  else
    lse_kernel<float><<<(unsigned)S, 256, 0, st>>>(L, c->K * c->G, c->G, c->dev.chi, logpsi_out,
                                                   (float*)w_out);
  return hipGetLastError();
}

}  // namespace nqs
