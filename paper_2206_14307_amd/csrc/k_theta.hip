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
// Epilogue: with x = Re theta, y = Im theta, e = exp(-2|x|),
//   2 cosh(theta) = exp(|x|) * c,  c = (1+e) cos y + i sgn(x) (1-e) sin y,
//   tanh(theta)   = (sgn(x)(1-e^2) + i 4 e sin y cos y) / |c|^2,
// so sum_h log 2cosh(theta_h) = sum_h |x_h| + log prod_h c_h, with the product
// kept as (mantissa, binary exponent) -- one log/atan2 per (RBM, image)
// instead of one per hidden unit.  sum |x| is accumulated in FP64.
#include "theta_common.h"

namespace nqs {

namespace {

template <int N, int PREC, int CB>
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
    double sax[CB];
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      pr[b] = R(1);
      pi[b] = R(0);
      pe[b] = 0;
      sax[b] = 0.0;
    }
    for (int tt = 0; tt < tiles_per_rbm; ++tt) {
      const int ht = k * tiles_per_rbm + tt;
      typename T::Acc acc[CB];
#pragma unroll
      for (int b = 0; b < CB; ++b) acc[b] = typename T::Acc{0, 0, 0, 0};
      const typename T::AFrag* ap = wfrag + (size_t)ht * NK * 64 + lane;
#pragma unroll
      for (int kk = 0; kk < NK; ++kk) {
        const typename T::AFrag a = ap[kk * 64];
#pragma unroll
        for (int b = 0; b < CB; ++b) acc[b] = mfma(a, bx[b][kk], acc[b]);
      }
      const int h0 = 8 * ht + 2 * q;
      const R b0r = bias[2 * h0], b0i = bias[2 * h0 + 1];
      const R b1r = bias[2 * h0 + 2], b1i = bias[2 * h0 + 3];
#pragma unroll
      for (int b = 0; b < CB; ++b) {
        R tv[4];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const R x = (R)acc[b][2 * u] + (u ? b1r : b0r);
          const R y = (R)acc[b][2 * u + 1] + (u ? b1i : b0i);
          if (t_out)
            logcosh_step<R, true>(x, y, pr[b], pi[b], sax[b], tv[2 * u], tv[2 * u + 1]);
          else
            logcosh_step<R, false>(x, y, pr[b], pi[b], sax[b], tv[2 * u], tv[2 * u + 1]);
        }
        if (t_out && live[b]) {
          R* dst = t_out + ((((size_t)s_of[b] * n_htiles + ht) * G + g_of[b]) * 8 + 2 * q) * 2;
#pragma unroll
          for (int v = 0; v < 4; ++v) dst[v] = tv[v];
        }
      }
      if ((tt & 7) == 7) {
#pragma unroll
        for (int b = 0; b < CB; ++b) renorm(pr[b], pi[b], pe[b]);
      }
    }
    // combine the four lane groups holding different hidden units of one image
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      double Pr = (double)pr[b], Pi = (double)pi[b];
      int E = pe[b];
      double sx = sax[b];
#pragma unroll
      for (int o = 16; o <= 32; o <<= 1) {
        const double orr = __shfl_xor(Pr, o, 64), oi = __shfl_xor(Pi, o, 64);
        const int oe = __shfl_xor(E, o, 64);
        const double os = __shfl_xor(sx, o, 64);
        const double nr = Pr * orr - Pi * oi;
        Pi = Pr * oi + Pi * orr;
        Pr = nr;
        E += oe;
        sx += os;
      }
      // a . (g sigma): sites j = q (mod 4) per lane, then reduce over q
      double axr = 0.0, axi = 0.0;
      const int8_t* srow = spins + s_of[b] * N;
      const uint8_t* prow = perm + (size_t)g_of[b] * N;
      const R* ak = avec + (size_t)k * N * 2;
      for (int j = q; j < N; j += 4) {
        const double xj = 0.5 * (double)srow[prow[j]];
        axr += xj * (double)ak[2 * j];
        axi += xj * (double)ak[2 * j + 1];
      }
      axr += __shfl_xor(axr, 16, 64);
      axi += __shfl_xor(axi, 16, 64);
      axr += __shfl_xor(axr, 32, 64);
      axi += __shfl_xor(axi, 32, 64);
      if (q == 0 && live[b]) {
        const double mag = sqrt(Pr * Pr + Pi * Pi);
        const double lre = axr + sx + log(mag) + (double)E * 0.69314718055994530942;
        const double lim = axi + atan2(Pi, Pr);
        double* o = Lout + (((size_t)s_of[b] * K + k) * G + g_of[b]) * 2;
        o[0] = lre;
        o[1] = lim;
      }
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
  theta_kernel<N, PREC, CB><<<(unsigned)blocks, 256, 0, st>>>(
      spins, S, c->dev.perm, c->G, (const typename T::AFrag*)c->par.wfrag,
      (const R*)c->par.bias, (const R*)c->par.avec, c->K, c->M, c->n_htiles, Lout, (R*)t_out);
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
