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

// W fragments and biases of hidden tile ht for this lane.
template <int PREC, int NK>
__device__ __forceinline__ void load_tile(typename ThetaTraits<PREC>::AFrag (&wf)[NK],
                                          typename ThetaTraits<PREC>::Acc& b0,
                                          const typename ThetaTraits<PREC>::AFrag* wfrag,
                                          const typename ThetaTraits<PREC>::R* bias, int ht,
                                          int lane, int q) {
  const typename ThetaTraits<PREC>::AFrag* ap = wfrag + (size_t)ht * NK * 64 + lane;
#pragma unroll
  for (int kk = 0; kk < NK; ++kk) wf[kk] = ap[kk * 64];
  const int h0 = 8 * ht + 2 * q;
#pragma unroll
  for (int v = 0; v < 4; ++v) b0[v] = bias[2 * h0 + v];
}

// theta of one hidden tile for the CB column blocks: accumulators start from
// the biases.
template <int PREC, int CB, int NK>
__device__ __forceinline__ void mfma_tile(typename ThetaTraits<PREC>::Acc (&acc)[CB],
                                          const typename ThetaTraits<PREC>::AFrag (&wf)[NK],
                                          const typename ThetaTraits<PREC>::Acc& b0,
                                          const typename ThetaTraits<PREC>::BFrag (&bx)[CB][NK]) {
#pragma unroll
  for (int b = 0; b < CB; ++b) acc[b] = b0;
#pragma unroll
  for (int kk = 0; kk < NK; ++kk)
#pragma unroll
    for (int b = 0; b < CB; ++b) acc[b] = mfma(wf[kk], bx[b][kk], acc[b]);
}

// Epilogue of one hidden tile (two units per lane and column block).
template <int PREC, int CB, bool WANT_T>
__device__ __forceinline__ void epi_tile(const typename ThetaTraits<PREC>::Acc (&acc)[CB],
                                              typename ThetaTraits<PREC>::R (&pr)[CB],
                                              typename ThetaTraits<PREC>::R (&pi)[CB],
                                              uint32_t (&par)[CB], double (&sax)[CB],
                                              typename ThetaTraits<PREC>::R* t_out,
                                              const int64_t (&s_of)[CB], const int (&g_of)[CB],
                                              const bool (&live)[CB], int ht, int n_htiles,
                                              int G, int q) {
  using R = typename ThetaTraits<PREC>::R;
#pragma unroll
  for (int b = 0; b < CB; ++b) {
    R tv[4];
    const R ax0 = logcosh_step<R, WANT_T>((R)acc[b][0], (R)acc[b][1], pr[b], pi[b],
                                                  par[b], tv[0], tv[1]);
    const R ax1 = logcosh_step<R, WANT_T>((R)acc[b][2], (R)acc[b][3], pr[b], pi[b],
                                                  par[b], tv[2], tv[3]);
    sax[b] += (double)(ax0 + ax1);
    if constexpr (WANT_T) {
      if (live[b]) {
        R* dst = t_out + ((((size_t)s_of[b] * n_htiles + ht) * G + g_of[b]) * 8 + 2 * q) * 2;
#pragma unroll
        for (int v = 0; v < 4; ++v) dst[v] = tv[v];
      }
    }
  }
}

// Rows q = lane / 16 hold v[b] for the column blocks b < CB (CB = 4 or 2); on
// exit row q holds the combination over all four rows of v[q mod CB].  Two
// row swaps (v_permlane16_swap, v_permlane32_swap) serve all column blocks.
template <int CB, typename V, typename Op>
__device__ __forceinline__ V join_rows(const V (&v)[CB], Op op) {
  V x0 = v[0], y0 = v[1];
  swap16(x0, y0);
  V a = op(x0, y0);
  if constexpr (CB == 4) {
    V x1 = v[2], y1 = v[3];
    swap16(x1, y1);
    V bb = op(x1, y1);
    swap32(a, bb);
    return op(a, bb);
  } else {
    V bb = a;
    swap32(a, bb);
    return op(a, bb);
  }
}
// The same for complex products.
template <int CB, typename R>
__device__ __forceinline__ void join_rows_cmul(const R (&vr)[CB], const R (&vi)[CB], R& outr,
                                               R& outi) {
  auto cm = [](R& ar, R& ai, R br, R bi) {
    const R nr = ar * br - ai * bi;
    ai = ar * bi + ai * br;
    ar = nr;
  };
  R xr = vr[0], yr = vr[1], xi = vi[0], yi = vi[1];
  swap16(xr, yr);
  swap16(xi, yi);
  cm(xr, xi, yr, yi);
  R br, bi;
  if constexpr (CB == 4) {
    R ur = vr[2], wr = vr[3], ui = vi[2], wi = vi[3];
    swap16(ur, wr);
    swap16(ui, wi);
    cm(ur, ui, wr, wi);
    br = ur;
    bi = ui;
  } else {
    br = xr;
    bi = xi;
  }
  swap32(xr, br);
  swap32(xi, bi);
  cm(xr, xi, br, bi);
  outr = xr;
  outi = xi;
}

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
  // column blocks wave*CB .. wave*CB + CB - 1 (wave-uniform; one division)
  const int64_t wave =
      (int64_t)blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int cb_per_s = G / 16;
  const int64_t total_cb = S * cb_per_s;
  if (wave * CB >= total_cb) return;

  typename T::BFrag bx[CB][NK];
  SpinBits sb[CB];
  int64_t s_of[CB];
  int g_of[CB];
  bool live[CB];
  {
    int64_t sc = (wave * CB) / cb_per_s;
    int gb = (int)(wave * CB - sc * cb_per_s);
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      live[b] = wave * CB + b < total_cb;
      s_of[b] = live[b] ? sc : 0;
      g_of[b] = (live[b] ? gb : 0) * 16 + c;
      if constexpr (PREC == kPrecF32S3) {
        float xv[N / 4];
        uint32_t dx[N / 4];
        sb[b] = load_bfrag_s3<N>(spins + s_of[b] * N, perm + (size_t)g_of[b] * N, q, bx[b], xv,
                                 dx);
      } else {
        sb[b] = load_bfrag<N, PREC>(spins + s_of[b] * N, perm + (size_t)g_of[b] * N, q, bx[b]);
      }
      if (++gb == cb_per_s) {
        gb = 0;
        ++sc;
      }
    }
  }

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
    // Larger lattices (N > 36, longer MFMA chains per tile) software-pipeline
    // the tile loop: the next tile's MFMAs and fragment loads are issued before
    // the current epilogue.  At N <= 36, and for the site-grouped FP32 form at
    // any N (short MFMA chains: 10 BF16 MFMAs a tile at N = 100), the plain
    // loop, with fewer live registers, is faster.
    if constexpr (N <= 36 || PREC == kPrecF32S3) {
      for (int tt = 0; tt < tiles_per_rbm; ++tt) {
        const int ht = k * tiles_per_rbm + tt;
        typename T::AFrag wf[NK];
        typename T::Acc b0, acc[CB];
        load_tile<PREC, NK>(wf, b0, wfrag, bias, ht, lane, q);
        mfma_tile<PREC, CB, NK>(acc, wf, b0, bx);
        epi_tile<PREC, CB, WANT_T>(acc, pr, pi, par, sax, t_out, s_of, g_of, live, ht, n_htiles,
                                   G, q);
        if ((tt & 7) == 7) {
#pragma unroll
          for (int b = 0; b < CB; ++b) renorm(pr[b], pi[b], pe[b]);
        }
      }
    } else {
      // Software pipeline over the RBM's hidden tiles: the MFMAs of tile tt+1
      // are issued (into the other accumulator set) before the epilogue of tile
      // tt, and the fragments of tile tt+2 are loaded meanwhile.  Buffers A / B
      // alternate between even and odd tiles.
      const int T0 = k * tiles_per_rbm, TL = T0 + tiles_per_rbm - 1;
      typename T::AFrag wfA[NK], wfB[NK];
      typename T::Acc bA, bB, accA[CB], accB[CB];
      load_tile<PREC, NK>(wfA, bA, wfrag, bias, T0, lane, q);
      load_tile<PREC, NK>(wfB, bB, wfrag, bias, min(T0 + 1, TL), lane, q);
      mfma_tile<PREC, CB, NK>(accA, wfA, bA, bx);
      load_tile<PREC, NK>(wfA, bA, wfrag, bias, min(T0 + 2, TL), lane, q);
      int ht = T0;
      for (; ht + 2 <= TL; ht += 2) {
        mfma_tile<PREC, CB, NK>(accB, wfB, bB, bx);                       // tile ht+1
        epi_tile<PREC, CB, WANT_T>(accA, pr, pi, par, sax, t_out, s_of, g_of, live, ht, n_htiles,
                                   G, q);
        load_tile<PREC, NK>(wfB, bB, wfrag, bias, min(ht + 3, TL), lane, q);
        __builtin_amdgcn_sched_barrier(0);
        mfma_tile<PREC, CB, NK>(accA, wfA, bA, bx);                       // tile ht+2
        epi_tile<PREC, CB, WANT_T>(accB, pr, pi, par, sax, t_out, s_of, g_of, live, ht + 1,
                                   n_htiles, G, q);
        load_tile<PREC, NK>(wfA, bA, wfrag, bias, min(ht + 4, TL), lane, q);
        __builtin_amdgcn_sched_barrier(0);
        if (((ht - T0) & 7) == 6) {
  #pragma unroll
          for (int b = 0; b < CB; ++b) renorm(pr[b], pi[b], pe[b]);
        }
      }
      if (ht + 1 <= TL) {
        mfma_tile<PREC, CB, NK>(accB, wfB, bB, bx);
        epi_tile<PREC, CB, WANT_T>(accA, pr, pi, par, sax, t_out, s_of, g_of, live, ht, n_htiles,
                                   G, q);
        epi_tile<PREC, CB, WANT_T>(accB, pr, pi, par, sax, t_out, s_of, g_of, live, ht + 1,
                                   n_htiles, G, q);
      } else {
        epi_tile<PREC, CB, WANT_T>(accA, pr, pi, par, sax, t_out, s_of, g_of, live, ht, n_htiles,
                                   G, q);
      }
    }

    // a . (g sigma), per lane over its sites, for every column block
    R axr[CB], axi[CB];
#pragma unroll
    for (int b = 0; b < CB; ++b) axr[b] = axi[b] = R(0);
    const R* ak = avec + (size_t)k * N * 2;
    if constexpr (!bf16_mfma(PREC)) {
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
        const uint8_t* prow = perm + (size_t)g_of[b] * N;
#pragma unroll
        for (int jj = 0; jj < (N + 3) / 4; ++jj) {
          const int j = 4 * jj + q;
          if (j < N) {
            const R xj = __uint_as_float(x_bits<N>(sb[b], prow[j]));
            axr[b] = fmaf_t(xj, ak[2 * j], axr[b]);
            axi[b] = fmaf_t(xj, ak[2 * j + 1], axi[b]);
          }
        }
      }
    }

    // join the four lane groups; lane group q keeps column block q mod CB
    R jpr[CB], jpi[CB];
    int E[CB];
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      renorm(pr[b], pi[b], pe[b]);
      apply_parity(pr[b], pi[b], par[b]);
      jpr[b] = pr[b];
      jpi[b] = pi[b];
      E[b] = pe[b];
    }
    R Pj, Qj;
    join_rows_cmul<CB>(jpr, jpi, Pj, Qj);
    const int Es = join_rows<CB>(E, [](int u, int v) { return u + v; });
    const double sx = join_rows<CB>(sax, [](double u, double v) { return u + v; });
    const R xr = join_rows<CB>(axr, [](R u, R v) { return u + v; });
    const R xi = join_rows<CB>(axi, [](R u, R v) { return u + v; });
    const int bs = q & (CB - 1);
    int64_t s_sel = s_of[0];
    int g_sel = g_of[0];
    bool live_sel = live[0];
#pragma unroll
    for (int b = 1; b < CB; ++b)
      if (bs == b) {
        s_sel = s_of[b];
        g_sel = g_of[b];
        live_sel = live[b];
      }
    double Lre = (double)xr + sx, Lim = (double)xi;
    const double Ps = (double)Pj, Qs = (double)Qj;
    // log and arg of the joined product (FP32 precisions: of its mantissa in
    // [1/2, 1), in FP32)
    if constexpr (PREC == NQS_FP64) {
      Lre += log(sqrt(Ps * Ps + Qs * Qs)) + (double)Es * 0.69314718055994530942;
      Lim += atan2(Qs, Ps);
    } else {
      int ex = 0;
      const double mx = fmax(fabs(Ps), fabs(Qs));
      if (mx > 0.0) frexp(mx, &ex);
      const float pm = (float)ldexp(Ps, -ex), qm = (float)ldexp(Qs, -ex);
      const float lg = 0.5f * __log2f(fmaf(pm, pm, qm * qm));
      Lre += ((double)lg + (double)(Es + ex)) * 0.69314718055994530942;
      Lim += (double)atan2f(qm, pm);
    }
    if (q < CB && live_sel) {
      double* o = Lout + (((size_t)s_sel * K + k) * G + g_sel) * 2;
      o[0] = Lre;
      o[1] = Lim;
    }
  }
}

// Per-sample log-sum-exp over (k, g): log psi = m + log sum chi_g exp(L - m);
// the normalised image weights w = chi_g exp(L - log psi) feed E_loc and O_k.
// One wavefront per sample (shuffle reductions, no barriers), FP64 throughout.
// RAW: L unreduced as the wide E_loc kernel writes it, four reals per image
// (E, b, p, q) with L = E + log|p + i q| + i (b + arg(p + i q)).
template <bool RAW>
__device__ __forceinline__ double2 lse_L(const double* Ls, int i) {
  if constexpr (RAW) {
    const double p = Ls[4 * i + 2], q = Ls[4 * i + 3];
    return make_double2(Ls[4 * i] + 0.5 * log(p * p + q * q), Ls[4 * i + 1] + atan2(q, p));
  } else {
    return make_double2(Ls[2 * i], Ls[2 * i + 1]);
  }
}

template <typename R, bool RAW>
__global__ __launch_bounds__(256) void lse_kernel(const double* __restrict__ L, int64_t S, int KG,
                                                  int G, const double* __restrict__ chi,
                                                  double* __restrict__ logpsi, R* __restrict__ w) {
  const int64_t s = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= S) return;
  const int lane = threadIdx.x & 63;
  const double* Ls = L + (size_t)s * KG * (RAW ? 4 : 2);
  double m = -INFINITY;
  for (int i = lane; i < KG; i += 64) m = fmax(m, lse_L<RAW>(Ls, i).x);
  m = wave_max(m);
  double sr = 0.0, si = 0.0;
  for (int i = lane; i < KG; i += 64) {
    const double2 l = lse_L<RAW>(Ls, i);
    const double e = chi[i % G] * exp(l.x - m);
    double sn, cs;
    sincos(l.y, &sn, &cs);
    sr = fma(e, cs, sr);
    si = fma(e, sn, si);
  }
  sr = wave_sum(sr);
  si = wave_sum(si);
  const double lre = m + 0.5 * log(sr * sr + si * si);
  const double lim = atan2(si, sr);
  if (lane == 0) {
    logpsi[2 * s] = lre;
    logpsi[2 * s + 1] = lim;
  }
  if (w) {
    R* ws = w + (size_t)s * KG * 2;
    for (int i = lane; i < KG; i += 64) {
      const double2 l = lse_L<RAW>(Ls, i);
      const double e = chi[i % G] * exp(l.x - lre);
      double sn, cs;
      sincos(l.y - lim, &sn, &cs);
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
  // column blocks per wave: 4 for FP32 / FP64 at N <= 36, otherwise 2 (fewer
  // live registers where the fragments or the MFMA chains are longer)
  constexpr int CB = (N <= 36 && !bf16_mfma(PREC)) ? 4 : 2;
  const void* wf = PREC == kPrecF32X3   ? c->par.wfrag3
                   : PREC == kPrecF32S3 ? c->par.wfrag_s3
                                        : c->par.wfrag;
  if (!wf) return hipErrorInvalidValue;
  const int64_t total_cb = S * (c->G / 16);
  const int64_t waves = (total_cb + CB - 1) / CB;
  const int64_t blocks = (waves + 3) / 4;
  if (t_out)
    theta_kernel<N, PREC, CB, true><<<(unsigned)blocks, 256, 0, st>>>(
        spins, S, c->dev.perm, c->G, (const typename T::AFrag*)wf,
        (const R*)c->par.bias, (const R*)c->par.avec, c->K, c->M, c->n_htiles, Lout, (R*)t_out);
  else
    theta_kernel<N, PREC, CB, false><<<(unsigned)blocks, 256, 0, st>>>(
        spins, S, c->dev.perm, c->G, (const typename T::AFrag*)wf,
        (const R*)c->par.bias, (const R*)c->par.avec, c->K, c->M, c->n_htiles, Lout, nullptr);
  return hipGetLastError();
}

template <int N>
hipError_t theta_prec(const nqs_ctx* c, const int8_t* spins, int64_t S, double* Lout, void* t_out,
                      hipStream_t st) {
  switch (c->prec) {
    case NQS_FP64: return theta_for<N, NQS_FP64>(c, spins, S, Lout, t_out, st);
    // FP32 models: theta from the three-term BF16 split of W (FP32 numerics),
    // site-grouped (at 8x8 and 10x10 2.1-2.4x faster than FP32 MFMA)
    case NQS_FP32:
      if constexpr (N % 4 == 0) return theta_for<N, kPrecF32S3>(c, spins, S, Lout, t_out, st);
      else if constexpr (N <= 36) return theta_for<N, kPrecF32X3>(c, spins, S, Lout, t_out, st);
      else return theta_for<N, NQS_FP32>(c, spins, S, Lout, t_out, st);
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
                      void* w_out, hipStream_t st, bool raw) {
  if (S <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((S + 3) / 4);
  const int KG = c->K * c->G;
  if (c->prec == NQS_FP64)
    lse_kernel<double, false><<<blocks, 256, 0, st>>>(L, S, KG, c->G, c->dev.chi, logpsi_out,
                                                      (double*)w_out);
  else if (raw)
    lse_kernel<float, true><<<blocks, 256, 0, st>>>(L, S, KG, c->G, c->dev.chi, logpsi_out,
                                                    (float*)w_out);
  else
    lse_kernel<float, false><<<blocks, 256, 0, st>>>(L, S, KG, c->G, c->dev.chi, logpsi_out,
                                                     (float*)w_out);
  return hipGetLastError();
}

}  // namespace nqs
