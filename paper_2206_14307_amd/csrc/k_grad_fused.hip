// Fused log-derivatives O_k = d log psi / d theta_k (Sec. 3.2, below
// Eq. (12)) for models whose hidden layer fits one wavefront (K*M <= 128),
// with theta of FP32 models on BF16 MFMA from the exact site-grouped
// three-term split of W (FP32 products, FP32 accumulation), of BF16X2 models
// in split BF16, and everything else in FP32.
//
// With u_kg = chi_g psi_s^(k)(g sigma) / e^m (any common shift m), the image
// x_g = g sigma and t = tanh(theta):
//   O_W[k][h][j] = sum_g u_kg t_kgh x_gj / D,  O_b[k][h] = sum_g u_kg t_kgh / D,
//   O_a[k][j]    = sum_g u_kg x_gj / D,        D = sum_kg u_kg,
// and log psi = m + log D.
//
// One wavefront per sample walks the G/16 column blocks of 16 images.  Per
// block, theta runs on MFMA with tanh(theta) left in registers (as in the
// fused E_loc kernel); the weights use a running maximum m of Re L over the
// blocks seen so far (the accumulators are rescaled by e^{m_old - m_new}
// when it grows).  The products u t go through a 16 x 16 LDS tile per hidden
// tile (u itself through the row padding of the first tile) into the B
// operand of a second MFMA contraction over the images, whose A operand is
// the gathered image x with an extra all-ones row:
//   C[j][col] = sum_g A[j][g] B[g][col],  A = [x_g | 1],  B = [Re u t | Im u t | u],
// so the ones row gives O_b and D, and the u columns give O_a.  The
// contraction runs on 16x16x32 BF16 MFMA with each FP32 value of B split
// exactly into three BF16 terms (split3_bf16; x = +-1/2 and 1 are exact in
// BF16), so its products are the FP32 products and only the FP32
// accumulation rounds: lane (q, c) supplies images 4q .. 4q+3 (hi and mid in
// one MFMA, lo in a second), and the A operand is x of those images at site
// 16 st + c, staged twice over in one 16-byte LDS word per (q, site).
// Nothing of size S x G x K*M reaches HBM: the traffic is the spin rows and O.
#include "fused_theta.h"

namespace nqs {

namespace {

constexpr int kGradWaves = 8;

template <int N, int PREC, int K, int M>
struct GradCfg {
  using T = ThetaTraits<PREC>;
  static constexpr int KM = K * M;
  static constexpr int NHT = KM / 8;             // hidden tiles: 8 units = 16 B columns
  static constexpr int NCT = NHT + 1;            // + the u tile (2K columns)
  static_assert(2 * K <= 4, "the u columns live in the 4 padding floats of a tile row");
  // the output staging reuses the wave's tiles: 8 units x N complex, or K x N
  static_assert(NHT * 16 * 20 >= 16 * N && NHT * 16 * 20 >= 2 * K * N, "output staging");
  static constexpr int NST = (N + 1 + 15) / 16;  // site tiles incl. the ones row
  static constexpr int NK = nk_of<N, PREC>();
  // one 16 x 16 tile, rows (images) 20 floats apart: the contraction's reads
  // of rows 4q + r by the four lane groups q fall on disjoint bank groups.
  // Floats 16 .. 19 of a row of tile 0 hold the u columns (Re u_k, Im u_k).
  static constexpr int TR = 20;
  static constexpr int TS = 16 * TR;
  static constexpr int XQ = 4 * 16 * NST;        // image words: [q][site] incl. ones + zeros
  static constexpr size_t LDS = (size_t)NHT * NK * 64 * sizeof(typename T::AFrag) +
                                (size_t)kGradWaves * NHT * TS * sizeof(float) +
                                (size_t)kGradWaves * XQ * 16 +
                                (size_t)(2 * KM + 2 * K * N) * sizeof(float);
};

// value of lane (lane ^ 8) within its 16-lane row
__device__ __forceinline__ float row_ror8(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x128, 0xf, 0xf, false));
}

template <int N, int PREC, int K, int M>
__global__ __launch_bounds__(64 * kGradWaves) void grad_fused_kernel(
    const int8_t* __restrict__ spins, int64_t S, const uint8_t* __restrict__ perm, int G,
    const typename ThetaTraits<PREC>::AFrag* __restrict__ wfrag,
    const float* __restrict__ bias, const float* __restrict__ avec,
    const double* __restrict__ chi, int use_bias0, int Prbm0, int64_t P, float* __restrict__ O,
    double* __restrict__ logpsi) {
  using Cfg = GradCfg<N, PREC, K, M>;
  using T = ThetaTraits<PREC>;
  using AF = typename T::AFrag;
  constexpr int NHT = Cfg::NHT, NCT = Cfg::NCT, NST = Cfg::NST, NK = Cfg::NK, TS = Cfg::TS;
  constexpr int TR = Cfg::TR, XQ = Cfg::XQ;
  constexpr int TPR = M / 8;
  __shared__ __align__(16) AF Wl[NHT * NK * 64];
  __shared__ float tb[kGradWaves][NHT * TS];
  // the block's images as BF16 words [q][site]: x of images 4q .. 4q+3, twice
  __shared__ __align__(16) uint4 xq[kGradWaves][XQ];
  __shared__ float bl[2 * Cfg::KM], al[2 * K * N];   // hidden and visible biases

  for (int idx = threadIdx.x; idx < NHT * NK * 64; idx += blockDim.x) Wl[idx] = wfrag[idx];
  for (int idx = threadIdx.x; idx < 2 * Cfg::KM; idx += blockDim.x) bl[idx] = bias[idx];
  for (int idx = threadIdx.x; idx < 2 * K * N; idx += blockDim.x) al[idx] = avec[idx];
  const int lane0 = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float* tw = tb[wv];
  uint4* xw = xq[wv];
  for (int idx = lane0; idx < 4 * (16 * NST - N); idx += 64) {            // ones row, zero pad
    const int qq = idx / (16 * NST - N), j = N + idx % (16 * NST - N);
    const uint32_t one = j == N ? 0x3F803F80u : 0u;                         // BF16 1.0, twice
    xw[qq * 16 * NST + j] = make_uint4(one, one, one, one);
  }
  __syncthreads();

  const int nblk = G / 16;
  for (int64_t s = (int64_t)blockIdx.x * kGradWaves + wv; s < S;
       s += (int64_t)gridDim.x * kGradWaves) {
    const int8_t* srow = spins + s * N;
    f32x4 acc[NST][NCT];
#pragma unroll
    for (int st = 0; st < NST; ++st)
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) acc[st][ct] = f32x4{0, 0, 0, 0};
    double m_run = -INFINITY;

    for (int blk = 0; blk < nblk; ++blk) {
      // lane-derived values are recomputed per block instead of being hoisted
      // out of the loops and kept live (or spilled) across them
      int lane = lane0;
      asm volatile("" : "+v"(lane));
      const int q = lane >> 4, c = lane & 15;
      const int g = blk * 16 + c;
      const uint8_t* prow = perm + (size_t)g * N;
      typename T::BFrag bx[NK];
      // image c into the contraction's A words: BF16 x at slots c % 4 and c % 4 + 4
      // of word (c / 4, site)
      unsigned short* xh = reinterpret_cast<unsigned short*>(xw) + (c >> 2) * 16 * NST * 8 + (c & 3);
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
            xr = fmaf(xv[i], al[2 * (k * N + 4 * i + q)], xr);
            xi = fmaf(xv[i], al[2 * (k * N + 4 * i + q) + 1], xi);
          }
          axp[2 * k] = xr;
          axp[2 * k + 1] = xi;
        }
#pragma unroll
        for (int i = 0; i < N / 4; ++i) {
          xh[(4 * i + q) * 8] = (unsigned short)dx[i];
          xh[(4 * i + q) * 8 + 4] = (unsigned short)dx[i];
        }
      } else if constexpr (bf16_mfma(PREC)) {
        load_bfrag<N, PREC>(srow, prow, q, bx);
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) {
          // the fragment's BF16 pairs as words, halves taken with integer shifts
          const uint4 wb = __builtin_bit_cast(uint4, bx[kk]);
          const uint32_t wd[4] = {wb.x, wb.y, wb.z, wb.w};
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int kap = 32 * kk + 8 * q + e;
            if (kap < N) {
              const unsigned short h = (unsigned short)(wd[e >> 1] >> (16 * (e & 1)));
              xh[kap * 8] = h;
              xh[kap * 8 + 4] = h;
            }
          }
        }
      } else {
        load_bfrag<N, PREC>(srow, prow, q, bx);
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) {
          const unsigned short h = (unsigned short)(__float_as_uint((float)bx[kk]) >> 16);
          xh[(4 * kk + q) * 8] = h;
          xh[(4 * kk + q) * 8 + 4] = h;
        }
      }
      float tr[NHT * 2], ti[NHT * 2], Pr[K], Pi[K], Ai[K];
      double Er[K];
      theta_block<N, PREC, K, M>(Wl, bx, bl, al, srow, prow, lane, tr, ti, Er, Pr, Pi, Ai, axp);

      double mloc = Er[0];
#pragma unroll
      for (int k = 1; k < K; ++k) mloc = fmax(mloc, Er[k]);
      const double m_blk = wave_max(mloc);
      if (m_blk > m_run) {                             // uniform across the wave
        const float sc = exp_t((float)(m_run - m_blk));  // 0 on the first block
#pragma unroll
        for (int st = 0; st < NST; ++st)
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[st][ct][r] *= sc;
        m_run = m_blk;
      }
      const float ch = (float)chi[g];
      float ur[K], ui[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const float e = ch * exp_t((float)(Er[k] - m_run));
        float sn, cs;
        sincos_t(Ai[k], &sn, &cs);
        ur[k] = e * (Pr[k] * cs - Pi[k] * sn);
        ui[k] = e * (Pr[k] * sn + Pi[k] * cs);
      }
      // B tiles: row = image c, columns [Re u t of units 8ht..8ht+7 | Im ...]
#pragma unroll
      for (int ht = 0; ht < NHT; ++ht) {
        const int k = ht / TPR;
        float* row = tw + ht * TS + c * TR;
#pragma unroll
        for (int u2 = 0; u2 < 2; ++u2) {
          const float a = tr[2 * ht + u2], b = ti[2 * ht + u2];
          row[2 * q + u2] = ur[k] * a - ui[k] * b;
          row[8 + 2 * q + u2] = ur[k] * b + ui[k] * a;
        }
      }
      if (q == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
          tw[c * TR + 16 + 2 * k] = ur[k];
          tw[c * TR + 16 + 2 * k + 1] = ui[k];
        }
      }
      wave_sync_lds();
      // contraction over the block's images: lane (q, c) supplies images
      // 4q .. 4q+3 of column c (split into BF16 terms) and of site 16 st + c
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) {
        float v[4];
        if (ct < NHT) {
#pragma unroll
          for (int r = 0; r < 4; ++r) v[r] = tw[ct * TS + (4 * q + r) * TR + c];
        } else {
          // the u tile: columns 0 .. 2K-1 from the padding of tile 0, the rest zero
          const int cu = c < 2 * K ? c : 2 * K - 1;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float u = tw[(4 * q + r) * TR + 16 + cu];
            v[r] = c < 2 * K ? u : 0.f;
          }
        }
        bf16x8 b1, b2;
        split3_bf16(v, b1, b2);
#pragma unroll
        for (int st = 0; st < NST; ++st) {
          const bf16x8 ax = __builtin_bit_cast(bf16x8, xw[q * 16 * NST + 16 * st + c]);
          acc[st][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, b1, acc[st][ct], 0, 0, 0);
          acc[st][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, b2, acc[st][ct], 0, 0, 0);
        }
      }
      wave_sync_lds();
    }

    int lane = lane0, Prbm = Prbm0, use_bias = use_bias0;
    asm volatile("" : "+v"(lane));
    asm volatile("" : "+s"(Prbm), "+s"(use_bias));
    const int q = lane >> 4, c = lane & 15;
    // D from the ones row (site index N) of the u tile: lane (N%16/4, 2k), reg N%4
    constexpr int stN = N / 16, laneN = 16 * ((N % 16) / 4), rN = N % 4;
    float Dr = 0.f, Di = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      Dr += __int_as_float(
          __builtin_amdgcn_readlane(__float_as_int(acc[stN][NHT][rN]), laneN + 2 * k));
      Di += __int_as_float(
          __builtin_amdgcn_readlane(__float_as_int(acc[stN][NHT][rN]), laneN + 2 * k + 1));
    }
    const float d2 = Dr * Dr + Di * Di;
    const float ir = Dr / d2, ii = -Di / d2;
    if (logpsi && lane == 0) {
      logpsi[2 * s] = m_run + (double)(0.5f * log_t(d2));
      logpsi[2 * s + 1] = (double)atan2_t(Di, Dr);
    }
    float* Os = O + (size_t)s * P * 2;
    // Output through LDS: the 8 units of column tile ct are consecutive in
    // one RBM, so O_W of the tile is one contiguous run of 8 N complex values.
    // Column col < 8 of the tile is Re of unit 8 ct + col, col + 8 its Im.
#pragma unroll
    for (int ct = 0; ct < NHT; ++ct) {
#pragma unroll
      for (int st = 0; st < NST; ++st)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float re = acc[st][ct][r], im = row_ror8(re);
          const int j = 16 * st + 4 * q + r;
          if (c < 8 && j < N) {
            tw[2 * (c * N + j)] = re * ir - im * ii;
            tw[2 * (c * N + j) + 1] = re * ii + im * ir;
          } else if (c < 8 && j == N && use_bias) {
            const int h = 8 * ct + c;
            const size_t idx = (size_t)(h / M) * Prbm + (size_t)M * N + N + h % M;
            Os[2 * idx] = re * ir - im * ii;
            Os[2 * idx + 1] = re * ii + im * ir;
          }
        }
      wave_sync_lds();
      const int h0 = 8 * ct;
      float2* dst = reinterpret_cast<float2*>(Os) + (size_t)(h0 / M) * Prbm + (size_t)(h0 % M) * N;
      const float2* src = reinterpret_cast<const float2*>(tw);
      for (int e = lane; e < 8 * N; e += 64) dst[e] = src[e];
      wave_sync_lds();
    }
    // a: columns 2k (Re) and 2k + 1 (Im) of the u tile, N values per RBM
    if (use_bias) {
#pragma unroll
      for (int st = 0; st < NST; ++st)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float re = acc[st][NHT][r], im = __shfl_xor(re, 1, 64);
          const int j = 16 * st + 4 * q + r;
          if (!(c & 1) && c < 2 * K && j < N) {
            tw[2 * ((c >> 1) * N + j)] = re * ir - im * ii;
            tw[2 * ((c >> 1) * N + j) + 1] = re * ii + im * ir;
          }
        }
      wave_sync_lds();
      const float2* src = reinterpret_cast<const float2*>(tw);
      for (int e = lane; e < K * N; e += 64) {
        const int k = e / N;
        reinterpret_cast<float2*>(Os)[(size_t)k * Prbm + (size_t)M * N + e % N] = src[e];
      }
      wave_sync_lds();
    }
  }
}

template <int N, int PREC, int K, int M>
hipError_t run(const nqs_ctx* c, const int8_t* spins, int64_t S, void* O, double* logpsi,
               hipStream_t st) {
  int64_t blocks = (S + kGradWaves - 1) / kGradWaves;
  blocks = std::min<int64_t>(blocks, 2 * (int64_t)(c->n_cu > 0 ? c->n_cu : 256));
  const void* wf = PREC == kPrecF32S3 ? c->par.wfrag_s3 : c->par.wfrag;
  if (!wf) return hipErrorInvalidValue;
  grad_fused_kernel<N, PREC, K, M><<<(unsigned)blocks, 64 * kGradWaves, 0, st>>>(
      spins, S, c->dev.perm, c->G, (const typename ThetaTraits<PREC>::AFrag*)wf,
      (const float*)c->par.bias, (const float*)c->par.avec, c->dev.chi, c->d.use_bias, c->P_rbm,
      c->P, (float*)O, logpsi);
  return hipGetLastError();
}

template <int N, int K, int M>
hipError_t run_prec(const nqs_ctx* c, const int8_t* spins, int64_t S, void* O, double* logpsi,
                    hipStream_t st) {
  // theta of FP32 models on BF16 MFMA in the site-grouped three-term form
  return c->prec == NQS_FP32 ? run<N, kPrecF32S3, K, M>(c, spins, S, O, logpsi, st)
                             : run<N, NQS_BF16X2, K, M>(c, spins, S, O, logpsi, st);
}

}  // namespace

bool grad_fused_supported(const nqs_ctx* c) {
  if (c->prec == NQS_FP64) return false;
  const int N = c->N, K = c->K, M = c->M;
  return (N == 16 && K == 1 && M == 16) || (N == 16 && K == 2 && M == 8) ||
         (N == 36 && K == 1 && M == 72) || (N == 36 && K == 2 && M == 16) ||
         (N == 36 && K == 1 && M == 16);
}

hipError_t launch_grad_fused(const nqs_ctx* c, const int8_t* spins, int64_t S, void* O,
                             double* logpsi, hipStream_t st) {
  if (S <= 0) return hipSuccess;
  const int N = c->N, K = c->K, M = c->M;
  if (N == 16 && K == 1 && M == 16) return run_prec<16, 1, 16>(c, spins, S, O, logpsi, st);
  if (N == 16 && K == 2 && M == 8) return run_prec<16, 2, 8>(c, spins, S, O, logpsi, st);
  if (N == 36 && K == 1 && M == 72) return run_prec<36, 1, 72>(c, spins, S, O, logpsi, st);
  if (N == 36 && K == 2 && M == 16) return run_prec<36, 2, 16>(c, spins, S, O, logpsi, st);
  if (N == 36 && K == 1 && M == 16) return run_prec<36, 1, 16>(c, spins, S, O, logpsi, st);
  return hipErrorNotSupported;
}

}  // namespace nqs
