// Log-derivatives O_k = d log psi / d theta_k (Sec. 3.2, below Eq. (12)) for
// models whose hidden layer does not fit one wavefront (K*M > 128), theta in
// FP32 (on BF16 MFMA from the exact three-term split of W) or split BF16.
//
// With the normalised image weights w_kg = chi_g psi_s^(k)(g sigma)/psi(sigma)
// (written by the log-sum-exp kernel after a theta pass that keeps only the
// per-image log amplitudes), t = tanh(theta) and the images x_g = g sigma:
//   O_W[k][h][j] = sum_g w_kg t_kgh x_gj,  O_b[k][h] = sum_g w_kg t_kgh,
//   O_a[k][j]    = sum_g w_kg x_gj.
// tanh(theta) never reaches HBM: this kernel recomputes theta on MFMA.
//
// One workgroup of kGW wavefronts per configuration.  The work items of a
// configuration are its hidden tiles (8 units = 16 interleaved Re/Im rows of
// W) plus, with biases, one item for O_a; wavefront w takes items w, w + kGW,
// ... in rounds.  All wavefronts walk the G/16 image blocks in lockstep, so
// the block's images are staged once in LDS for all of them (double-buffered,
// one barrier per block): as BF16 rows [x | x | 0] (split BF16) or
// [x | x | x | 0] (FP32), and as the contraction's words below.  Per block a
// tile item
//   * computes theta^T = X W^T on MFMA (the image rows as the A operand, the W
//     fragments of the tile, kept in registers for the whole item, as the B
//     operand): lane (q, c) = (lane/16, lane%16) receives row c of the tile
//     (Re or Im of unit c/2) for images 4q .. 4q+3;
//   * exchanges the other component with the neighbouring lane (c ^ 1), and
//     each of the two lanes evaluates tanh for two of the four images and
//     multiplies by w; a second exchange leaves lane c with component c & 1
//     of w t for all four images -- which is already the A-operand layout of
//     the contraction with the images taken in the order 4q + r at step r;
//   * accumulates C[row][site] += sum_g (w t)[row][g] x[g][site] on 16x16x32
//     BF16 MFMA: each FP32 value v of w t is split exactly into three BF16
//     terms (hi = v with its low 16 bits cleared, mid the same of v - hi, lo =
//     v - hi - mid, which has at most 8 significant bits), and x = +-1/2 is
//     exact in BF16, so every product is the exact FP32 product and only the
//     FP32 accumulation rounds -- at a quarter of the MFMA time of 16x16x4
//     FP32.  Lane (q, c) puts hi and mid of its four images in the K slots of
//     one MFMA and lo in a second; the B operand is x of images 4q .. 4q+3 at
//     site 16 sb + c, staged twice over in one 16-byte LDS word per (q, site)
//     (the column of ones at site N gives O_b).
// The O_a item multiplies rows of w instead of w t.  Each lane then writes
// units 8 ht + 2q, 8 ht + 2q + 1 at sites 16 sb + c: 16 consecutive complex
// values per row of lanes.
#include "theta_common.h"

namespace nqs {

namespace {

constexpr int kGW = 8;             // wavefronts per workgroup (one configuration)

template <int N, int PREC>
struct GradWideCfg {
  static constexpr int NK = nk_of<N, PREC>();
  static constexpr int NSB = (N + 1 + 15) / 16;      // site blocks incl. the ones column
  static constexpr int XS = 16 * NSB + 4;            // FP32 theta rows (conflict-free reads)
  static constexpr int XB = 32 * NK + 8;             // BF16 row stride (elements)
  static constexpr bool BF = bf16_mfma(PREC);         // theta on BF16 MFMA
  static constexpr int XC = x_copies(PREC);           // copies of x along its K axis
};

__device__ __forceinline__ float swap_adjacent(float v) {   // value of lane l ^ 1
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xf, 0xf, false));
}

template <int N, int PREC>
__global__ __launch_bounds__(64 * kGW) __attribute__((amdgpu_waves_per_eu(4))) void grad_wide_kernel(
    const int8_t* __restrict__ spins, int64_t S, const uint8_t* __restrict__ perm, int G, int K,
    int M, int use_bias, int Prbm, int64_t P,
    const typename ThetaTraits<PREC>::AFrag* __restrict__ wfrag, const float* __restrict__ bias,
    const float* __restrict__ w, float* __restrict__ O) {
  using Cfg = GradWideCfg<N, PREC>;
  using T = ThetaTraits<PREC>;
  constexpr int NK = Cfg::NK, NSB = Cfg::NSB, XS = Cfg::XS, XB = Cfg::XB;
  __shared__ __align__(16) float xt[Cfg::BF ? 1 : 2][Cfg::BF ? 4 : 16 * XS];
  __shared__ __align__(16) unsigned short xb[Cfg::BF ? 2 : 1][Cfg::BF ? 16 * XB : 8];
  // [q][site]: BF16 x of images 4q .. 4q+3, twice (16 lanes of one q read 16
  // consecutive words: no bank conflicts)
  __shared__ __align__(16) uint4 xq[2][4 * 16 * NSB];
  extern __shared__ __align__(16) float wl[];          // [K][G] complex: this configuration's w

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int q = lane >> 4, c = lane & 15;
  const bool odd = c & 1;
  const int KM = K * M, n_ht = KM / 8, nblk = G / 16;
  const int n_items = n_ht + (use_bias ? 1 : 0);
  const int rounds = (n_items + kGW - 1) / kGW;

  // constant parts of the staged operands: in the contraction's, site N is 1
  // (O_b) and the sites beyond are 0; the split-BF16 theta rows are zero
  // beyond position 2N
  for (int e = tid; e < 2 * 4 * (16 * NSB - N); e += 64 * kGW) {
    const int b = e / (4 * (16 * NSB - N)), r = e % (4 * (16 * NSB - N));
    const int j = N + r / 4;
    const uint32_t one = j == N ? 0x3F803F80u : 0u;                 // BF16 1.0, twice
    xq[b][(r % 4) * 16 * NSB + j] = make_uint4(one, one, one, one);
  }
  constexpr int PADB = 32 * NK - Cfg::XC * N;          // zero K positions of a BF16 row
  if constexpr (Cfg::BF && PADB > 0) {
    for (int e = tid; e < 2 * 16 * PADB; e += 64 * kGW) {
      const int b = e / (16 * PADB), r = e % (16 * PADB);
      xb[b][(r / PADB) * XB + Cfg::XC * N + r % PADB] = 0;
    }
  }

  for (int64_t s = blockIdx.x; s < S; s += gridDim.x) {
    const int8_t* srow = spins + s * N;
    __syncthreads();                                   // previous configuration done with wl / rows
    const float* ws = w + (size_t)s * K * G * 2;
    for (int e = tid; e < 2 * K * G; e += 64 * kGW) wl[e] = ws[e];
    // stage the images of block blk into buffer b: thread item (site j, image
    // group qq) reads images 16 blk + 4 qq + r, r = 0..3
    auto stage = [&](int blk, int b) {
      for (int e = tid; e < 4 * N; e += 64 * kGW) {
        const int qq = e / N, j = e - qq * N;
        uint32_t h[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ii = 4 * qq + r;
          const int v = srow[perm[(size_t)(blk * 16 + ii) * N + j]];
          h[r] = v > 0 ? 0x3F00u : 0xBF00u;                        // BF16 +-1/2
          if constexpr (Cfg::BF) {
#pragma unroll
            for (int cp = 0; cp < Cfg::XC; ++cp) xb[b][ii * XB + cp * N + j] = (unsigned short)h[r];
          } else {
            xt[b][ii * XS + j] = v > 0 ? 0.5f : -0.5f;
          }
        }
        const uint32_t lo = h[0] | (h[1] << 16), hi = h[2] | (h[3] << 16);
        xq[b][qq * 16 * NSB + j] = make_uint4(lo, hi, lo, hi);
      }
    };
    stage(0, 0);
    __syncthreads();

    for (int rd = 0; rd < rounds; ++rd) {
      const int item = rd * kGW + wv;
      const bool is_tile = item < n_ht;
      const bool is_a = use_bias && item == n_ht;
      const int ht = is_tile ? item : 0;
      const int k = is_tile ? ht / (M / 8) : 0;
      typename T::AFrag wf[NK];
#pragma unroll
      for (int kk = 0; kk < NK; ++kk) wf[kk] = wfrag[((size_t)ht * NK + kk) * 64 + lane];
      const float b0 = bias[16 * ht + c];
      f32x4 acc[NSB];
#pragma unroll
      for (int sb = 0; sb < NSB; ++sb) acc[sb] = f32x4{0.f, 0.f, 0.f, 0.f};

      for (int blk = 0; blk < nblk; ++blk) {
        const int cur = (rd * nblk + blk) & 1;
        // stage the next block (the next round starts again at block 0)
        if (blk + 1 < nblk) stage(blk + 1, cur ^ 1);
        else if (rd + 1 < rounds) stage(0, cur ^ 1);
        const float* xc = xt[Cfg::BF ? 0 : cur];
        float A[4];
        if (is_tile) {
          f32x4 th = f32x4{b0, b0, b0, b0};
          if constexpr (Cfg::BF) {
#pragma unroll
            for (int kk = 0; kk < NK; ++kk) {
              const bf16x8 a = *reinterpret_cast<const bf16x8*>(&xb[cur][c * XB + 32 * kk + 8 * q]);
              th = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, wf[kk], th, 0, 0, 0);
            }
          } else {
#pragma unroll
            for (int kk = 0; kk < NK; ++kk)
              th = __builtin_amdgcn_mfma_f32_16x16x4f32(xc[c * XS + 4 * kk + q], wf[kk], th, 0, 0, 0);
          }
          // th[v]: component c & 1 of theta of unit 8 ht + c/2, image 4q + v
          float pv[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) pv[v] = swap_adjacent(th[v]);
          // this lane evaluates images 4q + v0, 4q + v0 + 1 (v0 = 0 even lanes, 2 odd)
          const float x0 = odd ? pv[2] : th[0], y0 = odd ? th[2] : pv[0];
          const float x1 = odd ? pv[3] : th[1], y1 = odd ? th[3] : pv[1];
          float t0r, t0i, t1r, t1i;
          tanh_c(x0, y0, t0r, t0i);
          tanh_c(x1, y1, t1r, t1i);
          const int g0 = blk * 16 + 4 * q + (odd ? 2 : 0);
          const float2 w0 = *reinterpret_cast<const float2*>(&wl[2 * (k * G + g0)]);
          const float2 w1 = *reinterpret_cast<const float2*>(&wl[2 * (k * G + g0 + 1)]);
          const float u0r = w0.x * t0r - w0.y * t0i, u0i = w0.x * t0i + w0.y * t0r;
          const float u1r = w1.x * t1r - w1.y * t1i, u1i = w1.x * t1i + w1.y * t1r;
          // even lanes keep Re (images 0, 1), odd lanes Im (images 2, 3); trade the rest
          const float r0 = swap_adjacent(odd ? u0r : u0i), r1 = swap_adjacent(odd ? u1r : u1i);
          A[0] = odd ? r0 : u0r;
          A[1] = odd ? r1 : u1r;
          A[2] = odd ? u0i : r0;
          A[3] = odd ? u1i : r1;
        } else {
          // O_a item: row c = component c & 1 of w_(c/2) (rows beyond 2K are zero)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int kr = c >> 1;
            A[v] = is_a && kr < K ? wl[2 * (kr * G + blk * 16 + 4 * q + v) + (c & 1)] : 0.f;
          }
        }
        if (is_tile || is_a) {
          bf16x8 a1, a2;
          split3_bf16(A, a1, a2);
#pragma unroll
          for (int sb = 0; sb < NSB; ++sb) {
            const bf16x8 bx = __builtin_bit_cast(bf16x8, xq[cur][q * 16 * NSB + 16 * sb + c]);
            acc[sb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bx, acc[sb], 0, 0, 0);
            acc[sb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, bx, acc[sb], 0, 0, 0);
          }
        }
        __syncthreads();
      }

      // lane (q, c): rows 4q .. 4q+3 = (Re, Im) of units 2q, 2q + 1 of the item, site 16 sb + c
      float2* Os = reinterpret_cast<float2*>(O) + (size_t)s * P;
      if (is_tile) {
        const int u0 = (8 * ht) % M + 2 * q;
#pragma unroll
        for (int sb = 0; sb < NSB; ++sb) {
          const int j = 16 * sb + c;
#pragma unroll
          for (int uu = 0; uu < 2; ++uu) {
            const float2 v = make_float2(acc[sb][2 * uu], acc[sb][2 * uu + 1]);
            if (j < N) Os[(size_t)k * Prbm + (size_t)(u0 + uu) * N + j] = v;
            else if (j == N && use_bias) Os[(size_t)k * Prbm + (size_t)M * N + N + u0 + uu] = v;
          }
        }
      } else if (is_a) {
#pragma unroll
        for (int sb = 0; sb < NSB; ++sb) {
          const int j = 16 * sb + c;
#pragma unroll
          for (int uu = 0; uu < 2; ++uu) {
            const int kr = 2 * q + uu;
            if (j < N && kr < K)
              Os[(size_t)kr * Prbm + (size_t)M * N + j] =
                  make_float2(acc[sb][2 * uu], acc[sb][2 * uu + 1]);
          }
        }
      }
    }
  }
}

template <int N, int PREC>
hipError_t run(const nqs_ctx* c, const int8_t* spins, int64_t S, const float* w, void* O,
               hipStream_t st) {
  const size_t lds = (size_t)c->K * c->G * 2 * sizeof(float);
  const int64_t blocks = std::min<int64_t>(S, (int64_t)(c->n_cu > 0 ? c->n_cu : 256) * 8);
  grad_wide_kernel<N, PREC><<<(unsigned)blocks, 64 * kGW, lds, st>>>(
      spins, S, c->dev.perm, c->G, c->K, c->M, c->d.use_bias, c->P_rbm, c->P,
      (const typename ThetaTraits<PREC>::AFrag*)(PREC == kPrecF32X3 ? c->par.wfrag3
                                                                    : c->par.wfrag),
      (const float*)c->par.bias, w,
      (float*)O);
  return hipGetLastError();
}

}  // namespace

bool grad_wide_supported(const nqs_ctx* c) {
  if (c->prec == NQS_FP64 || c->KM <= 128 || c->M % 8 != 0 || c->K > 8) return false;
  // the configuration's weights [K][G] complex float stay in LDS
  if ((size_t)c->K * c->G * 8 > 64 * 1024) return false;
  return c->N == 36 || c->N == 64 || c->N == 100;
}

hipError_t launch_grad_wide(const nqs_ctx* c, const int8_t* spins, int64_t S, const void* w,
                            void* O, hipStream_t st) {
  if (S <= 0) return hipSuccess;
  const bool bf = c->prec == NQS_BF16X2;
  const float* wf = (const float*)w;
  switch (c->N) {
    case 36: return bf ? run<36, NQS_BF16X2>(c, spins, S, wf, O, st)
                       : run<36, kPrecF32X3>(c, spins, S, wf, O, st);
    case 64: return bf ? run<64, NQS_BF16X2>(c, spins, S, wf, O, st)
                       : run<64, kPrecF32X3>(c, spins, S, wf, O, st);
    case 100: return bf ? run<100, NQS_BF16X2>(c, spins, S, wf, O, st)
                        : run<100, kPrecF32X3>(c, spins, S, wf, O, st);
    default: return hipErrorNotSupported;
  }
}

}  // namespace nqs
