// Log-derivatives O_k = d log psi / d theta_k (Sec. 3.2, below Eq. (12)).
//
// With the normalised image weights w_kg = chi_g psi_s^(k)(g sigma)/psi(sigma),
// t = tanh(theta) and the images x_g = g sigma:
//   O_W[k][h][j] = sum_g w_kg t_kgh x_gj,  O_b[k][h] = sum_g w_kg t_kgh,
//   O_a[k][j]    = sum_g w_kg x_gj.
// Per sample this is one contraction over the G images,
// (interleaved Re/Im rows of w t, plus rows of w) x (images x [sites | 1]),
// run on 16x16x4 MFMA (FP32 or FP64): the extra all-ones column yields O_b,
// the extra w rows yield O_a.  One wavefront per (sample, 16-row tile) with
// all site-column blocks accumulated side by side.
#include "device_common.h"
#include "nqs_internal.h"

namespace nqs {

namespace {

__device__ __forceinline__ f64x4 mfma4(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename R> struct AccOf;
template <> struct AccOf<double> { using type = f64x4; };
template <> struct AccOf<float> { using type = f32x4; };

template <typename R, int N>
__global__ __launch_bounds__(256) void grad_kernel(
    const int8_t* __restrict__ spins, int64_t S, const uint8_t* __restrict__ perm, int G, int K,
    int M, int n_htiles, int use_bias, int Prbm, int64_t P, const R* __restrict__ t,
    const R* __restrict__ w, R* __restrict__ O) {
  using Acc = typename AccOf<R>::type;
  constexpr int NJB = (N + 1 + 15) / 16;
  const int lane = threadIdx.x & 63;
  const int i = lane & 15, kq = lane >> 4;
  const int li = logical_row<R>(i);                  // logical A row of this lane
  const int n_rt = n_htiles + (use_bias ? K : 0);
  const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wave >= S * n_rt) return;
  const int64_t s = wave / n_rt;
  const int rt = (int)(wave % n_rt);
  const bool wrow = rt < n_htiles;
  const int hrow = 8 * rt + li / 2;                  // hidden unit of this A row (W tiles)
  const int krow = wrow ? hrow / M : rt - n_htiles;  // RBM of this A row
  const int8_t* srow = spins + s * N;
  const R* ws = w + ((size_t)s * K + krow) * G * 2;
  const R* ts = t + ((size_t)s * n_htiles + (wrow ? rt : 0)) * G * 16 + (li / 2) * 2;

  Acc acc[NJB];
#pragma unroll
  for (int jb = 0; jb < NJB; ++jb) acc[jb] = Acc{0, 0, 0, 0};
  for (int g0 = 0; g0 < G; g0 += 4) {
    const int g = g0 + kq;
    const R wr = ws[2 * g], wi = ws[2 * g + 1];
    R a;
    if (wrow) {
      const R tr = ts[(size_t)g * 16], ti = ts[(size_t)g * 16 + 1];
      a = (li & 1) ? (wr * ti + wi * tr) : (wr * tr - wi * ti);
    } else {
      a = li == 0 ? wr : (li == 1 ? wi : R(0));
    }
    const uint8_t* prow = perm + (size_t)g * N;
#pragma unroll
    for (int jb = 0; jb < NJB; ++jb) {
      const int j = 16 * jb + i;
      R b = R(0);
      if (j < N) b = R(0.5) * (R)srow[prow[j]];
      else if (j == N) b = R(1);
      acc[jb] = mfma4(a, b, acc[jb]);
    }
  }
  // lane (kq, i) holds rows 4 kq .. 4 kq + 3 of column 16 jb + i
  R* Os = O + (size_t)s * P * 2;
#pragma unroll
  for (int jb = 0; jb < NJB; ++jb) {
    const int j = 16 * jb + i;
    if (j > N) continue;
    if (wrow) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int h = 8 * rt + 2 * kq + u;
        const int k = h / M, hh = h % M;
        size_t idx;
        if (j < N) idx = (size_t)k * Prbm + (size_t)hh * N + j;
        else if (use_bias) idx = (size_t)k * Prbm + (size_t)M * N + N + hh;
        else continue;
        Os[2 * idx] = (R)acc[jb][2 * u];
        Os[2 * idx + 1] = (R)acc[jb][2 * u + 1];
      }
    } else if (kq == 0 && j < N) {
      const size_t idx = (size_t)krow * Prbm + (size_t)M * N + j;
      Os[2 * idx] = (R)acc[jb][0];
      Os[2 * idx + 1] = (R)acc[jb][1];
    }
  }
}

template <typename R, int N>
hipError_t grad_for(const nqs_ctx* c, const int8_t* spins, int64_t S, const void* t, const void* w,
                    void* O, hipStream_t st) {
  const int n_rt = c->n_htiles + (c->d.use_bias ? c->K : 0);
  const int64_t waves = S * n_rt;
  grad_kernel<R, N><<<(unsigned)((waves + 3) / 4), 256, 0, st>>>(
      spins, S, c->dev.perm, c->G, c->K, c->M, c->n_htiles, c->d.use_bias, c->P_rbm, c->P,
      (const R*)t, (const R*)w, (R*)O);
  return hipGetLastError();
}

template <typename R>
hipError_t grad_typed(const nqs_ctx* c, const int8_t* spins, int64_t S, const void* t,
                      const void* w, void* O, hipStream_t st) {
  switch (c->L) {
    case 4: return grad_for<R, 16>(c, spins, S, t, w, O, st);
    case 6: return grad_for<R, 36>(c, spins, S, t, w, O, st);
    case 8: return grad_for<R, 64>(c, spins, S, t, w, O, st);
    default: return grad_for<R, 100>(c, spins, S, t, w, O, st);
  }
}

}  // namespace

hipError_t launch_grad(const nqs_ctx* c, const int8_t* spins, int64_t S, const void* t,
                       const void* w, void* O, hipStream_t st) {
  if (S <= 0) return hipSuccess;
  return c->prec == NQS_FP64 ? grad_typed<double>(c, spins, S, t, w, O, st)
                             : grad_typed<float>(c, spins, S, t, w, O, st);
}

}  // namespace nqs
