// Stochastic reconfiguration step (Sec. 3.2, Eq. (12); ridge lambda of
// Sec. 3.4) solved in sample space.
//
// With O_bar = (O - <O>)/sqrt(S) and eps = (E_loc - <E_loc>)/sqrt(S), the
// P x P system (O_bar^H O_bar + lambda) dtheta = -dtau O_bar^H eps has the
// same solution as dtheta = -dtau O_bar^H (O_bar O_bar^H + lambda)^{-1} eps
// (push-through identity), an S x S Hermitian positive definite system:
//  1. column means of O, then O_bar written transposed as separate real and
//     imaginary planes [P][S] (unit-stride sample axis for the MFMA operands);
//  2. Gram T = O_bar O_bar^H + lambda I on 16x16x4 MFMA (FP32 for complex64
//     O, on LDS-staged 128 x 128 tiles; FP64 for complex128), complex product
//     as four real products, lower block triangle only, stored in FP64;
//  3. blocked right-looking FP64 Cholesky T = L L^H with 32 x 32 blocks:
//     diagonal factorisation in LDS, panel triangular solve, Hermitian
//     updates on FP64 MFMA (within a panel of 8 block columns per column,
//     then one rank-256 update of the trailing matrix per panel);
//  4. L y = eps, L^H x = y, dtheta = -dtau O_bar^H x.
// S is padded to a multiple of 32 with zero rows (their T block is lambda I
// and their eps is 0, so they drop out of x and dtheta).
#include <algorithm>
#include <cmath>
#include <string>

#include "device_common.h"
#include "nqs_internal.h"

namespace nqs {

namespace {

constexpr int kB = 32;   // Cholesky / Gram block
constexpr int kPanel = 8;  // block columns per Cholesky panel (one trailing update each)

__device__ __forceinline__ f64x4 mma(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mma(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename R> struct AccT;
template <> struct AccT<float> { using type = f32x4; };
template <> struct AccT<double> { using type = f64x4; };
// output row of register r in lane group q (see logical_row in device_common.h)
template <typename R> __device__ __forceinline__ int out_row(int q, int r) {
  return sizeof(R) == 8 ? q + 4 * r : 4 * q + r;
}

// ---------------------------------------------------------------- centring
template <typename RO>
__global__ void colmean_kernel(const RO* __restrict__ O, int64_t S, int64_t P,
                               double* __restrict__ mean) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P) return;
  double sr = 0.0, si = 0.0;
  for (int64_t s = 0; s < S; ++s) {
    sr += (double)O[(s * P + k) * 2];
    si += (double)O[(s * P + k) * 2 + 1];
  }
  mean[2 * k] = sr / (double)S;
  mean[2 * k + 1] = si / (double)S;
}

// O_bar transposed: Tre[k][s], Tim[k][s] for k < P4, s < S32 (zero padding)
template <typename RO, typename RG>
__global__ void center_t_kernel(const RO* __restrict__ O, int64_t S, int64_t P, int64_t P4,
                                int64_t S32, const double* __restrict__ mean, double inv_sqrt_s,
                                RG* __restrict__ Tre, RG* __restrict__ Tim) {
  __shared__ double tr[32][33], ti[32][33];
  const int64_t s0 = (int64_t)blockIdx.x * 32, k0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8 threads
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t s = s0 + yy, k = k0 + tx;
    double vr = 0.0, vi = 0.0;
    if (s < S && k < P) {
      vr = ((double)O[(s * P + k) * 2] - mean[2 * k]) * inv_sqrt_s;
      vi = ((double)O[(s * P + k) * 2 + 1] - mean[2 * k + 1]) * inv_sqrt_s;
    }
    tr[yy][tx] = vr;
    ti[yy][tx] = vi;
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t k = k0 + yy, s = s0 + tx;
    if (k < P4 && s < S32) {
      Tre[k * S32 + s] = (RG)tr[tx][yy];
      Tim[k * S32 + s] = (RG)ti[tx][yy];
    }
  }
}

// eps[s] = (E_loc[s] - <E_loc>) / sqrt(S), zero for the padding rows
__global__ void eps_kernel(const double* __restrict__ el, int64_t S, int64_t S32,
                           double* __restrict__ v) {
  __shared__ double red[2][16];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double sr = 0.0, si = 0.0;
  for (int64_t s = tid; s < S; s += blockDim.x) {
    sr += el[2 * s];
    si += el[2 * s + 1];
  }
  sr = wave_sum(sr);
  si = wave_sum(si);
  if (lane == 0) {
    red[0][wv] = sr;
    red[1][wv] = si;
  }
  __syncthreads();
  sr = 0.0;
  si = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
    sr += red[0][q];
    si += red[1][q];
  }
  const double mr = sr / (double)S, mi = si / (double)S, f = 1.0 / sqrt((double)S);
  for (int64_t s = tid; s < S32; s += blockDim.x) {
    v[2 * s] = s < S ? (el[2 * s] - mr) * f : 0.0;
    v[2 * s + 1] = s < S ? (el[2 * s + 1] - mi) * f : 0.0;
  }
}

// ------------------------------------------------------------------- Gram
__device__ __forceinline__ void tri_index(int64_t t, int64_t& I, int64_t& J) {
  I = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (I * (I + 1) / 2 > t) --I;
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  J = t - I * (I + 1) / 2;
}

// T[I-block][J-block] (I >= J) = sum_k Ob[s][k] conj(Ob[s'][k]) (+ lambda on the diagonal)
template <typename RG>
__global__ __launch_bounds__(256) void gram_kernel(const RG* __restrict__ Tre,
                                                   const RG* __restrict__ Tim, int64_t P4,
                                                   int64_t S32, int64_t nblk, double lambda,
                                                   double* __restrict__ T) {
  using Acc = typename AccT<RG>::type;
  const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= nblk * (nblk + 1) / 2) return;
  int64_t I, J;
  tri_index(t, I, J);
  Acc cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cr[a][b] = Acc{0, 0, 0, 0};
      ci[a][b] = Acc{0, 0, 0, 0};
    }
  const int64_t ra = I * kB + c, rb = J * kB + c;
  for (int64_t k0 = 0; k0 < P4; k0 += 4) {
    const int64_t kk = (k0 + q) * S32;
    RG ar[2], ai[2], br[2], bi[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      ar[a] = Tre[kk + ra + 16 * a];
      ai[a] = Tim[kk + ra + 16 * a];
      br[a] = Tre[kk + rb + 16 * a];
      bi[a] = Tim[kk + rb + 16 * a];
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        cr[a][b] = mma(ar[a], br[b], cr[a][b]);
        cr[a][b] = mma(ai[a], bi[b], cr[a][b]);
        ci[a][b] = mma(ai[a], br[b], ci[a][b]);
        ci[a][b] = mma(-ar[a], bi[b], ci[a][b]);
      }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = I * kB + 16 * a + out_row<RG>(q, r);
        const int64_t col = J * kB + 16 * b + c;
        double vr = (double)cr[a][b][r], vi = (double)ci[a][b][r];
        if (row == col) vr += lambda;
        T[(row * S32 + col) * 2] = vr;
        T[(row * S32 + col) * 2 + 1] = vi;
      }
}

// FP32 Gram on 128 x 128 output tiles, one workgroup of four wavefronts per
// lower tile (each wavefront a 64 x 64 quarter, 4 x 4 MFMA tiles of 16 x 16
// for each of the real and imaginary parts).  The two row panels of the tile
// go through LDS in stages of kGK sample-axis columns, double-buffered: the
// next stage's global loads are issued before the current stage's MFMAs.
// Per k, a panel row of 128 values is stored as [half][c][a] (row
// 64 half + 16 a + c at 64 half + 4 c + a) so that lane (q, c) reads its four
// operands a = 0..3 with one 16-byte LDS load; kGP pads the k rows apart.
// Only 32 x 32 blocks on or below the block diagonal are written.
constexpr int kGT = 128, kGK = 8, kGP = kGT + 4;

__global__ __launch_bounds__(256) void gram_tile_kernel(const float* __restrict__ Tre,
                                                        const float* __restrict__ Tim, int64_t P4,
                                                        int64_t S32, int64_t ntile, double lambda,
                                                        double* __restrict__ T) {
  __shared__ __align__(16) float As[2][2][kGK][kGP];   // [buffer][re, im][k][row slot]
  __shared__ __align__(16) float Bs[2][2][kGK][kGP];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, q = lane >> 4, c = lane & 15;
  const int wy = wv >> 1, wx = wv & 1;
  int64_t I, J;
  tri_index((int64_t)blockIdx.x, I, J);
  (void)ntile;
  const int64_t rowA = I * kGT, rowB = J * kGT;

  // stage loader: 1024 float4 per stage (A/B x re/im x kGK x 32), four per thread
  float4 pre[4];
  auto load_stage = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int idx = tid + 256 * i;
      const int ab = idx >> 9, rem = idx & 511, pl = rem >> 8, k = (rem >> 5) & 7, r4 = rem & 31;
      const int64_t row = (ab ? rowB : rowA) + 4 * r4, kk = k0 + k;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (kk < P4 && row < S32)
        v = *reinterpret_cast<const float4*>((pl ? Tim : Tre) + kk * S32 + row);
      pre[i] = v;
    }
  };
  auto store_stage = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int idx = tid + 256 * i;
      const int ab = idx >> 9, rem = idx & 511, pl = rem >> 8, k = (rem >> 5) & 7, r4 = rem & 31;
      float* dst = ab ? &Bs[buf][pl][k][0] : &As[buf][pl][k][0];
      const float vals[4] = {pre[i].x, pre[i].y, pre[i].z, pre[i].w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = 4 * r4 + e;                       // tile row 0..127
        dst[64 * (r >> 6) + 4 * (r & 15) + ((r >> 4) & 3)] = vals[e];
      }
    }
  };

  f32x4 cr[4][4], ci[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      cr[a][b] = f32x4{0, 0, 0, 0};
      ci[a][b] = f32x4{0, 0, 0, 0};
    }
  const int64_t nst = (P4 + kGK - 1) / kGK;
  load_stage(0);
  store_stage(0);
  __syncthreads();
  for (int64_t st = 0; st < nst; ++st) {
    const int cur = (int)(st & 1);
    if (st + 1 < nst) load_stage((st + 1) * kGK);
#pragma unroll
    for (int ks = 0; ks < kGK; ks += 4) {
      const float4 a_r = *reinterpret_cast<const float4*>(&As[cur][0][ks + q][64 * wy + 4 * c]);
      const float4 a_i = *reinterpret_cast<const float4*>(&As[cur][1][ks + q][64 * wy + 4 * c]);
      const float4 b_r = *reinterpret_cast<const float4*>(&Bs[cur][0][ks + q][64 * wx + 4 * c]);
      const float4 b_i = *reinterpret_cast<const float4*>(&Bs[cur][1][ks + q][64 * wx + 4 * c]);
      const float ar[4] = {a_r.x, a_r.y, a_r.z, a_r.w}, ai[4] = {a_i.x, a_i.y, a_i.z, a_i.w};
      const float br[4] = {b_r.x, b_r.y, b_r.z, b_r.w}, bi[4] = {b_i.x, b_i.y, b_i.z, b_i.w};
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) cr[a][b] = mma(ar[a], br[b], cr[a][b]);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) ci[a][b] = mma(ai[a], br[b], ci[a][b]);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) cr[a][b] = mma(ai[a], bi[b], cr[a][b]);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) ci[a][b] = mma(-ar[a], bi[b], ci[a][b]);
    }
    if (st + 1 < nst) {
      store_stage(cur ^ 1);
      __syncthreads();
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = rowA + 64 * wy + 16 * a + out_row<float>(q, r);
        const int64_t col = rowB + 64 * wx + 16 * b + c;
        if (row >= S32 || col >= S32 || row / kB < col / kB) continue;
        double vr = (double)cr[a][b][r], vi = (double)ci[a][b][r];
        if (row == col) vr += lambda;
        T[(row * S32 + col) * 2] = vr;
        T[(row * S32 + col) * 2 + 1] = vi;
      }
}

// --------------------------------------------------------------- Cholesky
// Factor the diagonal block k in LDS (lower triangle), flag non-positive pivots.
__global__ __launch_bounds__(256) void potrf_diag_kernel(double* __restrict__ T, int64_t S32,
                                                         int64_t k, int* __restrict__ flag) {
  __shared__ double ar[kB][kB + 1], ai[kB][kB + 1];
  const int tid = threadIdx.x;
  const int64_t kb = k * kB;
  for (int e = tid; e < kB * kB; e += blockDim.x) {
    const int i = e / kB, j = e % kB;
    ar[i][j] = T[((kb + i) * S32 + kb + j) * 2];
    ai[i][j] = T[((kb + i) * S32 + kb + j) * 2 + 1];
  }
  __syncthreads();
  for (int j = 0; j < kB; ++j) {
    if (tid == 0) {
      double d = ar[j][j];
      if (!(d > 0.0) || !isfinite(d)) {
        flag[0] = 1;
        d = 1.0;
      }
      ar[j][j] = sqrt(d);
      ai[j][j] = 0.0;
    }
    __syncthreads();
    const double dj = ar[j][j];
    for (int i = j + 1 + tid; i < kB; i += blockDim.x) {
      ar[i][j] /= dj;
      ai[i][j] /= dj;
    }
    __syncthreads();
    for (int e = tid; e < kB * kB; e += blockDim.x) {
      const int i = e / kB, l = e % kB;
      if (l > j && i >= l) {
        // A[i][l] -= A[i][j] conj(A[l][j])
        ar[i][l] -= ar[i][j] * ar[l][j] + ai[i][j] * ai[l][j];
        ai[i][l] -= ai[i][j] * ar[l][j] - ar[i][j] * ai[l][j];
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < kB * kB; e += blockDim.x) {
    const int i = e / kB, j = e % kB;
    if (i >= j) {
      T[((kb + i) * S32 + kb + j) * 2] = ar[i][j];
      T[((kb + i) * S32 + kb + j) * 2 + 1] = ai[i][j];
    }
  }
}

// Panel: rows r below block k solve X L_kk^H = A (one row per thread).
__global__ __launch_bounds__(256) void trsm_panel_kernel(double* __restrict__ T, int64_t S32,
                                                         int64_t k) {
  __shared__ double lr[kB][kB + 1], li[kB][kB + 1];
  const int64_t kb = k * kB;
  for (int e = threadIdx.x; e < kB * kB; e += blockDim.x) {
    const int i = e / kB, j = e % kB;
    lr[i][j] = T[((kb + i) * S32 + kb + j) * 2];
    li[i][j] = T[((kb + i) * S32 + kb + j) * 2 + 1];
  }
  __syncthreads();
  const int64_t r = kb + kB + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= S32) return;
  double xr[kB], xi[kB];
  double* row = T + (r * S32 + kb) * 2;
#pragma unroll
  for (int j = 0; j < kB; ++j) {
    double vr = row[2 * j], vi = row[2 * j + 1];
#pragma unroll
    for (int l = 0; l < j; ++l) {
      // v -= x_l conj(L[j][l])
      vr -= xr[l] * lr[j][l] + xi[l] * li[j][l];
      vi -= xi[l] * lr[j][l] - xr[l] * li[j][l];
    }
    xr[j] = vr / lr[j][j];
    xi[j] = vi / lr[j][j];
  }
#pragma unroll
  for (int j = 0; j < kB; ++j) {
    row[2 * j] = xr[j];
    row[2 * j + 1] = xi[j];
  }
}

// Trailing update: A_IJ -= X_I X_J^H for I >= J > k (X = panel block column k).
// Hermitian rank-(32 nk) update T[I][J] -= L[I][K] L[J][K]^H over the block
// columns K = kc0 .. kc0 + nk - 1, one wavefront per 32 x 32 output block.
// jn = 0: every block I >= J >= j0 (the trailing triangle); jn > 0: only the
// block columns J = j0 .. j0 + jn - 1 (the rest of the current panel), all
// I >= J.
__global__ __launch_bounds__(256) void herk_update_kernel(double* __restrict__ T, int64_t S32,
                                                          int64_t kc0, int nk, int64_t j0, int jn,
                                                          int64_t nblk) {
  const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
  int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  int64_t I = -1, J = -1;
  if (jn == 0) {
    const int64_t m = nblk - j0;
    if (t >= m * (m + 1) / 2) return;
    tri_index(t, I, J);
    I += j0;
    J += j0;
  } else {
    for (int jj = 0; jj < jn; ++jj) {
      const int64_t cnt = nblk - (j0 + jj);
      if (t < cnt) {
        J = j0 + jj;
        I = J + t;
        break;
      }
      t -= cnt;
    }
    if (J < 0) return;
  }
  const int64_t kb = kc0 * kB;
  f64x4 cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cr[a][b] = f64x4{0, 0, 0, 0};
      ci[a][b] = f64x4{0, 0, 0, 0};
    }
  for (int k0 = 0; k0 < nk * kB; k0 += 4) {
    double xr[2], xi[2], yr[2], yi[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int64_t ri = I * kB + 16 * a + c, rj = J * kB + 16 * a + c;
      xr[a] = T[(ri * S32 + kb + k0 + q) * 2];
      xi[a] = T[(ri * S32 + kb + k0 + q) * 2 + 1];
      yr[a] = T[(rj * S32 + kb + k0 + q) * 2];
      yi[a] = T[(rj * S32 + kb + k0 + q) * 2 + 1];
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        cr[a][b] = mma(xr[a], yr[b], cr[a][b]);
        cr[a][b] = mma(xi[a], yi[b], cr[a][b]);
        ci[a][b] = mma(xi[a], yr[b], ci[a][b]);
        ci[a][b] = mma(-xr[a], yi[b], ci[a][b]);
      }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = I * kB + 16 * a + out_row<double>(q, r);
        const int64_t col = J * kB + 16 * b + c;
        if (row >= col) {
          T[(row * S32 + col) * 2] -= cr[a][b][r];
          T[(row * S32 + col) * 2 + 1] -= ci[a][b][r];
        }
      }
}

// ------------------------------------------------------------------ solves
// L y = v on block k (single thread; the block is small)
// Diagonal-block triangular solves: the 32 x 32 block goes to LDS, lane i
// holds v_i, and the substitution runs column by column (lane j finishes its
// unknown, the others subtract its contribution), 32 steps of one wavefront.
__device__ __forceinline__ void load_diag_block(const double* __restrict__ T, int64_t S32,
                                                int64_t kb, double (*lr)[kB + 1],
                                                double (*li)[kB + 1]) {
  for (int e = threadIdx.x; e < kB * kB; e += blockDim.x) {
    const int i = e / kB, j = e % kB;
    lr[i][j] = T[((kb + i) * S32 + kb + j) * 2];
    li[i][j] = T[((kb + i) * S32 + kb + j) * 2 + 1];
  }
  __syncthreads();
}

// L y = v on diagonal block k (y overwrites v)
__global__ __launch_bounds__(64) void fsolve_diag_kernel(const double* __restrict__ T, int64_t S32,
                                                         int64_t k, double* __restrict__ v) {
  __shared__ double lr[kB][kB + 1], li[kB][kB + 1];
  const int t = threadIdx.x;
  const int64_t kb = k * kB;
  load_diag_block(T, S32, kb, lr, li);
  double vr = 0.0, vi = 0.0;
  if (t < kB) {
    vr = v[2 * (kb + t)];
    vi = v[2 * (kb + t) + 1];
  }
  for (int j = 0; j < kB; ++j) {
    if (t == j) {
      vr /= lr[j][j];
      vi /= lr[j][j];
    }
    const double yr = __shfl(vr, j, 64), yi = __shfl(vi, j, 64);
    if (t > j && t < kB) {
      vr -= lr[t][j] * yr - li[t][j] * yi;
      vi -= lr[t][j] * yi + li[t][j] * yr;
    }
  }
  if (t < kB) {
    v[2 * (kb + t)] = vr;
    v[2 * (kb + t) + 1] = vi;
  }
}

// v_i -= sum_l L[i][kb + l] y_l for rows i below block k
__global__ void fsolve_update_kernel(const double* __restrict__ T, int64_t S32, int64_t k,
                                     double* __restrict__ v) {
  const int64_t kb = k * kB;
  const int64_t i = kb + kB + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S32) return;
  double vr = v[2 * i], vi = v[2 * i + 1];
  for (int l = 0; l < kB; ++l) {
    const double Lr = T[(i * S32 + kb + l) * 2], Li = T[(i * S32 + kb + l) * 2 + 1];
    const double yr = v[2 * (kb + l)], yi = v[2 * (kb + l) + 1];
    vr -= Lr * yr - Li * yi;
    vi -= Lr * yi + Li * yr;
  }
  v[2 * i] = vr;
  v[2 * i + 1] = vi;
}

// L^H x = v on block k (single thread)
// L^H x = v on diagonal block k (x overwrites v)
__global__ __launch_bounds__(64) void bsolve_diag_kernel(const double* __restrict__ T, int64_t S32,
                                                         int64_t k, double* __restrict__ v) {
  __shared__ double lr[kB][kB + 1], li[kB][kB + 1];
  const int t = threadIdx.x;
  const int64_t kb = k * kB;
  load_diag_block(T, S32, kb, lr, li);
  double vr = 0.0, vi = 0.0;
  if (t < kB) {
    vr = v[2 * (kb + t)];
    vi = v[2 * (kb + t) + 1];
  }
  for (int j = kB - 1; j >= 0; --j) {
    if (t == j) {
      vr /= lr[j][j];
      vi /= lr[j][j];
    }
    const double xr = __shfl(vr, j, 64), xi = __shfl(vi, j, 64);
    if (t < j) {
      // v_t -= conj(L[j][t]) x_j
      vr -= lr[j][t] * xr + li[j][t] * xi;
      vi -= lr[j][t] * xi - li[j][t] * xr;
    }
  }
  if (t < kB) {
    v[2 * (kb + t)] = vr;
    v[2 * (kb + t) + 1] = vi;
  }
}

// v_j -= sum_l conj(L[kb + l][j]) x_l for columns j left of block k
__global__ void bsolve_update_kernel(const double* __restrict__ T, int64_t S32, int64_t k,
                                     double* __restrict__ v) {
  const int64_t kb = k * kB;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= kb) return;
  double vr = v[2 * j], vi = v[2 * j + 1];
  for (int l = 0; l < kB; ++l) {
    const double Lr = T[((kb + l) * S32 + j) * 2], Li = T[((kb + l) * S32 + j) * 2 + 1];
    const double xr = v[2 * (kb + l)], xi = v[2 * (kb + l) + 1];
    vr -= Lr * xr + Li * xi;
    vi -= Lr * xi - Li * xr;
  }
  v[2 * j] = vr;
  v[2 * j + 1] = vi;
}

// dtheta[k] = -dtau sum_s conj(Ob[s][k]) x[s]   (one wavefront per parameter)
template <typename RG>
__global__ __launch_bounds__(256) void dtheta_kernel(const RG* __restrict__ Tre,
                                                     const RG* __restrict__ Tim, int64_t P,
                                                     int64_t S32, const double* __restrict__ x,
                                                     double dtau, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t k = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= P) return;
  double sr = 0.0, si = 0.0;
  for (int64_t s = lane; s < S32; s += 64) {
    const double ar = (double)Tre[k * S32 + s], ai = (double)Tim[k * S32 + s];
    const double xr = x[2 * s], xi = x[2 * s + 1];
    sr += ar * xr + ai * xi;
    si += ar * xi - ai * xr;
  }
  sr = wave_sum(sr);
  si = wave_sum(si);
  if (lane == 0) {
    out[2 * k] = -dtau * sr;
    out[2 * k + 1] = -dtau * si;
  }
}

inline size_t al(size_t v) { return (v + 255) / 256 * 256; }
inline int64_t r32(int64_t v) { return (v + kB - 1) / kB * kB; }
inline int64_t r4(int64_t v) { return (v + 3) / 4 * 4; }

template <typename RO, typename RG>
hipError_t sr_run(const nqs_ctx* c, const void* Ov, const double* el, int64_t S, double lambda,
                  double dtau, double* out, void* ws, hipStream_t st, int* flag_host) {
  const RO* O = (const RO*)Ov;
  const int64_t P = c->P, P4 = r4(P), S32 = r32(S), nblk = S32 / kB;
  char* p = (char*)ws;
  double* T = (double*)p;
  p += al((size_t)S32 * S32 * 16);
  RG* Tre = (RG*)p;
  p += al((size_t)P4 * S32 * sizeof(RG));
  RG* Tim = (RG*)p;
  p += al((size_t)P4 * S32 * sizeof(RG));
  double* v = (double*)p;
  p += al((size_t)S32 * 16);
  double* mean = (double*)p;
  p += al((size_t)P * 16);
  int* flag = (int*)p;

  hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), st);
  if (e != hipSuccess) return e;
  colmean_kernel<RO><<<(unsigned)((P + 255) / 256), 256, 0, st>>>(O, S, P, mean);
  dim3 gct((unsigned)(S32 / 32), (unsigned)((P4 + 31) / 32));
  center_t_kernel<RO, RG><<<gct, 256, 0, st>>>(O, S, P, P4, S32, mean, 1.0 / std::sqrt((double)S),
                                               Tre, Tim);
  eps_kernel<<<1, 1024, 0, st>>>(el, S, S32, v);
  const int64_t ntri = nblk * (nblk + 1) / 2;
  prof_begin(c, K_GRAM, st);
  if constexpr (sizeof(RG) == 4) {
    const int64_t ntile = (S32 + kGT - 1) / kGT;
    gram_tile_kernel<<<(unsigned)(ntile * (ntile + 1) / 2), 256, 0, st>>>(
        (const float*)Tre, (const float*)Tim, P4, S32, ntile, lambda, T);
  } else {
    gram_kernel<RG><<<(unsigned)((ntri + 3) / 4), 256, 0, st>>>(Tre, Tim, P4, S32, nblk, lambda, T);
  }
  prof_end(c, K_GRAM, st);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  prof_begin(c, K_CHOL, st);
  // right-looking, in panels of kPanel block columns: each block column is
  // factored, solved below and applied to the rest of its panel; the panel
  // as a whole then updates the trailing matrix in one rank-(32 kPanel) pass
  for (int64_t K0 = 0; K0 < nblk; K0 += kPanel) {
    const int64_t K1 = std::min<int64_t>(K0 + kPanel, nblk);
    for (int64_t k = K0; k < K1; ++k) {
      potrf_diag_kernel<<<1, 256, 0, st>>>(T, S32, k, flag);
      const int64_t rows = S32 - (k + 1) * kB;
      if (rows > 0) trsm_panel_kernel<<<(unsigned)((rows + 255) / 256), 256, 0, st>>>(T, S32, k);
      if (k + 1 < K1) {
        const int jn = (int)(K1 - k - 1);
        int64_t nt = 0;
        for (int jj = 0; jj < jn; ++jj) nt += nblk - (k + 1 + jj);
        herk_update_kernel<<<(unsigned)((nt + 3) / 4), 256, 0, st>>>(T, S32, k, 1, k + 1, jn, nblk);
      }
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (K1 < nblk) {
      const int64_t m = nblk - K1, nt = m * (m + 1) / 2;
      herk_update_kernel<<<(unsigned)((nt + 3) / 4), 256, 0, st>>>(T, S32, K0, (int)(K1 - K0), K1,
                                                                  0, nblk);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  for (int64_t k = 0; k < nblk; ++k) {
    fsolve_diag_kernel<<<1, 64, 0, st>>>(T, S32, k, v);
    const int64_t rows = S32 - (k + 1) * kB;
    if (rows > 0) fsolve_update_kernel<<<(unsigned)((rows + 255) / 256), 256, 0, st>>>(T, S32, k, v);
  }
  for (int64_t k = nblk - 1; k >= 0; --k) {
    bsolve_diag_kernel<<<1, 64, 0, st>>>(T, S32, k, v);
    if (k > 0) bsolve_update_kernel<<<(unsigned)((k * kB + 255) / 256), 256, 0, st>>>(T, S32, k, v);
  }
  prof_end(c, K_CHOL, st);
  dtheta_kernel<RG><<<(unsigned)((P + 3) / 4), 256, 0, st>>>(Tre, Tim, P, S32, v, dtau, out);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(flag_host, flag, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return e;
  return hipStreamSynchronize(st);
}

}  // namespace

size_t sr_workspace_bytes(const nqs_ctx* c, int64_t S) {
  const int64_t S32 = r32(std::max<int64_t>(S, 1)), P4 = r4(c->P);
  const size_t rg = c->prec == NQS_FP64 ? 8 : 4;
  return al((size_t)S32 * S32 * 16) + 2 * al((size_t)P4 * S32 * rg) + al((size_t)S32 * 16) +
         al((size_t)c->P * 16) + al(64);
}

}  // namespace nqs

using namespace nqs;

extern "C" nqs_status nqs_sr_solve(nqs_ctx* c, const void* O, const double* eloc, int64_t S,
                                   double lambda, double dtau, double* dtheta_out, void* ws,
                                   size_t ws_bytes, hipStream_t st) {
  if (!c) return NQS_ERR_ARG;
  auto fail = [&](nqs_status s, const std::string& m) {
    c->last_error = m;
    return s;
  };
  if (S < 1 || !O || !eloc || !dtheta_out) return fail(NQS_ERR_ARG, "sr_solve: bad arguments");
  if (!(lambda >= 0.0) || !std::isfinite(lambda) || !std::isfinite(dtau))
    return fail(NQS_ERR_ARG, "sr_solve: lambda must be finite and >= 0, dtau finite");
  const size_t need = sr_workspace_bytes(c, S);
  if (!ws || ws_bytes < need)
    return fail(NQS_ERR_ARG, "sr_solve: workspace too small: need " + std::to_string(need));
  int flag = 0;
  prof_begin(c, K_SR, st);
  const hipError_t e =
      c->prec == NQS_FP64
          ? sr_run<double, double>(c, O, eloc, S, lambda, dtau, dtheta_out, ws, st, &flag)
          : sr_run<float, float>(c, O, eloc, S, lambda, dtau, dtheta_out, ws, st, &flag);
  prof_end(c, K_SR, st);
  if (e != hipSuccess) return fail(NQS_ERR_DEVICE, std::string("sr_solve: ") + hipGetErrorString(e));
  if (flag) return fail(NQS_ERR_NOT_PD, "sr_solve: Gram matrix is not positive definite");
  return NQS_OK;
}
