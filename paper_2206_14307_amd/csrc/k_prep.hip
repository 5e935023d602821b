// Parameter preparation (once per parameter set): precision-specific copies
// of W laid out as MFMA A-operand fragments, biases, and the per-bond tables
// of the exchange identity
//   cosh(theta + s D) = cosh(theta) cosh(D) (1 + s tanh(theta) tanh(D)),
// D_h = W_h,p - W_h,q for bond (p, q), s = +-1, which turns the amplitude
// ratio of a bond exchange (Sec. 3.2, Eq. (10)) into a product with no
// transcendental functions.  Tables are computed in FP64 and rounded once.
#include "device_common.h"
#include "nqs_internal.h"

namespace nqs {

namespace {

__device__ inline double2 ctanh64(double x, double y) {
  // tanh(x+iy) = (sinh 2x + i sin 2y) / (cosh 2x + cos 2y), scaled for large |x|
  if (fabs(x) > 20.0) return make_double2(x > 0 ? 1.0 : -1.0, 0.0);
  const double d = cosh(2.0 * x) + cos(2.0 * y);
  return make_double2(sinh(2.0 * x) / d, sin(2.0 * y) / d);
}

__device__ inline double2 ccosh64(double x, double y) {
  return make_double2(cosh(x) * cos(y), sinh(x) * sin(y));
}

__device__ inline double2 cexp64(double x, double y) {
  const double e = exp(x);
  return make_double2(e * cos(y), e * sin(y));
}

// params layout per RBM: [W (M x N) | a (N) | b (M)] (complex double)
__device__ inline double2 Wval(const double2* p, int Prbm, int M, int N, int h, int site) {
  const int k = h / M, hh = h % M;
  return p[(size_t)k * Prbm + (size_t)hh * N + site];
}

// Interleaved A matrix: row 2h = Re W_h, row 2h+1 = Im W_h.  16x16x4 MFMA
// fragment: lane l of K-step kk holds A[16 ht + l%16][4 kk + l/16].
template <typename R>
__global__ void prep_wfrag_kernel(const double2* p, int Prbm, int M, int N, int n_htiles, int nk,
                                  R* out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)n_htiles * nk * 64;
  if (idx >= total) return;
  const int l = idx % 64, kk = (idx / 64) % nk, ht = idx / (64 * nk);
  const int row = 16 * ht + logical_row<R>(l % 16);
  const int site = 4 * kk + l / 16;
  double v = 0.0;
  if (site < N) {
    const double2 w = Wval(p, Prbm, M, N, row / 2, site);
    v = (row & 1) ? w.y : w.x;
  }
  out[idx] = (R)v;
}

// Split-BF16 fragments for the 16x16x32 BF16 MFMA: the K axis is
// [hi part over sites 0..N-1 | lo part over sites 0..N-1 | zero padding];
// lane l of K-step kk holds A[16 ht + l%16][32 kk + 8 (l/16) + e], e < 8.
// hi = bf16(w), lo = bf16(w - hi) with w the FP32 value, round to nearest even.
__device__ inline unsigned short bf16_rne(float f) {
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline float bf16_to_f(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }

__global__ void prep_wfrag_bf16_kernel(const double2* p, int Prbm, int M, int N, int n_htiles,
                                       int nk, unsigned short* out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)n_htiles * nk * 64;
  if (idx >= total) return;
  const int l = idx % 64, kk = (idx / 64) % nk, ht = idx / (64 * nk);
  const int row = 16 * ht + (l % 16);
  for (int e = 0; e < 8; ++e) {
    const int kap = 32 * kk + 8 * (l / 16) + e;
    unsigned short v = 0;
    if (kap < 2 * N) {
      const int site = kap < N ? kap : kap - N;
      const double2 w = Wval(p, Prbm, M, N, row / 2, site);
      const float wf = (float)((row & 1) ? w.y : w.x);
      const unsigned short hi = bf16_rne(wf);
      v = kap < N ? hi : bf16_rne(wf - bf16_to_f(hi));
    }
    out[idx * 8 + e] = v;
  }
}

// FP32 models: fragments of [W_hi | W_mid | W_lo | 0] along the K axis for
// the three-term BF16 form of theta (hi = the FP32 W with its low 16 bits
// cleared, mid the same of W - hi, lo = W - hi - mid, exact in BF16).
__global__ void prep_wfrag_x3_kernel(const double2* p, int Prbm, int M, int N, int n_htiles,
                                     int nk3, unsigned short* out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)n_htiles * nk3 * 64;
  if (idx >= total) return;
  const int l = idx % 64, kk = (idx / 64) % nk3, ht = idx / (64 * nk3);
  const int row = 16 * ht + (l % 16);
  for (int e = 0; e < 8; ++e) {
    const int kap = 32 * kk + 8 * (l / 16) + e;
    unsigned short v = 0;
    if (kap < 3 * N) {
      const double2 w = Wval(p, Prbm, M, N, row / 2, kap % N);
      const float wf = (float)((row & 1) ? w.y : w.x);
      const float hi = __uint_as_float(__float_as_uint(wf) & 0xffff0000u);
      const float r1 = wf - hi;
      const float mid = __uint_as_float(__float_as_uint(r1) & 0xffff0000u);
      const float part = kap < N ? hi : kap < 2 * N ? mid : r1 - mid;
      v = (unsigned short)(__float_as_uint(part) >> 16);
    }
    out[idx * 8 + e] = v;
  }
}

// FP32 models, fused gradient kernel: the same three terms with the K slots
// grouped by site.  Lane l = (q, c) of MFMA m holds, at slot e, row 16 ht + c
// and flat slot f = 8 m + e of lane group q: hi (f even) or mid (f odd) of site
// 4 (f / 2) + q for f < 2 N/4, lo of site 4 (f - 2 N/4) + q for f < 3 N/4, else
// zero.  N is a multiple of 4.
__global__ void prep_wfrag_s3_kernel(const double2* p, int Prbm, int M, int N, int n_htiles,
                                     int nm, unsigned short* out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)n_htiles * nm * 64;
  if (idx >= total) return;
  const int l = idx % 64, mm = (idx / 64) % nm, ht = idx / (64 * nm);
  const int row = 16 * ht + (l % 16), q = l / 16, ni = N / 4;
  for (int e = 0; e < 8; ++e) {
    const int f = 8 * mm + e;
    int i = -1, term = 0;
    if (f < 2 * ni) {
      i = f / 2;
      term = f & 1;
    } else if (f < 3 * ni) {
      i = f - 2 * ni;
      term = 2;
    }
    unsigned short v = 0;
    if (i >= 0) {
      const double2 w = Wval(p, Prbm, M, N, row / 2, 4 * i + q);
      const float wf = (float)((row & 1) ? w.y : w.x);
      const float hi = __uint_as_float(__float_as_uint(wf) & 0xffff0000u);
      const float r1 = wf - hi;
      const float mid = __uint_as_float(__float_as_uint(r1) & 0xffff0000u);
      const float part = term == 0 ? hi : term == 1 ? mid : r1 - mid;
      v = (unsigned short)(__float_as_uint(part) >> 16);
    }
    out[idx * 8 + e] = v;
  }
}

template <typename R>
__global__ void prep_bias_kernel(const double2* p, int Prbm, int K, int M, int N, int use_bias,
                                 R* bias, R* avec) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < K * M) {
    const int k = idx / M, hh = idx % M;
    double2 b = make_double2(0.0, 0.0);
    if (use_bias) b = p[(size_t)k * Prbm + (size_t)M * N + N + hh];
    bias[2 * idx] = (R)b.x;
    bias[2 * idx + 1] = (R)b.y;
  }
  if (idx < K * N) {
    const int k = idx / N, j = idx % N;
    double2 a = make_double2(0.0, 0.0);
    if (use_bias) a = p[(size_t)k * Prbm + (size_t)M * N + j];
    avec[2 * idx] = (R)a.x;
    avec[2 * idx + 1] = (R)a.y;
  }
}

// Tpm[beta][0][h] = tanh(D_h,beta), Tpm[beta][1][h] = -tanh(D_h,beta).
template <typename R>
__global__ void prep_T_kernel(const double2* p, int Prbm, int M, int N, int KM, int NB,
                              const int32_t* bonds, R* Tpm) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)NB * KM) return;
  const int beta = idx / KM, h = idx % KM;
  const double2 wp = Wval(p, Prbm, M, N, h, bonds[2 * beta]);
  const double2 wq = Wval(p, Prbm, M, N, h, bonds[2 * beta + 1]);
  const double2 t = ctanh64(wp.x - wq.x, wp.y - wq.y);
  R* row = Tpm + (size_t)beta * 2 * KM * 2;
  row[2 * h] = (R)t.x;
  row[2 * h + 1] = (R)t.y;
  row[2 * KM + 2 * h] = (R)(-t.x);
  row[2 * KM + 2 * h + 1] = (R)(-t.y);
}

// Bond rows of the fused E_loc kernel.  The hidden units of RBM k are split
// into eight lane streams h = kM + 8j + r (r = 2q + u, j < M/8); the fused
// kernel multiplies one stream per (lane, bond) and joins the eight streams
// across lanes.  Two forms of the factor s + t T_h are tabulated:
//   direct      row = [T_h, h < KM | start values]
//   reciprocal  row = [U_h = 1/T_h | start values], s + t T = T (t + s U),
// each with ROW = 2 KM + 18 K reals.  Start values (k, r) at 2KM + 16k + 2r
// begin each stream's product: 1 (direct) or C_kr = prod_j T (reciprocal),
// and stream r = 0 also carries the bond prefactor
//   F_s = (J/2) e^{s A} prod_h cosh D_h   (A = a_p - a_q, bias term)
// for s = +1; the s = -1 start of stream 0 sits at 2KM + 16K + 2k.
// In the reciprocal form the partial products along a stream equal (finished
// factors) x (suffix product of T), so that form is used only if every suffix
// product |prod_{i >= j} T_i| lies in [2^lg_lo, 2^lg_hi]; flag[1] is set
// otherwise.
template <typename R>
__global__ void prep_fused_rows_kernel(const double2* p, int Prbm, int K, int M, int N, int NB,
                                       int use_bias, const int32_t* bonds, const double* bond_J,
                                       double lg_lo, double lg_hi, R* Tdir, R* Urec,
                                       double* flag) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= NB * K * 8) return;
  const int beta = idx / (K * 8), k = (idx / 8) % K, r = idx % 8;
  const int KM = K * M, TPR = M / 8, ROW = 2 * KM + 18 * K;
  const int bp = bonds[2 * beta], bq = bonds[2 * beta + 1];
  R* dir = Tdir + (size_t)beta * ROW;
  R* rec = Urec + (size_t)beta * ROW;
  double cr = 1.0, ci = 0.0, lg = 0.0;
  bool ok = true;
  for (int j = TPR - 1; j >= 0; --j) {
    const int h = k * M + 8 * j + r;
    const double2 wp = Wval(p, Prbm, M, N, h, bp);
    const double2 wq = Wval(p, Prbm, M, N, h, bq);
    const double2 t = ctanh64(wp.x - wq.x, wp.y - wq.y);
    const double a2 = t.x * t.x + t.y * t.y;
    const double nr = cr * t.x - ci * t.y;
    ci = cr * t.y + ci * t.x;
    cr = nr;
    lg += 0.5 * log2(a2);                         // -inf for T = 0
    ok = ok && lg >= lg_lo && lg <= lg_hi;
    dir[2 * h] = (R)t.x;
    dir[2 * h + 1] = (R)t.y;
    rec[2 * h] = a2 > 0.0 ? (R)(t.x / a2) : (R)0;
    rec[2 * h + 1] = a2 > 0.0 ? (R)(-t.y / a2) : (R)0;
  }
  if (!ok) flag[1] = 1.0;
  double fr[2] = {1.0, 1.0}, fi[2] = {0.0, 0.0};
  if (r == 0) {
    double hr = 1.0, hi = 0.0;
    for (int hh = 0; hh < M; ++hh) {
      const double2 wp = Wval(p, Prbm, M, N, k * M + hh, bp);
      const double2 wq = Wval(p, Prbm, M, N, k * M + hh, bq);
      const double2 c = ccosh64(wp.x - wq.x, wp.y - wq.y);
      const double nr = hr * c.x - hi * c.y;
      hi = hr * c.y + hi * c.x;
      hr = nr;
    }
    double ar = 0.0, ai = 0.0;
    if (use_bias) {
      const double2 ap = p[(size_t)k * Prbm + (size_t)M * N + bp];
      const double2 aq = p[(size_t)k * Prbm + (size_t)M * N + bq];
      ar = ap.x - aq.x;
      ai = ap.y - aq.y;
    }
    const double hJ = 0.5 * bond_J[beta];
    for (int s = 0; s < 2; ++s) {
      const double sg = s == 0 ? 1.0 : -1.0;
      const double2 e = cexp64(sg * ar, sg * ai);
      fr[s] = hJ * (e.x * hr - e.y * hi);
      fi[s] = hJ * (e.x * hi + e.y * hr);
    }
  }
  const int st = 2 * KM + 16 * k + 2 * r;
  dir[st] = (R)fr[0];
  dir[st + 1] = (R)fi[0];
  rec[st] = (R)(cr * fr[0] - ci * fi[0]);
  rec[st + 1] = (R)(cr * fi[0] + ci * fr[0]);
  if (r == 0) {
    const int sn = 2 * KM + 16 * K + 2 * k;
    dir[sn] = (R)fr[1];
    dir[sn + 1] = (R)fi[1];
    rec[sn] = (R)(cr * fr[1] - ci * fi[1]);
    rec[sn + 1] = (R)(cr * fi[1] + ci * fr[1]);
  }
}

// F[k][beta][s] = (J_beta / 2) exp(s A_beta) prod_h cosh(D_h,beta), s = +1 (0), -1 (1).
template <typename R>
__global__ void prep_F_kernel(const double2* p, int Prbm, int K, int M, int N, int NB, int use_bias,
                              const int32_t* bonds, const double* bond_J, R* F) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= K * NB) return;
  const int k = idx / NB, beta = idx % NB;
  const int bp = bonds[2 * beta], bq = bonds[2 * beta + 1];
  double cr = 1.0, ci = 0.0;
  for (int hh = 0; hh < M; ++hh) {
    const double2 wp = Wval(p, Prbm, M, N, k * M + hh, bp);
    const double2 wq = Wval(p, Prbm, M, N, k * M + hh, bq);
    const double2 c = ccosh64(wp.x - wq.x, wp.y - wq.y);
    const double nr = cr * c.x - ci * c.y;
    ci = cr * c.y + ci * c.x;
    cr = nr;
  }
  double ar = 0.0, ai = 0.0;
  if (use_bias) {
    const double2 ap = p[(size_t)k * Prbm + (size_t)M * N + bp];
    const double2 aq = p[(size_t)k * Prbm + (size_t)M * N + bq];
    ar = ap.x - aq.x;
    ai = ap.y - aq.y;
  }
  const double hJ = 0.5 * bond_J[beta];
  for (int s = 0; s < 2; ++s) {
    const double sg = s == 0 ? 1.0 : -1.0;
    const double2 e = cexp64(sg * ar, sg * ai);
    R* o = F + ((size_t)(k * NB + beta) * 2 + s) * 2;
    o[0] = (R)(hJ * (e.x * cr - e.y * ci));
    o[1] = (R)(hJ * (e.x * ci + e.y * cr));
  }
}

// Site-pair tables of the sampler's exchange move (up site at image position
// p, down site at q, so theta -> theta - (W_p - W_q)):
// Tpair[p][q][h] = tanh(W_hp - W_hq), Fpair[k][p][q] = exp(-(a_p - a_q)) prod_h cosh(W_hp - W_hq).
template <typename R>
__global__ void prep_Tpair_kernel(const double2* p, int Prbm, int M, int N, int KM, R* Tpair) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)N * N * KM) return;
  const int h = idx % KM;
  const int pq = idx / KM;
  const int sp = pq / N, sq = pq % N;
  const double2 wp = Wval(p, Prbm, M, N, h, sp);
  const double2 wq = Wval(p, Prbm, M, N, h, sq);
  const double2 t = ctanh64(wp.x - wq.x, wp.y - wq.y);
  Tpair[2 * idx] = (R)t.x;
  Tpair[2 * idx + 1] = (R)t.y;
}

template <typename R>
__global__ void prep_Fpair_kernel(const double2* p, int Prbm, int K, int M, int N, int use_bias,
                                  R* Fpair) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= K * N * N) return;
  const int k = idx / (N * N), sp = (idx / N) % N, sq = idx % N;
  double cr = 1.0, ci = 0.0;
  for (int hh = 0; hh < M; ++hh) {
    const double2 wp = Wval(p, Prbm, M, N, k * M + hh, sp);
    const double2 wq = Wval(p, Prbm, M, N, k * M + hh, sq);
    const double2 c = ccosh64(wp.x - wq.x, wp.y - wq.y);
    const double nr = cr * c.x - ci * c.y;
    ci = cr * c.y + ci * c.x;
    cr = nr;
  }
  double ar = 0.0, ai = 0.0;
  if (use_bias) {
    const double2 ap = p[(size_t)k * Prbm + (size_t)M * N + sp];
    const double2 aq = p[(size_t)k * Prbm + (size_t)M * N + sq];
    ar = ap.x - aq.x;
    ai = ap.y - aq.y;
  }
  const double2 e = cexp64(-ar, -ai);
  Fpair[2 * idx] = (R)(e.x * cr - e.y * ci);
  Fpair[2 * idx + 1] = (R)(e.x * ci + e.y * cr);
}

template <typename R>
hipError_t prep_pairs_typed(const nqs_ctx* c, hipStream_t st) {
  const double2* p = reinterpret_cast<const double2*>(c->par.params);
  const int64_t nT = (int64_t)c->N * c->N * c->KM;
  prep_Tpair_kernel<R><<<(unsigned)((nT + 255) / 256), 256, 0, st>>>(p, c->P_rbm, c->M, c->N,
                                                                       c->KM, (R*)c->par.Tpair);
  const int nF = c->K * c->N * c->N;
  prep_Fpair_kernel<R><<<(nF + 63) / 64, 64, 0, st>>>(p, c->P_rbm, c->K, c->M, c->N,
                                                      c->d.use_bias, (R*)c->par.Fpair);
  return hipGetLastError();
}

__global__ void check_finite_kernel(const double* p, int64_t n, double* flag) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(p[i])) flag[0] = 1.0;
}

template <typename R>
hipError_t prep_typed(const nqs_ctx* c, hipStream_t st) {
  const double2* p = reinterpret_cast<const double2*>(c->par.params);
  const int64_t nfrag = (int64_t)c->n_htiles * c->nk * 64;
  if (c->prec == NQS_BF16X2) {
    prep_wfrag_bf16_kernel<<<(nfrag + 255) / 256, 256, 0, st>>>(
        p, c->P_rbm, c->M, c->N, c->n_htiles, c->nk, (unsigned short*)c->par.wfrag);
  } else {
    prep_wfrag_kernel<R><<<(nfrag + 255) / 256, 256, 0, st>>>(p, c->P_rbm, c->M, c->N,
                                                               c->n_htiles, c->nk, (R*)c->par.wfrag);
  }
  if (c->par.wfrag3) {
    const int nk3 = (3 * c->N + 31) / 32;
    const int64_t nf3 = (int64_t)c->n_htiles * nk3 * 64;
    prep_wfrag_x3_kernel<<<(nf3 + 255) / 256, 256, 0, st>>>(
        p, c->P_rbm, c->M, c->N, c->n_htiles, nk3, (unsigned short*)c->par.wfrag3);
  }
  if (c->par.wfrag_s3) {
    const int nm = (3 * (c->N / 4) + 7) / 8;
    const int64_t nfs = (int64_t)c->n_htiles * nm * 64;
    prep_wfrag_s3_kernel<<<(nfs + 255) / 256, 256, 0, st>>>(
        p, c->P_rbm, c->M, c->N, c->n_htiles, nm, (unsigned short*)c->par.wfrag_s3);
  }
  const int nb = (std::max(c->K * c->M, c->K * c->N) + 255) / 256;
  prep_bias_kernel<R><<<nb, 256, 0, st>>>(p, c->P_rbm, c->K, c->M, c->N, c->d.use_bias,
                                          (R*)c->par.bias, (R*)c->par.avec);
  const int64_t nT = (int64_t)c->NB * c->KM;
  prep_T_kernel<R><<<(nT + 255) / 256, 256, 0, st>>>(p, c->P_rbm, c->M, c->N, c->KM, c->NB,
                                                      c->dev.bonds, (R*)c->par.Tpm);
  prep_F_kernel<R><<<(c->K * c->NB + 63) / 64, 64, 0, st>>>(
      p, c->P_rbm, c->K, c->M, c->N, c->NB, c->d.use_bias, c->dev.bonds, c->dev.bond_J,
      (R*)c->par.F);
  // suffix-product range of the reciprocal form: FP32 keeps 2^+-96 clear of
  // overflow and of the denormal range; FP64 2^+-900
  const double lg = sizeof(R) == 4 ? 96.0 : 900.0;
  prep_fused_rows_kernel<R><<<(c->NB * c->K * 8 + 63) / 64, 64, 0, st>>>(
      p, c->P_rbm, c->K, c->M, c->N, c->NB, c->d.use_bias, c->dev.bonds, c->dev.bond_J, -lg, lg,
      (R*)c->par.Tdir, (R*)c->par.Urec, c->par.flag);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_check_finite(const double* p, int64_t n, double* flag, hipStream_t st) {
  check_finite_kernel<<<64, 256, 0, st>>>(p, n, flag);
  return hipGetLastError();
}

hipError_t launch_prep(const nqs_ctx* c, hipStream_t st) {
  hipError_t e = c->prec == NQS_FP64 ? prep_typed<double>(c, st) : prep_typed<float>(c, st);
  if (e != hipSuccess) return e;
  return launch_prep_pairs(c, st);
}

hipError_t launch_prep_pairs(const nqs_ctx* c, hipStream_t st) {
  return c->prec == NQS_FP64 ? prep_pairs_typed<double>(c, st) : prep_pairs_typed<float>(c, st);
}

}  // namespace nqs
