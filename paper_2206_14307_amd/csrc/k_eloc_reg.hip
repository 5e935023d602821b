// Local energies for models whose tanh(theta) row fits in registers
// (K*M <= 128 hidden units): persistent workgroups keep the +tanh(D) bond
// table in LDS for the whole launch and every lane keeps its image's
// tanh(theta) row in VGPRs, so the exchange product of Sec. 3.2, Eq. (10)
// reads one LDS word pair per factor and nothing from HBM.
//
// Sign folding: with s = +-1 and M even (M is a multiple of 8),
//   prod_h (1 + s t_h T_h) = prod_h (s + t_h T_h),
// so the sign enters as the addend of the first FMA and only the +T table
// is stored (8 VALU operations per factor, as with a pre-signed table).
//
// Lane = (image g of a 32-image tile, half of the antiparallel bond list);
// two bonds per pass and two partial products per bond (even / odd h) give
// four independent FMA chains per lane.
#include "device_common.h"
#include "nqs_internal.h"
#include "pair_list.h"
#include "hops.h"

namespace nqs {

namespace {

constexpr int kRegWaves = 8;

template <typename R> struct Vec2;
template <> struct Vec2<float> { using type = float4; };   // two complex floats
template <> struct Vec2<double> { using type = double2; }; // one complex double

template <typename R, int N, int K, int M>
struct RegCfg {
  static constexpr int NB = 4 * N;
  static constexpr int KM = K * M;
  // T row stride in R units: 2 KM plus padding that staggers LDS banks
  static constexpr int STRIDE = 2 * KM + (sizeof(R) == 4 ? 4 : 2);
  static constexpr size_t LDS = (size_t)NB * STRIDE * sizeof(R) + (size_t)kRegWaves * NB * 2;
};

__device__ __forceinline__ int build_list(const int8_t* srow, const int32_t* bonds, int NB,
                                          int16_t* list, int lane) {
  int n = 0;
  for (int base = 0; base < NB; base += 64) {
    const int b = base + lane;
    bool anti = false;
    if (b < NB) anti = srow[bonds[2 * b]] != srow[bonds[2 * b + 1]];
    const unsigned long long m = __ballot(anti);
    const int pos = __popcll(m & ((1ull << lane) - 1ull));
    if (anti) list[n + pos] = (int16_t)b;
    n += __popcll(m);
  }
  wave_sync_lds();
  return n;
}

// P <- P * (s + t T)
template <typename R>
__device__ __forceinline__ void mul_s_plus(R& pr, R& pi, R s, R tr, R ti, R Tr, R Ti) {
  const R a = fmaf_t(tr, Tr, fmaf_t(-ti, Ti, s));
  const R b = fmaf_t(tr, Ti, ti * Tr);
  const R nr = fmaf_t(pr, a, -(pi * b));
  pi = fmaf_t(pr, b, pi * a);
  pr = nr;
}

template <typename R, int N, int K, int M>
__global__ __launch_bounds__(64 * kRegWaves) void eloc_reg_kernel(
    const int8_t* __restrict__ spins, int64_t S, int G, int n_htiles,
    const int32_t* __restrict__ bonds, const int32_t* __restrict__ bmap, const R* __restrict__ t,
    const R* __restrict__ w, const R* __restrict__ Tpm, const R* __restrict__ F,
    double* __restrict__ partial) {
  using Cfg = RegCfg<R, N, K, M>;
  constexpr int NB = Cfg::NB, KM = Cfg::KM, ST = Cfg::STRIDE;
  __shared__ __align__(16) R Tl[NB * ST];
  __shared__ int16_t lists[kRegWaves][NB];

  for (int idx = threadIdx.x; idx < NB * KM; idx += blockDim.x) {
    const int beta = idx / KM, h = idx % KM;
    const R* src = Tpm + ((size_t)beta * 2 * KM + h) * 2;   // + sign rows
    Tl[beta * ST + 2 * h] = src[0];
    Tl[beta * ST + 2 * h + 1] = src[1];
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int ntiles = G / 32;
  const int64_t n_items = S * ntiles;
  const int64_t stride = (int64_t)gridDim.x * kRegWaves;
  int16_t* list = lists[wv];
  for (int64_t item = (int64_t)blockIdx.x * kRegWaves + wv; item < n_items; item += stride) {
    const int64_t s = item / ntiles;
    const int tile = (int)(item % ntiles);
    const int g = tile * 32 + (lane & 31);
    const int half = lane >> 5;
    const int8_t* srow = spins + s * N;
    const int nc = build_list(srow, bonds, NB, list, lane);

    R tr[KM], ti[KM];
#pragma unroll
    for (int ht = 0; ht < KM / 8; ++ht) {
      const R* tp = t + (((size_t)s * n_htiles + ht) * G + g) * 16;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        tr[8 * ht + e] = tp[2 * e];
        ti[8 * ht + e] = tp[2 * e + 1];
      }
    }
    R wr[K], wi[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      wr[k] = w[(((size_t)s * K + k) * G + g) * 2];
      wi[k] = w[(((size_t)s * K + k) * G + g) * 2 + 1];
    }

    double accr = 0.0, acci = 0.0;
    for (int i0 = half; i0 < nc; i0 += 4) {
      int beta[2], sidx[2];
      R sgn[2], valid[2];
#pragma unroll
      for (int n = 0; n < 2; ++n) {
        const int ii = i0 + 2 * n;
        valid[n] = ii < nc ? R(1) : R(0);
        const int b = list[ii < nc ? ii : i0];
        const int v = bmap[(size_t)g * NB + b];
        beta[n] = v >> 1;
        const int s_b = -(int)srow[bonds[2 * b]];
        const int sp = (v & 1) ? -s_b : s_b;
        sgn[n] = (R)sp;
        sidx[n] = sp > 0 ? 0 : 1;
      }
      const R* T0 = Tl + beta[0] * ST;
      const R* T1 = Tl + beta[1] * ST;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        R pe0r = 1, pe0i = 0, po0r = 1, po0i = 0, pe1r = 1, pe1i = 0, po1r = 1, po1i = 0;
#pragma unroll
        for (int hh = 0; hh < M; hh += 2) {
          const int h = k * M + hh;
          if constexpr (sizeof(R) == 4) {
            const float4 a = *reinterpret_cast<const float4*>(T0 + 2 * h);
            const float4 c = *reinterpret_cast<const float4*>(T1 + 2 * h);
            mul_s_plus<R>(pe0r, pe0i, sgn[0], tr[h], ti[h], a.x, a.y);
            mul_s_plus<R>(po0r, po0i, sgn[0], tr[h + 1], ti[h + 1], a.z, a.w);
            mul_s_plus<R>(pe1r, pe1i, sgn[1], tr[h], ti[h], c.x, c.y);
            mul_s_plus<R>(po1r, po1i, sgn[1], tr[h + 1], ti[h + 1], c.z, c.w);
          } else {
            const double2 a0 = *reinterpret_cast<const double2*>(T0 + 2 * h);
            const double2 a1 = *reinterpret_cast<const double2*>(T0 + 2 * h + 2);
            const double2 c0 = *reinterpret_cast<const double2*>(T1 + 2 * h);
            const double2 c1 = *reinterpret_cast<const double2*>(T1 + 2 * h + 2);
            mul_s_plus<R>(pe0r, pe0i, sgn[0], tr[h], ti[h], a0.x, a0.y);
            mul_s_plus<R>(po0r, po0i, sgn[0], tr[h + 1], ti[h + 1], a1.x, a1.y);
            mul_s_plus<R>(pe1r, pe1i, sgn[1], tr[h], ti[h], c0.x, c0.y);
            mul_s_plus<R>(po1r, po1i, sgn[1], tr[h + 1], ti[h + 1], c1.x, c1.y);
          }
        }
#pragma unroll
        for (int n = 0; n < 2; ++n) {
          const R per = n ? pe1r : pe0r, pei = n ? pe1i : pe0i;
          const R por = n ? po1r : po0r, poi = n ? po1i : po0i;
          const R pr = per * por - pei * poi, pi = per * poi + pei * por;
          const R* f = F + (((size_t)k * NB + beta[n]) * 2 + sidx[n]) * 2;
          const R fr = f[0] * wr[k] - f[1] * wi[k], fi = f[0] * wi[k] + f[1] * wr[k];
          accr += (double)(valid[n] * (fr * pr - fi * pi));
          acci += (double)(valid[n] * (fr * pi + fi * pr));
        }
      }
    }
    accr = wave_sum(accr);
    acci = wave_sum(acci);
    if (lane == 0) {
      partial[2 * item] = accr;
      partial[2 * item + 1] = acci;
    }
    wave_sync_lds();   // the list is rewritten for the next item
  }
}

template <typename R, int N, int K, int M>
hipError_t run(const nqs_ctx* c, const int8_t* spins, int64_t S, const void* t, const void* w,
               double* partial, hipStream_t st) {
  const int64_t items = S * (c->G / 32);
  int64_t blocks = (items + kRegWaves - 1) / kRegWaves;
  blocks = std::min<int64_t>(blocks, c->n_cu > 0 ? c->n_cu : 256);
  eloc_reg_kernel<R, N, K, M><<<(unsigned)blocks, 64 * kRegWaves, 0, st>>>(
      spins, S, c->G, c->n_htiles, c->dev.bonds, c->dev.bmap, (const R*)t, (const R*)w,
      (const R*)c->par.Tpm, (const R*)c->par.F, partial);
  return hipGetLastError();
}


// Two-hop H^2 terms (Sec. 3.3) for single-RBM models with register-resident
// tanh(theta).  For exchanges b1 then b2 with signs s1, s2 (orientation
// folded) and unsigned T1 = tanh D1, T2 = tanh D2:
//   s1 s2 cosh(theta + s1 D1 + s2 D2)/(cosh theta cosh D1 cosh D2) = s2 A + T2 B,
//   A = s1 + t T1,  B = s1 t + T1,
// and (s1 s2)^M = 1, so the second-hop product is prod_h (s2 A_h + T2_h B_h)
// and the first-hop product prod_h A_h.
//
// One wavefront per (sample, first-hop slot, 32-image tile).  The two lanes
// of an image split the hidden units by parity (lane half = lane / 32 takes
// h = 2j + half), both walk every second-hop bond, and the two partial
// products are joined with v_permlane32_swap, which serves the two bonds of a
// pass at once (bond 0 complete in lanes 0..31, bond 1 in lanes 32..63).  The
// +T table stays in LDS for the launch, each row ordered [even h | odd h].
//
// Ratio form: f = s2 A + T2 B = A (s2 + T2 Q) with Q = B / A.  Once per
// (first hop, image) Q replaces t in registers and every second-hop product
// starts from prod A over the lane's units: 8 VALU operations per factor
// instead of about 11.  Used when every suffix product of |A|^2 along the
// lane's units lies in 2^[-120, 120] (binary exponents summed exactly) on all
// lanes of the wave; otherwise t is reloaded and the direct form runs.
__device__ __forceinline__ int ilogb_bits(float v) { return ((__float_as_int(v) >> 23) & 0xff) - 127; }
__device__ __forceinline__ int ilogb_bits(double v) {
  return (int)((__double_as_longlong(v) >> 52) & 0x7ff) - 1023;
}
__device__ __forceinline__ float rcp_fast(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double rcp_fast(double v) { return 1.0 / v; }

// (x of lanes 0..31) * (x of lanes 32..63), in every lane
template <typename R>
__device__ __forceinline__ void join_halves(R& xr, R& xi) {
  R yr = xr, yi = xi;
  swap32(xr, yr);
  swap32(xi, yi);
  const R nr = xr * yr - xi * yi;
  xi = xr * yi + xi * yr;
  xr = nr;
}

template <typename R, int N, int M>
__global__ __launch_bounds__(64 * kRegWaves) void twohop_reg_kernel(
    const int8_t* __restrict__ spins, int64_t S, int G, int n_htiles,
    const int32_t* __restrict__ bonds, const double* __restrict__ bond_J,
    const int32_t* __restrict__ bmap, const R* __restrict__ t, const R* __restrict__ w,
    const R* __restrict__ Tpm, const R* __restrict__ F, double* __restrict__ partial2,
    int allow_ratio) {
  using Cfg = RegCfg<R, N, 1, M>;
  constexpr int NB = Cfg::NB, ST = Cfg::STRIDE, MH = M / 2;
  __shared__ __align__(16) R Tl[NB * ST];
  __shared__ int16_t lists[kRegWaves][2][NB];
  __shared__ int8_t rows[kRegWaves][N];
  for (int idx = threadIdx.x; idx < NB * M; idx += blockDim.x) {
    const int beta = idx / M, h = idx % M;
    const R* src = Tpm + ((size_t)beta * 2 * M + h) * 2;
    const int pos = (h & 1) * MH + (h >> 1);             // [even h | odd h]
    Tl[beta * ST + 2 * pos] = src[0];
    Tl[beta * ST + 2 * pos + 1] = src[1];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int ntiles = G / 32;
  const int64_t n_items = S * NB * ntiles;
  const int64_t stride = (int64_t)gridDim.x * kRegWaves;
  int16_t* l1 = lists[wv][0];
  int16_t* l2 = lists[wv][1];
  int8_t* row2 = rows[wv];
  for (int64_t item = (int64_t)blockIdx.x * kRegWaves + wv; item < n_items; item += stride) {
    const int64_t s = item / ((int64_t)NB * ntiles);
    const int slot = (int)((item / ntiles) % NB);
    const int tile = (int)(item % ntiles);
    const int8_t* srow = spins + s * N;
    const int nc = build_list(srow, bonds, NB, l1, lane);
    if (slot >= nc) continue;                            // wave-uniform
    const int b1 = l1[slot];
    const int i1 = bonds[2 * b1], j1 = bonds[2 * b1 + 1];
    for (int i = lane; i < N; i += 64) row2[i] = srow[i];
    wave_sync_lds();
    if (lane == 0) {
      row2[i1] = srow[j1];
      row2[j1] = srow[i1];
    }
    wave_sync_lds();
    const int nc2 = build_pair_list(row2, bonds, NB, l2, lane, b1, i1, j1);
    double diag2 = 0.0;
    for (int b = lane; b < NB; b += 64)
      diag2 += 0.25 * bond_J[b] * (double)(row2[bonds[2 * b]] * row2[bonds[2 * b + 1]]);
    diag2 = wave_sum(diag2);

    // lane-derived values are recomputed per item rather than hoisted out of
    // the item loop and kept live (or spilled) across it
    int lane_i = lane;
    asm volatile("" : "+v"(lane_i));
    const int half = lane_i >> 5;
    const int g = tile * 32 + (lane_i & 31);
    // this lane's units h = 2j + half: tanh(theta) from the [S][M/8][G][8] layout
    R tr[MH], ti[MH];
    auto load_t = [&](int gg) {
#pragma unroll
      for (int ht = 0; ht < M / 8; ++ht) {
        const R* tp = t + (((size_t)s * n_htiles + ht) * G + gg) * 16;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          tr[4 * ht + e] = tp[2 * (2 * e + half)];
          ti[4 * ht + e] = tp[2 * (2 * e + half) + 1];
        }
      }
    };
    load_t(g);
    const R wr = w[((size_t)s * G + g) * 2], wi = w[((size_t)s * G + g) * 2 + 1];
    const int v1 = bmap[(size_t)g * NB + b1];
    const int beta1 = v1 >> 1;
    const int s1b = -(int)srow[i1];
    const int s1i = (v1 & 1) ? -s1b : s1b;
    const R s1 = (R)s1i;
    const R* T1 = Tl + beta1 * ST + half * M;           // this lane's half of the row
    const R* f1 = F + ((size_t)beta1 * 2 + (s1i > 0 ? 0 : 1)) * 2;
    const R g1r = f1[0] * wr - f1[1] * wi, g1i = f1[0] * wi + f1[1] * wr;   // w F1
    double accr = 0.0, acci = 0.0;

    // ratio form: Q, prod A over the lane's units and the exponent check in one pass
    R par = 1, pai = 0;
    bool ok = allow_ratio != 0;
    {
      int esum = 0, pmax = 0, pmin = 0;              // suffix sums = total - prefix sums
#pragma unroll
      for (int j = 0; j < MH; ++j) {
        if ((j & 3) == 0) __builtin_amdgcn_sched_barrier(0);
        const R Tr = T1[2 * j], Ti = T1[2 * j + 1];
        const R ar = fmaf_t(tr[j], Tr, fmaf_t(-ti[j], Ti, s1));
        const R ai = fmaf_t(tr[j], Ti, ti[j] * Tr);
        const R br = fmaf_t(s1, tr[j], Tr), bi = fmaf_t(s1, ti[j], Ti);
        const R a2 = ar * ar + ai * ai;
        ok &= (a2 > R(0)) & (a2 < R(INFINITY));       // no short-circuit branches
        pmax = max(pmax, esum);
        pmin = min(pmin, esum);
        esum += ilogb_bits(a2);
        const R inv = rcp_fast(a2);
        tr[j] = (br * ar + bi * ai) * inv;           // Q = B conj(A) / |A|^2
        ti[j] = (bi * ar - br * ai) * inv;
        const R nr = fmaf_t(par, ar, -(pai * ai));
        pai = fmaf_t(par, ai, pai * ar);
        par = nr;
      }
      ok &= (esum - pmin <= 120) & (esum - pmax >= -120);
    }
    // Q is used only on the ratio branch: pin it here so that the compiler
    // does not sink its computation into the branch and keep A, B live
#pragma unroll
    for (int j = 0; j < MH; ++j) asm volatile("" : "+v"(tr[j]), "+v"(ti[j]));
    const bool ratio = __all(ok);
    if (!ratio) {
      int g2 = g;                                // fresh addresses for the reload
      asm volatile("" : "+v"(g2));
      load_t(g2);
    }
    {
      // first-hop product over all units (both halves)
      R pr = par, pi = pai;
      if (!ratio) {
        pr = 1;
        pi = 0;
#pragma unroll
        for (int j = 0; j < MH; ++j) {
          const R Tr = T1[2 * j], Ti = T1[2 * j + 1];
          const R a = fmaf_t(tr[j], Tr, fmaf_t(-ti[j], Ti, s1));
          const R b = fmaf_t(tr[j], Ti, ti[j] * Tr);
          const R nr = fmaf_t(pr, a, -(pi * b));
          pi = fmaf_t(pr, b, pi * a);
          pr = nr;
        }
      }
      join_halves(pr, pi);
      if (half == 0) {
        accr += diag2 * (double)(g1r * pr - g1i * pi);
        acci += diag2 * (double)(g1r * pi + g1i * pr);
        // b1 exchanged back: s^{b1 b1} = s, ratio 1 in every image
        const double jj = 0.25 * bond_J[b1] * bond_J[b1];
        accr += jj * (double)wr;
        acci += jj * (double)wi;
      }
    }
    for (int i0 = 0; i0 < nc2; i0 += 2) {
      int beta[2], sidx[2];
      R sgn[2];
      double mult[2];
#pragma unroll
      for (int n = 0; n < 2; ++n) {
        const int ii = i0 + n;
        const int e = l2[ii < nc2 ? ii : i0];
        const int b = e & kPairBond;
        mult[n] = (e & kPairTwice) ? 2.0 : 1.0;
        const int v = bmap[(size_t)g * NB + b];
        beta[n] = v >> 1;
        const int s_b = -(int)row2[bonds[2 * b]];
        const int sp = (v & 1) ? -s_b : s_b;
        sgn[n] = (R)sp;
        sidx[n] = sp > 0 ? 0 : 1;
      }
      const R* U0 = Tl + beta[0] * ST + half * M;
      const R* U1 = Tl + beta[1] * ST + half * M;
      R p0r, p0i, p1r, p1i;
      if (ratio) {
        p0r = p1r = par;
        p0i = p1i = pai;
#pragma unroll
        for (int j = 0; j < MH; ++j) {
          if ((j & 3) == 0) __builtin_amdgcn_sched_barrier(0);
          const R Qr = tr[j], Qi = ti[j];
          {
            const R Vr = U0[2 * j], Vi = U0[2 * j + 1];
            const R fr = fmaf_t(Vr, Qr, fmaf_t(-Vi, Qi, sgn[0]));
            const R fi = fmaf_t(Vr, Qi, Vi * Qr);
            const R nr = fmaf_t(p0r, fr, -(p0i * fi));
            p0i = fmaf_t(p0r, fi, p0i * fr);
            p0r = nr;
          }
          {
            const R Vr = U1[2 * j], Vi = U1[2 * j + 1];
            const R fr = fmaf_t(Vr, Qr, fmaf_t(-Vi, Qi, sgn[1]));
            const R fi = fmaf_t(Vr, Qi, Vi * Qr);
            const R nr = fmaf_t(p1r, fr, -(p1i * fi));
            p1i = fmaf_t(p1r, fi, p1i * fr);
            p1r = nr;
          }
        }
      } else {
        p0r = p1r = 1;
        p0i = p1i = 0;
#pragma unroll
        for (int j = 0; j < MH; ++j) {
          if ((j & 3) == 0) __builtin_amdgcn_sched_barrier(0);
          const R Tr = T1[2 * j], Ti = T1[2 * j + 1];
          const R Ar = fmaf_t(tr[j], Tr, fmaf_t(-ti[j], Ti, s1));
          const R Ai = fmaf_t(tr[j], Ti, ti[j] * Tr);
          const R Br = fmaf_t(s1, tr[j], Tr), Bi = fmaf_t(s1, ti[j], Ti);
          {
            const R Vr = U0[2 * j], Vi = U0[2 * j + 1];
            const R fr = fmaf_t(Vr, Br, fmaf_t(-Vi, Bi, sgn[0] * Ar));
            const R fi = fmaf_t(Vr, Bi, fmaf_t(Vi, Br, sgn[0] * Ai));
            const R nr = fmaf_t(p0r, fr, -(p0i * fi));
            p0i = fmaf_t(p0r, fi, p0i * fr);
            p0r = nr;
          }
          {
            const R Vr = U1[2 * j], Vi = U1[2 * j + 1];
            const R fr = fmaf_t(Vr, Br, fmaf_t(-Vi, Bi, sgn[1] * Ar));
            const R fi = fmaf_t(Vr, Bi, fmaf_t(Vi, Br, sgn[1] * Ai));
            const R nr = fmaf_t(p1r, fr, -(p1i * fi));
            p1i = fmaf_t(p1r, fi, p1i * fr);
            p1r = nr;
          }
        }
      }
      // join the halves: lanes 0..31 get bond 0's product, lanes 32..63 bond 1's
      swap32(p0r, p1r);
      swap32(p0i, p1i);
      const R pr = p0r * p1r - p0i * p1i, pi = p0r * p1i + p0i * p1r;
      const bool valid = i0 + half < nc2;
      const R* f2 = F + ((size_t)beta[half] * 2 + sidx[half]) * 2;
      const R hr = f2[0] * g1r - f2[1] * g1i, hi = f2[0] * g1i + f2[1] * g1r;
      accr += valid ? mult[half] * (double)(hr * pr - hi * pi) : 0.0;
      acci += valid ? mult[half] * (double)(hr * pi + hi * pr) : 0.0;
    }
    accr = wave_sum(accr);
    acci = wave_sum(acci);
    if (lane == 0) {
      const size_t o = ((size_t)s * NB + slot) * ntiles + tile;
      partial2[2 * o] = accr;
      partial2[2 * o + 1] = acci;
    }
    wave_sync_lds();
  }
}

template <typename R, int N, int M>
hipError_t run_twohop(const nqs_ctx* c, const int8_t* spins, int64_t S, const void* t,
                      const void* w, double* partial2, hipStream_t st) {
  const int64_t items = S * c->NB * (c->G / 32);
  int64_t blocks = (items + kRegWaves - 1) / kRegWaves;
  blocks = std::min<int64_t>(blocks, c->n_cu > 0 ? c->n_cu : 256);
  twohop_reg_kernel<R, N, M><<<(unsigned)blocks, 64 * kRegWaves, 0, st>>>(
      spins, S, c->G, c->n_htiles, c->dev.bonds, c->dev.bond_J, c->dev.bmap, (const R*)t,
      (const R*)w, (const R*)c->par.Tpm, (const R*)c->par.F, partial2, c->direct_only ? 0 : 1);
  return hipGetLastError();
}

}  // namespace

// Returns hipErrorNotSupported when no register-resident variant covers the model.
hipError_t launch_eloc_bonds_reg(const nqs_ctx* c, const int8_t* spins, int64_t S, const void* t,
                                 const void* w, double* partial, hipStream_t st) {
  const int N = c->N, K = c->K, M = c->M;
  if (c->prec == NQS_FP64) {
    if (N == 16 && K == 1 && M == 16) return run<double, 16, 1, 16>(c, spins, S, t, w, partial, st);
    if (N == 16 && K == 2 && M == 8) return run<double, 16, 2, 8>(c, spins, S, t, w, partial, st);
  } else {
    if (N == 16 && K == 1 && M == 16) return run<float, 16, 1, 16>(c, spins, S, t, w, partial, st);
    if (N == 36 && K == 1 && M == 72) return run<float, 36, 1, 72>(c, spins, S, t, w, partial, st);
    if (N == 36 && K == 2 && M == 16) return run<float, 36, 2, 16>(c, spins, S, t, w, partial, st);
  }
  return hipErrorNotSupported;
}

bool twohop_reg_supported(const nqs_ctx* c) {
  if (c->K != 1) return false;
  if (c->prec == NQS_FP64) return c->N == 16 && c->M == 16;
  return (c->N == 16 && c->M == 16) || (c->N == 36 && c->M == 72);
}

hipError_t launch_twohop_reg(const nqs_ctx* c, const int8_t* spins, int64_t S, const void* t,
                             const void* w, double* partial2, hipStream_t st) {
  if (!twohop_reg_supported(c)) return hipErrorNotSupported;
  if (c->prec == NQS_FP64) {
    if (c->N == 16 && c->M == 16) return run_twohop<double, 16, 16>(c, spins, S, t, w, partial2, st);
  } else {
    if (c->N == 16 && c->M == 16) return run_twohop<float, 16, 16>(c, spins, S, t, w, partial2, st);
    if (c->N == 36 && c->M == 72) return run_twohop<float, 36, 72>(c, spins, S, t, w, partial2, st);
  }
  return hipErrorNotSupported;
}

}  // namespace nqs
