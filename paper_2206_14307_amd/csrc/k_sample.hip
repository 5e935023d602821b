// Exchange Metropolis sampling of |psi|^2 (Sec. 3.2; N_skip rule of Sec. 3.4).
//
// One workgroup per chain, one lane per symmetry image.  The chain keeps, in
// the caller's workspace, tanh(theta) of every (image, hidden unit) and the
// normalised image weights u_kg = chi_g psi_s^(k)(g sigma)/psi(sigma), in the
// layouts the theta and log-sum-exp kernels write (those kernels build the
// cache and refresh it between launches, which bounds rounding drift).
//
// A proposal exchanges the up site i and the down site j.  In image g they
// sit at p = perm_g^-1(i), q = perm_g^-1(j), so theta -> theta - (W_p - W_q)
// and, with T = tanh(W_p - W_q) (the precomputed site-pair table),
//   psi_s(g sigma')/psi_s(g sigma) = exp(-(a_p - a_q)) prod_h cosh(W_hp - W_hq)
//                                    * prod_h (t_h T_h - 1)        (M even),
// the ratio is psi(sigma')/psi(sigma) = sum_kg u_kg R_kg, and an accepted
// move updates t' = (t - T)/(1 - t T) (tanh addition) and u' = u R / ratio.
//
// Randomness: proposal n of a chain uses Philox4x64-10 (Salmon et al., SC'11)
// with counter (n, 0, 0, 0) and key (seed, chain id): r0 picks the
// k-th up site, k = (r0 >> 11) * (N/2) >> 53, r1 the k'-th down site, and the
// move is accepted iff (r2 >> 11) * 2^-53 < |ratio|^2.
#include <algorithm>
#include <string>

#include "device_common.h"
#include "nqs_internal.h"

namespace nqs {

namespace {

constexpr int kSegment = 256;      // proposals per launch between cache refreshes
constexpr int kNskipMax = 1000;

__device__ __forceinline__ void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                              uint64_t k0, uint64_t k1, uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// reciprocal for the cache update (hardware rcp, ~1 ulp; the cache is rebuilt
// from the spins every segment)
__device__ __forceinline__ float rcp_fast(float v) { return __builtin_amdgcn_rcpf(v); }

// reciprocal of the squared modulus in the cache update: hardware rcp in
// FP32 (the cache is rebuilt from the spins every segment), a division in
// FP64
__device__ __forceinline__ float recip_t(float v) { return rcp_fast(v); }
__device__ __forceinline__ double recip_t(double v) { return 1.0 / v; }

// one cache or row tile of 8 complex values, moved in 16-byte pieces (the
// tiles are 64-byte aligned)
template <typename R>
__device__ __forceinline__ void load_tile(R (&d)[16], const R* p) {
  constexpr int NV = (int)(16 * sizeof(R) / sizeof(uint4));
  const uint4* q = reinterpret_cast<const uint4*>(p);
  uint4 v[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = q[i];
  __builtin_memcpy(d, v, sizeof(v));
}
template <typename R>
__device__ __forceinline__ void store_tile(R* p, const R (&d)[16]) {
  constexpr int NV = (int)(16 * sizeof(R) / sizeof(uint4));
  uint4 v[NV];
  __builtin_memcpy(v, d, sizeof(v));
  uint4* q = reinterpret_cast<uint4*>(p);
#pragma unroll
  for (int i = 0; i < NV; ++i) q[i] = v[i];
}

// position of the k-th (0-based) set bit of a 64-bit word (k < popcount)
__device__ __forceinline__ int select64(uint64_t x, int k) {
  int pos = 0;
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) {
    const uint64_t low = x & ((1ull << w) - 1ull);
    const int c = __popcll(low);
    if (k >= c) {
      k -= c;
      x >>= w;
      pos += w;
    }
  }
  return pos;
}

__device__ __forceinline__ int select128(uint64_t lo, uint64_t hi, int k) {
  const int c = __popcll(lo);
  return k < c ? select64(lo, k) : 64 + select64(hi, k - c);
}

template <typename R>
__global__ __launch_bounds__(1024) void sample_kernel(
    int N, int G, int K, int M, int n_htiles, const uint8_t* __restrict__ perminv,
    const R* __restrict__ Tpair, const R* __restrict__ Fpair, R* __restrict__ t, R* __restrict__ t2,
    R* __restrict__ w, uint64_t* __restrict__ state, int n_prop, int phase, int64_t p0,
    const int32_t* nskip_dev,
    int n_skip_host, uint64_t seed, int8_t* __restrict__ spins_out, int64_t n_per_chain,
    int64_t* __restrict__ acc_out, int8_t* __restrict__ cur_spins) {
  extern __shared__ __align__(16) unsigned char smem[];
  R* Rg = reinterpret_cast<R*>(smem);                                  // [G][K] complex
  // per-wave ratio sums [2][32], double-buffered by proposal parity (see the
  // register kernel): one barrier per proposal
  double* red = reinterpret_cast<double*>(smem + (size_t)G * K * 2 * sizeof(R));
  const int64_t c = blockIdx.x;
  const int g = threadIdx.x, lane = g & 63, wv = g >> 6, nw = (blockDim.x + 63) >> 6;
  const bool active = g < G;
  uint64_t lo = state[4 * c], hi = state[4 * c + 1], ctr = state[4 * c + 2];
  const uint64_t id = state[4 * c + 3];
  const uint64_t nmask_lo = N >= 64 ? ~0ull : ((1ull << N) - 1ull);
  const uint64_t nmask_hi = N > 64 ? ((1ull << (N - 64)) - 1ull) : 0ull;
  const int half = N / 2;
  const bool valid = (__popcll(lo & nmask_lo) + __popcll(hi & nmask_hi) == half) &&
                     ((lo & ~nmask_lo) == 0) && ((hi & ~nmask_hi) == 0);
  const int n_skip = phase == 1 ? (nskip_dev ? *nskip_dev : n_skip_host) : 1;
  const int KM = K * M;
  // tanh(theta) of the current state (tc) and of the proposed one (tn): the
  // ratio pass also writes the tanh-addition update of every entry to tn, and
  // an accepted proposal swaps the two (the acceptance rate is close to 1, so
  // this reads the cache once per proposal instead of twice)
  R* tc = t + (size_t)c * n_htiles * G * 16;
  R* tn = t2 + (size_t)c * n_htiles * G * 16;
  R* wc = w + (size_t)c * K * G * 2;
  int64_t acc = 0;
  for (int r = 0; r < n_prop && valid; ++r) {
    uint64_t rnd[4];
    philox4x64_10(ctr, 0, 0, 0, seed, id, rnd);
    const int kup = (int)(((rnd[0] >> 11) * (uint64_t)half) >> 53);
    const int kdn = (int)(((rnd[1] >> 11) * (uint64_t)half) >> 53);
    const int i = select128(lo, hi, kup);
    const int j = select128(~lo & nmask_lo, ~hi & nmask_hi, kdn);
    double cr = 0.0, ci = 0.0;
    int l1 = 0, l2 = 0;
    if (active) {
      l1 = perminv[(size_t)g * N + i];
      l2 = perminv[(size_t)g * N + j];
      const R* Trow = Tpair + ((size_t)l1 * N + l2) * KM * 2;
      for (int k = 0; k < K; ++k) {
        R pr = 1, pi = 0;
        // tiles of 8 units: this image's 16 cache values (one contiguous
        // piece of the [tile][G][16] layout) and 16 row values, each tile's
        // loads issued one tile ahead of its use, its updates stored whole
        const int nt = M / 8;
        const R* tp = tc + ((size_t)(k * nt) * G + g) * 16;
        R* up = tn + ((size_t)(k * nt) * G + g) * 16;
        const R* Tq = Trow + (size_t)2 * k * M;
        // the 8 factors of a tile into the product, the updated tile stored
        auto tile = [&](R (&tt)[16], const R (&TT)[16], R* dst) {
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const R tr = tt[2 * e], ti = tt[2 * e + 1];
            const R Tr = TT[2 * e], Ti = TT[2 * e + 1];
            const R a = fmaf_t(tr, Tr, fmaf_t(-ti, Ti, R(-1)));   // a + ib = t T - 1
            const R b = fmaf_t(tr, Ti, ti * Tr);
            const R nr = fmaf_t(pr, a, -(pi * b));
            pi = fmaf_t(pr, b, pi * a);
            pr = nr;
            // t' = (t - T) / (1 - t T) = (T - t) / (a + ib)
            const R dr = Tr - tr, di = Ti - ti;
            const R inv = recip_t(fmaf_t(a, a, b * b));
            tt[2 * e] = (dr * a + di * b) * inv;
            tt[2 * e + 1] = (di * a - dr * b) * inv;
          }
          store_tile(dst, tt);
        };
        // FP32: two register buffers, the next tile always in flight (FP64,
        // for small lattices only, keeps one: its tiles would not fit twice
        // in the 128 VGPRs of a 1024-lane workgroup)
        R t0[16], T0[16], t1[16], T1[16];
        if constexpr (sizeof(R) == 8) {
          for (int ht = 0; ht < nt; ++ht) {
            load_tile(t0, tp + (size_t)ht * G * 16);
            load_tile(T0, Tq + 16 * ht);
            tile(t0, T0, up + (size_t)ht * G * 16);
          }
        } else {
          // the loop body is free of conditions (the last prefetch reads the
          // last tile again): a conditional load is sunk to its use, and a
          // conditional path makes the wait before a tile cover the next
          // one's loads too
          load_tile(t0, tp);
          load_tile(T0, Tq);
          int ht = 0;
          for (; ht + 1 < nt; ht += 2) {
            load_tile(t1, tp + (size_t)(ht + 1) * G * 16);
            load_tile(T1, Tq + 16 * (ht + 1));
            tile(t0, T0, up + (size_t)ht * G * 16);
            const int h2 = min(ht + 2, nt - 1);
            load_tile(t0, tp + (size_t)h2 * G * 16);
            load_tile(T0, Tq + 16 * h2);
            tile(t1, T1, up + (size_t)(ht + 1) * G * 16);
          }
          if (ht < nt) tile(t0, T0, up + (size_t)ht * G * 16);   // odd tile count
        }
        const R* f = Fpair + (((size_t)k * N + l1) * N + l2) * 2;
        const R rr = f[0] * pr - f[1] * pi, ri = f[0] * pi + f[1] * pr;
        Rg[2 * (g * K + k)] = rr;
        Rg[2 * (g * K + k) + 1] = ri;
        const R wr = wc[2 * (k * G + g)], wi = wc[2 * (k * G + g) + 1];
        cr += (double)(wr * rr - wi * ri);
        ci += (double)(wr * ri + wi * rr);
      }
    }
    cr = wave_sum(cr);
    ci = wave_sum(ci);
    double* rb = red + 32 * (r & 1);
    if (lane == 0) {
      rb[wv] = cr;
      rb[16 + wv] = ci;
    }
    __syncthreads();
    double sr = 0.0, si = 0.0;
    for (int q = 0; q < nw; ++q) {
      sr += rb[q];
      si += rb[16 + q];
    }
    const double u = (double)(rnd[2] >> 11) * (1.0 / 9007199254740992.0);
    const bool accept = u < sr * sr + si * si;
    if (accept) {
      ++acc;
      R* const sw = tc;                        // the updated cache becomes current
      tc = tn;
      tn = sw;
      if (active) {
        const double den = sr * sr + si * si;
        for (int k = 0; k < K; ++k) {
          const R wr = wc[2 * (k * G + g)], wi = wc[2 * (k * G + g) + 1];
          const R rr = Rg[2 * (g * K + k)], ri = Rg[2 * (g * K + k) + 1];
          const double qr = (double)(wr * rr - wi * ri), qi = (double)(wr * ri + wi * rr);
          wc[2 * (k * G + g)] = (R)((qr * sr + qi * si) / den);
          wc[2 * (k * G + g) + 1] = (R)((qi * sr - qr * si) / den);
        }
      }
      const int b0 = i < 64 ? i : i - 64, b1 = j < 64 ? j : j - 64;
      if (i < 64) lo ^= 1ull << b0; else hi ^= 1ull << b0;
      if (j < 64) lo ^= 1ull << b1; else hi ^= 1ull << b1;
    }
    ++ctr;
    if (phase == 1) {
      const int64_t idx = p0 + r + 1;
      if (idx % n_skip == 0) {
        const int64_t m = idx / n_skip - 1;
        if (m < n_per_chain && g < N) {
          const uint64_t bit = g < 64 ? (lo >> g) & 1ull : (hi >> (g - 64)) & 1ull;
          spins_out[((size_t)c * n_per_chain + m) * N + g] = bit ? 1 : -1;
        }
      }
    }
  }
  if (g == 0) {
    state[4 * c] = lo;
    state[4 * c + 1] = hi;
    state[4 * c + 2] = ctr;
    acc_out[c] += valid ? acc : -((int64_t)1 << 40);   // marks a chain outside Sz = 0
  }
  if (g < N) {
    const uint64_t bit = g < 64 ? (lo >> g) & 1ull : (hi >> (g - 64)) & 1ull;
    cur_spins[(size_t)c * N + g] = bit ? 1 : -1;
  }
}

// Register-resident variant for one RBM with M <= 72 and G <= 512: each image
// is held by SPLIT lanes (lanes l and l + 32 of a wavefront for SPLIT = 2),
// each keeping its share of the image's tanh(theta) row in VGPRs for the whole
// segment (loaded once from the refreshed cache), so a proposal reads only the
// L2-resident site-pair rows.  The cache in HBM is not written back: the next
// segment starts from a fresh refresh.
template <typename R, int M, int SPLIT>
__global__ __launch_bounds__(640) void sample_reg_kernel(
    int N, int G, int n_htiles, const uint8_t* __restrict__ perminv,
    const R* __restrict__ Tpair, const R* __restrict__ Fpair, const R* __restrict__ t,
    const R* __restrict__ w, uint64_t* __restrict__ state, int n_prop, int phase, int64_t p0,
    int n_skip_host, uint64_t seed, int8_t* __restrict__ spins_out, int64_t n_per_chain,
    int64_t* __restrict__ acc_out, int8_t* __restrict__ cur_spins) {
  constexpr int MH = M / SPLIT;                  // hidden units per lane
  // per-wave ratio sums, double-buffered by proposal parity: proposal r + 2
  // writes a buffer only after every wave passed proposal r + 1's barrier,
  // i.e. after every wave read proposal r's sums
  __shared__ double red[2][32];
  extern __shared__ uint8_t pinv[];              // [G][N] inverse permutations (G N bytes)
  __shared__ uint64_t rbuf[64][3];               // random words of the next 64 proposals
  const int64_t c = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = (blockDim.x + 63) >> 6;
  const int g = SPLIT == 2 ? 32 * wv + (lane & 31) : tid;
  const int part = SPLIT == 2 ? lane >> 5 : 0;
  const bool active = g < G;
  const bool lead = active && part == 0;
  uint64_t lo = state[4 * c], hi = state[4 * c + 1], ctr = state[4 * c + 2];
  const uint64_t id = state[4 * c + 3];
  const uint64_t nmask_lo = N >= 64 ? ~0ull : ((1ull << N) - 1ull);
  const uint64_t nmask_hi = N > 64 ? ((1ull << (N - 64)) - 1ull) : 0ull;
  const int half = N / 2;
  const bool valid = (__popcll(lo & nmask_lo) + __popcll(hi & nmask_hi) == half) &&
                     ((lo & ~nmask_lo) == 0) && ((hi & ~nmask_hi) == 0);
  const int n_skip = phase == 1 ? n_skip_host : 1;
  const int gg = active ? g : 0;
  const int h0 = part * MH;
  R tr[MH], ti[MH];
  R wr, wi;
  {
    const R* tc = t + (size_t)c * n_htiles * G * 16;
#pragma unroll
    for (int e = 0; e < MH; ++e) {
      const int h = h0 + e;
      tr[e] = tc[((size_t)(h >> 3) * G + gg) * 16 + 2 * (h & 7)];
      ti[e] = tc[((size_t)(h >> 3) * G + gg) * 16 + 2 * (h & 7) + 1];
    }
    const R* wc = w + (size_t)c * G * 2;
    wr = wc[2 * gg];
    wi = wc[2 * gg + 1];
  }
  // the table lookups of every proposal read LDS instead of L2
  for (int e = tid; e < G * N; e += blockDim.x) pinv[e] = perminv[e];
  __syncthreads();
  int64_t acc = 0;
  for (int r = 0; r < n_prop && valid; ++r) {
    // Philox depends only on the proposal index: one wavefront draws the words
    // of 64 proposals at once (counters ctr .. ctr + 63), every wave reads them
    if ((r & 63) == 0) {
      __syncthreads();
      if (tid < 64) {
        uint64_t rr[4];
        philox4x64_10(ctr + (uint64_t)tid, 0, 0, 0, seed, id, rr);
        rbuf[tid][0] = rr[0];
        rbuf[tid][1] = rr[1];
        rbuf[tid][2] = rr[2];
      }
      __syncthreads();
    }
    const uint64_t rnd[3] = {rbuf[r & 63][0], rbuf[r & 63][1], rbuf[r & 63][2]};
    const int kup = (int)(((rnd[0] >> 11) * (uint64_t)half) >> 53);
    const int kdn = (int)(((rnd[1] >> 11) * (uint64_t)half) >> 53);
    const int i = select128(lo, hi, kup);
    const int j = select128(~lo & nmask_lo, ~hi & nmask_hi, kdn);
    const int l1 = pinv[gg * N + i], l2 = pinv[gg * N + j];
    const R* Trow = Tpair + (((size_t)l1 * N + l2) * M + h0) * 2;
    R pr = 1, pi = 0, qr = 1, qi = 0;
#pragma unroll
    for (int e = 0; e < MH; e += 2) {
      R Tr = Trow[2 * e], Ti = Trow[2 * e + 1];
      R a = fmaf_t(tr[e], Tr, fmaf_t(-ti[e], Ti, R(-1)));
      R b = fmaf_t(tr[e], Ti, ti[e] * Tr);
      R nr = fmaf_t(pr, a, -(pi * b));
      pi = fmaf_t(pr, b, pi * a);
      pr = nr;
      Tr = Trow[2 * e + 2];
      Ti = Trow[2 * e + 3];
      a = fmaf_t(tr[e + 1], Tr, fmaf_t(-ti[e + 1], Ti, R(-1)));
      b = fmaf_t(tr[e + 1], Ti, ti[e + 1] * Tr);
      nr = fmaf_t(qr, a, -(qi * b));
      qi = fmaf_t(qr, b, qi * a);
      qr = nr;
    }
    R ppr = pr * qr - pi * qi, ppi = pr * qi + pi * qr;
    if (SPLIT == 2) {
      const R orr = __shfl_xor(ppr, 32, 64), oi = __shfl_xor(ppi, 32, 64);
      const R nr = ppr * orr - ppi * oi;
      ppi = ppr * oi + ppi * orr;
      ppr = nr;
    }
    const R* f = Fpair + ((size_t)l1 * N + l2) * 2;
    const R Rr = f[0] * ppr - f[1] * ppi, Ri = f[0] * ppi + f[1] * ppr;
    double cr = 0.0, ci = 0.0;
    if (lead) {
      cr = (double)(wr * Rr - wi * Ri);
      ci = (double)(wr * Ri + wi * Rr);
    }
    cr = wave_sum(cr);
    ci = wave_sum(ci);
    double* rb = red[r & 1];
    if (lane == 0) {
      rb[wv] = cr;
      rb[16 + wv] = ci;
    }
    __syncthreads();
    double sr = 0.0, si = 0.0;
    for (int q = 0; q < nw; ++q) {
      sr += rb[q];
      si += rb[16 + q];
    }
    const double u = (double)(rnd[2] >> 11) * (1.0 / 9007199254740992.0);
    const double den = sr * sr + si * si;
    if (u < den) {
      ++acc;
#pragma unroll
      for (int e = 0; e < MH; ++e) {
        const R Tr = Trow[2 * e], Ti = Trow[2 * e + 1];
        const R nr = tr[e] - Tr, ni = ti[e] - Ti;        // (t - T) / (1 - t T)
        const R dr = R(1) - (tr[e] * Tr - ti[e] * Ti), di = -(tr[e] * Ti + ti[e] * Tr);
        const R inv = rcp_fast(dr * dr + di * di);
        tr[e] = (nr * dr + ni * di) * inv;
        ti[e] = (ni * dr - nr * di) * inv;
      }
      const double qr2 = (double)(wr * Rr - wi * Ri), qi2 = (double)(wr * Ri + wi * Rr);
      wr = (R)((qr2 * sr + qi2 * si) / den);
      wi = (R)((qi2 * sr - qr2 * si) / den);
      if (i < 64) lo ^= 1ull << i; else hi ^= 1ull << (i - 64);
      if (j < 64) lo ^= 1ull << j; else hi ^= 1ull << (j - 64);
    }
    ++ctr;
    if (phase == 1) {
      const int64_t idx = p0 + r + 1;
      if (idx % n_skip == 0) {
        const int64_t m = idx / n_skip - 1;
        if (m < n_per_chain && tid < N) {
          const uint64_t bit = tid < 64 ? (lo >> tid) & 1ull : (hi >> (tid - 64)) & 1ull;
          spins_out[((size_t)c * n_per_chain + m) * N + tid] = bit ? 1 : -1;
        }
      }
    }
  }
  if (tid == 0) {
    state[4 * c] = lo;
    state[4 * c + 1] = hi;
    state[4 * c + 2] = ctr;
    acc_out[c] += valid ? acc : -((int64_t)1 << 40);
  }
  if (tid < N) {
    const uint64_t bit = tid < 64 ? (lo >> tid) & 1ull : (hi >> (tid - 64)) & 1ull;
    cur_spins[(size_t)c * N + tid] = bit ? 1 : -1;
  }
}

// DPP lane exchanges within a 16-lane row (every lane active): quad_perm
// (1,0,3,2) pairs lane ^ 1, quad_perm (2,3,0,1) lane ^ 2, row_half_mirror the
// other quad of an 8-lane half row, row_mirror the other half of the row.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

// (bound_ctrl set: no lane reads out of its row in these patterns, and no
// old value has to be copied into the destination first)
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int2 b = __builtin_bit_cast(int2, v);
  int2 r;
  r.x = __builtin_amdgcn_mov_dpp(b.x, CTRL, 0xF, 0xF, true);
  r.y = __builtin_amdgcn_mov_dpp(b.y, CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, r);
}
// Sum over the 64 lanes of a wave (all active), the same value in every lane:
// butterfly within each row, then the four row sums read as scalars.
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_f64<kDppXor1>(v);
  v += dpp_f64<kDppXor2>(v);
  v += dpp_f64<kDppHalfMirror>(v);
  v += dpp_f64<kDppMirror>(v);
  const int2 b = __builtin_bit_cast(int2, v);
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    int2 q;
    q.x = __builtin_amdgcn_readlane(b.x, 16 * r);
    q.y = __builtin_amdgcn_readlane(b.y, 16 * r);
    s += __builtin_bit_cast(double, q);
  }
  return s;
}
// Complex product over groups of LPE consecutive lanes (LPE in {1, 2, 4, 8,
// 16}); every lane of a group ends with the group's product (up to the last
// bit of the imaginary part, whose rounding depends on the operand order).
template <int LPE>
__device__ __forceinline__ void group_cmul(float& pr, float& pi) {
  auto step = [&](float orr, float oi) {
    const float nr = fmaf_t(pr, orr, -(pi * oi));
    pi = fmaf_t(pr, oi, pi * orr);
    pr = nr;
  };
  if constexpr (LPE >= 2) step(dpp_f32<kDppXor1>(pr), dpp_f32<kDppXor1>(pi));
  if constexpr (LPE >= 4) step(dpp_f32<kDppXor2>(pr), dpp_f32<kDppXor2>(pi));
  if constexpr (LPE >= 8) step(dpp_f32<kDppHalfMirror>(pr), dpp_f32<kDppHalfMirror>(pi));
  if constexpr (LPE >= 16) step(dpp_f32<kDppMirror>(pr), dpp_f32<kDppMirror>(pi));
}

// tanh addition t' = (t - T) / (1 - t T), in place
__device__ __forceinline__ void tanh_add(float& tr, float& ti, float Tr, float Ti) {
  const float nr = tr - Tr, ni = ti - Ti;
  const float dr = fmaf_t(ti, Ti, fmaf_t(-tr, Tr, 1.f));
  const float di = fmaf_t(tr, Ti, ti * Tr);             // 1 - t T = dr - i di
  const float inv = rcp_fast(fmaf_t(dr, dr, di * di));
  tr = fmaf_t(nr, dr, -(ni * di)) * inv;
  ti = fmaf_t(ni, dr, nr * di) * inv;
}
// p *= t T - 1
__device__ __forceinline__ void mul_factor(float& pr, float& pi, float tr, float ti, float Tr,
                                           float Ti) {
  const float a = fmaf_t(tr, Tr, fmaf_t(-ti, Ti, -1.f));
  const float b = fmaf_t(tr, Ti, ti * Tr);
  const float nr = fmaf_t(pr, a, -(pi * b));
  pi = fmaf_t(pr, b, pi * a);
  pr = nr;
}

// Register-resident variant for one FP32 RBM whose G = 32 IPG images and M =
// 16 P + 8 R (R = 0 or 1) hidden units give every lane of a 256-lane
// workgroup (one wave per SIMD) IPG x UPL units, UPL = M / 8: lane (group
// gi = l / 8, k = l % 8) holds units 16 p + 2 k, 16 p + 2 k + 1 (p < P) and,
// if R = 1, 16 P + k, of images g = 32 m + gi (m < IPG).  The eight lanes of
// a group thus read each site-pair row in contiguous 128-byte pieces of
// 16-byte loads (and one 64-byte piece of 8-byte loads): a row read per lane
// would make every lane of a load its own cache access, and narrower loads
// cost the L1 address path the same per lane for half the bytes.  The group
// combines its partial products; lane k owns images m = k (mod 8), their
// weights u and ratios.  At most 256 VGPRs a lane leave room for two chains
// per compute unit.
template <int M, int IPG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void
sample_reg8_kernel(int N, int G, int n_htiles, const uint8_t* __restrict__ perminv,
                   const float* __restrict__ Tpair, const float* __restrict__ Fpair,
                   const float* __restrict__ t, const float* __restrict__ w,
                   uint64_t* __restrict__ state, int n_prop, int phase, int64_t p0,
                   int n_skip_host, uint64_t seed, int8_t* __restrict__ spins_out,
                   int64_t n_per_chain, int64_t* __restrict__ acc_out,
                   int8_t* __restrict__ cur_spins) {
  static_assert(M % 8 == 0, "eight lanes per image");
  constexpr int P = M / 16, R = (M % 16) / 8, UPL = M / 8, NSLOT = (IPG + 7) / 8;
  // per-wave ratio sums (re 0..3, im 4..7), double-buffered by proposal parity
  __shared__ double red[2][8];
  extern __shared__ uint8_t pinv[];              // [G][N] inverse permutations
  __shared__ uint64_t rbuf[64][3];               // random words of the next 64 proposals
  const int64_t c = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int gi = tid >> 3, k = tid & 7;
  uint64_t lo = state[4 * c], hi = state[4 * c + 1], ctr = state[4 * c + 2];
  const uint64_t id = state[4 * c + 3];
  const uint64_t nmask_lo = N >= 64 ? ~0ull : ((1ull << N) - 1ull);
  const uint64_t nmask_hi = N > 64 ? ((1ull << (N - 64)) - 1ull) : 0ull;
  const int half = N / 2;
  const bool valid = (__popcll(lo & nmask_lo) + __popcll(hi & nmask_hi) == half) &&
                     ((lo & ~nmask_lo) == 0) && ((hi & ~nmask_hi) == 0);
  const int n_skip = phase == 1 ? n_skip_host : 1;
  float tr[IPG][UPL], ti[IPG][UPL];
  float wr[NSLOT], wi[NSLOT];
  {
    const float* tc = t + (size_t)c * n_htiles * G * 16;
#pragma unroll
    for (int m = 0; m < IPG; ++m)
#pragma unroll
      for (int u = 0; u < UPL; ++u) {
        const int h = u < 2 * P ? 16 * (u >> 1) + 2 * k + (u & 1) : 16 * P + k;
        const size_t o = ((size_t)(h >> 3) * G + 32 * m + gi) * 16 + 2 * (h & 7);
        tr[m][u] = tc[o];
        ti[m][u] = tc[o + 1];
      }
    const float* wc = w + (size_t)c * G * 2;
#pragma unroll
    for (int q = 0; q < NSLOT; ++q) {
      const int m = k + 8 * q < IPG ? k + 8 * q : k;   // lanes without a second image
      wr[q] = wc[2 * (32 * m + gi)];
      wi[q] = wc[2 * (32 * m + gi) + 1];
    }
  }
  for (int e = tid; e < G * N; e += 256) pinv[e] = perminv[e];
  __syncthreads();
  // lane k's pieces of a row: float4 8 p + k (p < P), float2 16 P + k
  const float4* T4 = reinterpret_cast<const float4*>(Tpair) + k;
  const float2* T2 = reinterpret_cast<const float2*>(Tpair) + 16 * P + k;
  // unit u of a loaded row
  auto unit = [](const float4 (&b4)[P > 0 ? P : 1], const float2& b2, int u, float& Tr,
                 float& Ti) {
    if (u < 2 * P) {
      const float4 v = b4[u >> 1];
      Tr = (u & 1) ? v.z : v.x;
      Ti = (u & 1) ? v.w : v.y;
    } else {
      Tr = b2.x;
      Ti = b2.y;
    }
  };
  int64_t acc = 0;
  for (int r = 0; r < n_prop && valid; ++r) {
    if ((r & 63) == 0) {
      __syncthreads();
      if (tid < 64) {
        uint64_t rr[4];
        philox4x64_10(ctr + (uint64_t)tid, 0, 0, 0, seed, id, rr);
        rbuf[tid][0] = rr[0];
        rbuf[tid][1] = rr[1];
        rbuf[tid][2] = rr[2];
      }
      __syncthreads();
    }
    const uint64_t r0 = rbuf[r & 63][0], r1 = rbuf[r & 63][1], r2 = rbuf[r & 63][2];
    const int kup = (int)(((r0 >> 11) * (uint64_t)half) >> 53);
    const int kdn = (int)(((r1 >> 11) * (uint64_t)half) >> 53);
    const int i = select128(lo, hi, kup);
    const int j = select128(~lo & nmask_lo, ~hi & nmask_hi, kdn);
    // site-pair row of every image (row index p N + q, p/q the sites of i/j)
    int row[IPG];
#pragma unroll
    for (int m = 0; m < IPG; ++m)
      row[m] = (int)pinv[(32 * m + gi) * N + i] * N + pinv[(32 * m + gi) * N + j];
    // ratio pass: per image, the lane's partial product of (t T - 1), then
    // the group's product; rows read one image ahead
    // (the prefactor F is read with its row: a load issued after the next
    // image's rows would make its wait cover them too)
    const float2* F2 = reinterpret_cast<const float2*>(Fpair);
    float Rr[NSLOT], Ri[NSLOT];
    float4 b4[2][P > 0 ? P : 1];
    float2 b2[2], fb[2];
    auto load_row = [&](int q, int rw) {
#pragma unroll
      for (int p = 0; p < P; ++p) b4[q][p] = T4[(size_t)rw * (M / 2) + 8 * p];
      if constexpr (R) b2[q] = T2[(size_t)rw * M];
    };
    load_row(0, row[0]);
    fb[0] = F2[row[0]];
#pragma unroll
    for (int m = 0; m < IPG; ++m) {
      if (m + 1 < IPG) {
        load_row((m + 1) & 1, row[m + 1]);
        fb[(m + 1) & 1] = F2[row[m + 1]];
      }
      // the first factor starts the product (a product with 1 + 0i is not
      // folded away under IEEE semantics)
      float Tr, Ti;
      unit(b4[m & 1], b2[m & 1], 0, Tr, Ti);
      float pr = fmaf_t(tr[m][0], Tr, fmaf_t(-ti[m][0], Ti, -1.f));
      float pi = fmaf_t(tr[m][0], Ti, ti[m][0] * Tr);
#pragma unroll
      for (int u = 1; u < UPL; ++u) {
        unit(b4[m & 1], b2[m & 1], u, Tr, Ti);
        mul_factor(pr, pi, tr[m][u], ti[m][u], Tr, Ti);
      }
      group_cmul<8>(pr, pi);
      const float2 f = fb[m & 1];
      const float rr = f.x * pr - f.y * pi, ri = f.x * pi + f.y * pr;
      if (k == (m & 7)) {
        Rr[m >> 3] = rr;
        Ri[m >> 3] = ri;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    double cr = 0.0, ci = 0.0;
#pragma unroll
    for (int q = 0; q < NSLOT; ++q)
      if (k + 8 * q < IPG) {
        cr += (double)(wr[q] * Rr[q] - wi[q] * Ri[q]);
        ci += (double)(wr[q] * Ri[q] + wi[q] * Rr[q]);
      }
    cr = wave_sum_dpp(cr);
    ci = wave_sum_dpp(ci);
    double* rb = red[r & 1];
    if (lane == 0) {
      rb[wv] = cr;
      rb[4 + wv] = ci;
    }
    __syncthreads();
    const double sr = (rb[0] + rb[1]) + (rb[2] + rb[3]);
    const double si = (rb[4] + rb[5]) + (rb[6] + rb[7]);
    const double u = (double)(r2 >> 11) * (1.0 / 9007199254740992.0);
    const double den = sr * sr + si * si;
    // every lane holds the same sums: a wave-uniform decision
    if (__builtin_amdgcn_readfirstlane((int)(u < den))) {
      ++acc;
      const uint64_t mi = 1ull << (i & 63), mj = 1ull << (j & 63);
      lo ^= (i < 64 ? mi : 0ull) ^ (j < 64 ? mj : 0ull);
      hi ^= (i < 64 ? 0ull : mi) ^ (j < 64 ? 0ull : mj);
      // u' = u R / ratio
      const double id2 = 1.0 / den;
#pragma unroll
      for (int q = 0; q < NSLOT; ++q) {
        const double ar = (double)(wr[q] * Rr[q] - wi[q] * Ri[q]);
        const double ai = (double)(wr[q] * Ri[q] + wi[q] * Rr[q]);
        wr[q] = (float)((ar * sr + ai * si) * id2);
        wi[q] = (float)((ai * sr - ar * si) * id2);
      }
      // t' = (t - T) / (1 - t T).  The rows are read again, one image ahead;
      // an opaque zero offset keeps the compiler from hoisting these loads
      // above the acceptance test (registers for all of them at once)
      int z = 0;
      asm volatile("" : "+v"(z));
      load_row(0, row[0] + z);
#pragma unroll
      for (int m = 0; m < IPG; ++m) {
        if (m + 1 < IPG) load_row((m + 1) & 1, row[m + 1] + z);
#pragma unroll
        for (int u = 0; u < UPL; ++u) {
          float Tr, Ti;
          unit(b4[m & 1], b2[m & 1], u, Tr, Ti);
          tanh_add(tr[m][u], ti[m][u], Tr, Ti);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    ++ctr;
    if (phase == 1) {
      const int64_t idx = p0 + r + 1;
      if (idx % n_skip == 0) {
        const int64_t m = idx / n_skip - 1;
        if (m < n_per_chain && tid < N) {
          const uint64_t bit = tid < 64 ? (lo >> tid) & 1ull : (hi >> (tid - 64)) & 1ull;
          spins_out[((size_t)c * n_per_chain + m) * N + tid] = bit ? 1 : -1;
        }
      }
    }
  }
  if (tid == 0) {
    state[4 * c] = lo;
    state[4 * c + 1] = hi;
    state[4 * c + 2] = ctr;
    acc_out[c] += valid ? acc : -((int64_t)1 << 40);
  }
  if (tid < N) {
    const uint64_t bit = tid < 64 ? (lo >> tid) & 1ull : (hi >> (tid - 64)) & 1ull;
    cur_spins[(size_t)c * N + tid] = bit ? 1 : -1;
  }
}

template <int M, int IPG>
hipError_t launch_reg8(const nqs_ctx* c, int64_t n, const void* t, const void* w,
                       uint64_t* state, int cnt, int phase, int64_t p0, int ns, uint64_t seed,
                       int8_t* spins_out, int64_t n_per_chain, int64_t* acc, int8_t* cur,
                       hipStream_t st) {
  if (c->G != 32 * IPG || c->M != M || c->N > 128) return hipErrorNotSupported;
  sample_reg8_kernel<M, IPG><<<(unsigned)n, 256, (size_t)c->G * c->N, st>>>(
      c->N, c->G, c->n_htiles, c->dev.perminv, (const float*)c->par.Tpair,
      (const float*)c->par.Fpair, (const float*)t, (const float*)w, state, cnt, phase, p0, ns,
      seed, spins_out, n_per_chain, acc, cur);
  return hipGetLastError();
}

template <typename R, int M, int SPLIT>
hipError_t launch_reg(const nqs_ctx* c, int64_t n, const void* t, const void* w,
                      uint64_t* state, int cnt, int phase, int64_t p0, int ns, uint64_t seed,
                      int8_t* spins_out, int64_t n_per_chain, int64_t* acc, int8_t* cur,
                      hipStream_t st) {
  const int threads = SPLIT == 2 ? 64 * ((c->G + 31) / 32) : 64 * ((c->G + 63) / 64);
  if (threads > 640) return hipErrorNotSupported;
  sample_reg_kernel<R, M, SPLIT><<<(unsigned)n, threads, (size_t)c->G * c->N, st>>>(
      c->N, c->G, c->n_htiles, c->dev.perminv, (const R*)c->par.Tpair, (const R*)c->par.Fpair,
      (const R*)t, (const R*)w, state, cnt, phase, p0, ns, seed, spins_out, n_per_chain, acc,
      cur);
  return hipGetLastError();
}

// Dispatch to a register-resident instantiation, or hipErrorNotSupported.
hipError_t try_reg(const nqs_ctx* c, int64_t n, const void* t, const void* w, uint64_t* state,
                   int cnt, int phase, int64_t p0, int ns, uint64_t seed, int8_t* spins_out,
                   int64_t n_per_chain, int64_t* acc, int8_t* cur, hipStream_t st) {
  // FP32 only: the FP64 path (small lattices) stays on the cache-streaming kernel
  if (c->K != 1 || c->G > 512 || c->prec == NQS_FP64) return hipErrorNotSupported;
  // 6x6 (G = 288) with M = 72: eight lanes per image, 256 lanes per chain
  if (c->G == 288 && c->M == 72)
    return launch_reg8<72, 9>(c, n, t, w, state, cnt, phase, p0, ns, seed, spins_out,
                              n_per_chain, acc, cur, st);
#define NQS_REG_CASE(MM, SP)                                                                 \
  if (c->M == MM)                                                                            \
    return launch_reg<float, MM, SP>(c, n, t, w, state, cnt, phase, p0, ns, seed, spins_out, \
                                     n_per_chain, acc, cur, st);
  NQS_REG_CASE(8, 1)
  NQS_REG_CASE(16, 1)
  NQS_REG_CASE(32, 2)
  NQS_REG_CASE(72, 2)
#undef NQS_REG_CASE
  return hipErrorNotSupported;
}

__global__ void pack_kernel(const int8_t* __restrict__ spins, int64_t n, int N, uint64_t first,
                            uint64_t* __restrict__ state) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  uint64_t lo = 0, hi = 0;
  for (int i = 0; i < N; ++i)
    if (spins[c * N + i] > 0) {
      if (i < 64) lo |= 1ull << i;
      else hi |= 1ull << (i - 64);
    }
  state[4 * c] = lo;
  state[4 * c + 1] = hi;
  state[4 * c + 2] = 0;
  state[4 * c + 3] = first + (uint64_t)c;
}

__global__ void unpack_kernel(const uint64_t* __restrict__ state, int64_t n, int N,
                              int8_t* __restrict__ spins) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * N) return;
  const int64_t c = idx / N;
  const int i = (int)(idx % N);
  const uint64_t word = i < 64 ? state[4 * c] : state[4 * c + 1];
  spins[idx] = ((word >> (i & 63)) & 1ull) ? 1 : -1;
}

// N_skip = max(1, ceil(5 P / A)) from the burn-in counts of every chain.
__global__ void nskip_kernel(const int64_t* __restrict__ acc, int64_t n, int64_t proposals,
                             int32_t* __restrict__ out) {
  __shared__ long long part[256];
  long long a = 0;
  for (int64_t c = threadIdx.x; c < n; c += 256) a += acc[c] > 0 ? acc[c] : 0;
  part[threadIdx.x] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long A = 0;
    for (int q = 0; q < 256; ++q) A += part[q];
    const long long P = proposals * n;
    long long ns = A > 0 ? (5 * P + A - 1) / A : kNskipMax;
    ns = ns < 1 ? 1 : (ns > kNskipMax ? kNskipMax : ns);
    out[0] = (int32_t)ns;
  }
}

__global__ void acc_rate_kernel(const int64_t* __restrict__ acc, int64_t n, int64_t proposals,
                                float* __restrict__ rate) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  rate[c] = acc[c] < 0 ? NAN : (proposals > 0 ? (float)((double)acc[c] / (double)proposals) : 0.f);
}

inline size_t al(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace

size_t sample_workspace_bytes(const nqs_ctx* c, int64_t C) {
  const size_t rs = c->prec == NQS_FP64 ? 8 : 4, n = (size_t)std::max<int64_t>(C, 1);
  // two tanh(theta) caches (current and proposed state) for the streaming kernel
  return 2 * al(n * c->G * c->KM * 2 * rs) + al(n * c->K * c->G * 2 * rs) +
         al(n * c->K * c->G * 16) + al(n * 16) + al(n * c->N) + 2 * al(n * 8) + al(64);
}

}  // namespace nqs

using namespace nqs;

extern "C" {

nqs_status nqs_chain_init(nqs_ctx* c, const int8_t* spins, int64_t n_chains,
                          uint64_t first_chain_id, uint64_t* chain_state, hipStream_t st) {
  if (!c) return NQS_ERR_ARG;
  if (n_chains < 0 || (n_chains > 0 && (!spins || !chain_state))) {
    c->last_error = "chain_init: bad arguments";
    return NQS_ERR_ARG;
  }
  if (n_chains == 0) return NQS_OK;
  pack_kernel<<<(unsigned)((n_chains + 255) / 256), 256, 0, st>>>(spins, n_chains, c->N,
                                                                   first_chain_id, chain_state);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    c->last_error = std::string("chain_init: ") + hipGetErrorString(e);
    return NQS_ERR_DEVICE;
  }
  return NQS_OK;
}

nqs_status nqs_sample(nqs_ctx* c, int64_t n_chains, int64_t n_per_chain, int32_t n_skip,
                      int32_t n_burn, uint64_t seed, uint64_t* chain_state, int8_t* spins_out,
                      float* acc_rate_out, int32_t* n_skip_out, void* ws, size_t ws_bytes,
                      hipStream_t st) {
  if (!c) return NQS_ERR_ARG;
  auto fail = [&](nqs_status s, const std::string& m) {
    c->last_error = m;
    return s;
  };
  if (n_chains < 1 || n_per_chain < 0 || n_skip < 0 || n_burn < 0 || !chain_state)
    return fail(NQS_ERR_ARG, "sample: bad counts or NULL chain_state");
  if (n_skip == 0 && n_burn == 0)
    return fail(NQS_ERR_ARG, "sample: automatic N_skip needs burn-in proposals");
  if (n_per_chain > 0 && !spins_out) return fail(NQS_ERR_ARG, "sample: spins_out is NULL");
  if (n_skip > kNskipMax) return fail(NQS_ERR_ARG, "sample: n_skip above 1000");
  if (c->G > 1024) return fail(NQS_ERR_ARG, "sample: more than 1024 images");
  const size_t need = sample_workspace_bytes(c, n_chains);
  if (!ws || ws_bytes < need)
    return fail(NQS_ERR_ARG, "sample: workspace too small: need " + std::to_string(need));
  const size_t rs = c->prec == NQS_FP64 ? 8 : 4, n = (size_t)n_chains;
  char* p = (char*)ws;
  void* t = p;
  p += al(n * c->G * c->KM * 2 * rs);
  void* t2 = p;
  p += al(n * c->G * c->KM * 2 * rs);
  void* w = p;
  p += al(n * c->K * c->G * 2 * rs);
  double* L = (double*)p;
  p += al(n * c->K * c->G * 16);
  double* lp = (double*)p;
  p += al(n * 16);
  int8_t* cur = (int8_t*)p;
  p += al(n * c->N);
  int64_t* acc_burn = (int64_t*)p;
  p += al(n * 8);
  int64_t* acc_samp = (int64_t*)p;
  p += al(n * 8);
  int32_t* nsk = (int32_t*)p;

  hipError_t e = hipMemsetAsync(acc_burn, 0, n * 8, st);
  if (e == hipSuccess) e = hipMemsetAsync(acc_samp, 0, n * 8, st);
  if (e == hipSuccess) {
    unpack_kernel<<<(unsigned)((n * c->N + 255) / 256), 256, 0, st>>>(chain_state, n_chains, c->N,
                                                                       cur);
    e = hipGetLastError();
  }
  const int threads = std::max(64, (c->G + 63) / 64 * 64);
  const size_t lds = (size_t)c->G * c->K * 2 * rs + 64 * sizeof(double);
  auto refresh = [&]() -> hipError_t {
    hipError_t r = launch_theta(c, cur, n_chains, L, t, st);
    if (r == hipSuccess) r = launch_lse(c, L, n_chains, lp, w, st);
    return r;
  };
  auto run = [&](int phase, int64_t total, int ns_host, const int32_t* ns_dev,
                 int64_t* acc) -> hipError_t {
    for (int64_t p0 = 0; p0 < total; p0 += kSegment) {
      const int cnt = (int)std::min<int64_t>(kSegment, total - p0);
      hipError_t r = refresh();
      if (r != hipSuccess) return r;
      prof_begin(c, K_SAMPLE, st);
      r = try_reg(c, (int64_t)n, t, w, chain_state, cnt, phase, p0, ns_host, seed, spins_out,
                  n_per_chain, acc, cur, st);
      if (r == hipErrorNotSupported) {
        if (c->prec == NQS_FP64)
          sample_kernel<double><<<(unsigned)n, threads, lds, st>>>(
              c->N, c->G, c->K, c->M, c->n_htiles, c->dev.perminv, (const double*)c->par.Tpair,
              (const double*)c->par.Fpair, (double*)t, (double*)t2, (double*)w, chain_state, cnt,
              phase, p0,
              ns_dev, ns_host, seed, spins_out, n_per_chain, acc, cur);
        else
          sample_kernel<float><<<(unsigned)n, threads, lds, st>>>(
              c->N, c->G, c->K, c->M, c->n_htiles, c->dev.perminv, (const float*)c->par.Tpair,
              (const float*)c->par.Fpair, (float*)t, (float*)t2, (float*)w, chain_state, cnt,
              phase, p0,
              ns_dev, ns_host, seed, spins_out, n_per_chain, acc, cur);
        r = hipGetLastError();
      }
      prof_end(c, K_SAMPLE, st);
      if (r != hipSuccess) return r;
    }
    return hipSuccess;
  };
  if (e == hipSuccess) e = run(0, n_burn, 1, nullptr, acc_burn);
  int ns = n_skip;
  if (e == hipSuccess && n_skip == 0) {
    nskip_kernel<<<1, 256, 0, st>>>(acc_burn, n_chains, n_burn, nsk);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&ns, nsk, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  const int64_t total = n_per_chain * (int64_t)ns;
  if (e == hipSuccess) e = run(1, total, ns, nullptr, acc_samp);
  if (e == hipSuccess && acc_rate_out) {
    acc_rate_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(acc_samp, n_chains, total,
                                                                 acc_rate_out);
    e = hipGetLastError();
  }
  if (e == hipSuccess && n_skip_out) e = hipMemsetD32Async(n_skip_out, ns, 1, st);
  if (e != hipSuccess) return fail(NQS_ERR_DEVICE, std::string("sample: ") + hipGetErrorString(e));
  return NQS_OK;
}

}  // extern "C"
