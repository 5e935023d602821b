// Fused log psi + E_loc (Sec. 3.1 Eqs. (2), (6); Sec. 3.2 Eq. (10)) for
// models whose hidden layer does not fit in registers (K*M > 128,
// M a multiple of 16), with theta in FP32 or split BF16.
//
// A workgroup of kWideWaves wavefronts takes one sample at a time; every
// wavefront takes one 16-image column block, so all of them share the
// sample's antiparallel-bond list and do the same amount of work.  The hidden
// units are walked in chunks of kHC in lockstep across the workgroup:
//   * the chunk's rows of the bond table T = tanh(D) (all 4N bonds x kHC units)
//     are staged in LDS, double-buffered: each thread loads its share of the
//     next chunk into registers at the start of a chunk and stores it at the
//     end, so the loads overlap a whole chunk of work;
//   * theta of the chunk (kHC/8 hidden tiles) runs on 16x16 MFMA with the W
//     fragments read from L2, and the log 2cosh / tanh epilogue accumulates
//     log psi of the image across chunks;
//   * tanh(theta) of the chunk goes through a small LDS tile so that lane
//     (qg, c) holds all kHC values of image c, and the lane multiplies the
//     running products F_s prod_h (s + t_h T_h) of its bonds b = qg + 4 jb
//     (jb < wide_bonds) of the list, the bond rows read from LDS.
// At the end of each RBM the products are weighted with the image weights
// u = chi e^{L - m} (m a running maximum over the RBMs of the wave's images)
// and summed; the wave emits (m, sum u, sum u R) per (sample, column block)
// in the same format as the fused kernel, combined by its finish kernel.
// Bonds beyond 4 wide_bonds per sample are handled in further passes.
#include "theta_common.h"
#include "hops.h"

namespace nqs {

namespace {

constexpr int kWideWaves = 8;
// bonds per lane and pass (even: the products run two bonds at a time).
// Each pass recomputes theta, so 72 bonds per pass at 8x8 and 10x10 take
// their ~130 and ~200 antiparallel bonds in 2 and 3 passes where 64 took 3
// and 4 (10-11 % faster, with somewhat more spilling at N = 100).  The
// unordered-pair lists at 10x10 (~100 entries) take 2 passes either way, and
// there the extra registers only spill.
template <int N, bool PAIRS>
constexpr int wide_bonds() { return N >= 64 && !(PAIRS && N >= 100) ? 18 : 16; }
constexpr int kHC = 8;             // hidden units per chunk (multiple of 8)
constexpr int kRP = kHC / 2;       // float4 per staged row
constexpr int kTS = 2 * kHC + 4;   // LDS row stride of the staged table (floats)
constexpr int kXS = 2 * kHC + 4;   // LDS row stride of the tanh exchange tile (floats)

template <int N>
struct WideCfg {
  static constexpr int NB = 4 * N;
  static constexpr int NSTG = (NB * kRP + 64 * kWideWaves - 1) / (64 * kWideWaves);  // float4 / thread
  static constexpr int CAP16 = wide_cap16(NB);        // staged table, 16-byte units
  static constexpr size_t LDS = 2ull * CAP16 * 16 + (size_t)kWideWaves * 16 * kXS * 4 + NB * 2 +
                                NB * 4 + 16;
};

// PAIRS: the rows are exchange neighbours with parent bonds (parent[s]); the
// bond list is the parent's unordered-pair list and pairs counted twice weigh 2.
// WL: also write the images' log amplitudes, unreduced (see below).
template <int N, int PREC, bool PAIRS, bool WL>
__global__ __launch_bounds__(64 * kWideWaves) void eloc_wide_kernel(
    const int8_t* __restrict__ spins, int64_t S, const uint8_t* __restrict__ perm, int G, int K,
    int M, const typename ThetaTraits<PREC>::AFrag* __restrict__ wfrag,
    const float* __restrict__ bias, const float* __restrict__ avec,
    const int32_t* __restrict__ bonds, const int32_t* __restrict__ wmap,
    const int32_t* __restrict__ wrow,
    const double* __restrict__ chi, const float* __restrict__ Tpm, const float* __restrict__ F,
    double* __restrict__ part, const int16_t* __restrict__ parent, double* __restrict__ Lout) {
  using T = ThetaTraits<PREC>;
  using Cfg = WideCfg<N>;
  constexpr int NB = Cfg::NB, NK = nk_of<N, PREC>(), NSTG = Cfg::NSTG;
  constexpr int kWB = wide_bonds<N, PAIRS>();
  static_assert(kWB % 2 == 0 && kWB <= 32, "bond slots: pairs, one bit each in a word");
  static_assert(kTS == 4 * kWideRow16, "row size of the placement");
  __shared__ __align__(16) float Tc[2][Cfg::CAP16 * 4];
  __shared__ int wrl[NB];                    // row starts in floats
  __shared__ __align__(16) float tx[kWideWaves][16 * kXS];
  __shared__ uint16_t list[NB];
  __shared__ int nc_s;
  // WL: the wave's unreduced log amplitudes [RBM][image][4], held until the
  // end of its image round (stores from the chunk loop slowed it)
  __shared__ double lraw[WL ? kWideWaves : 1][WL ? kWideLrawK * 16 * 4 : 1];

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int q = lane >> 4, c = lane & 15;
  const int KM = K * M, NCH = KM / kHC, CPR = M / kHC, nblk = G / 16;
  const int rounds = (nblk + kWideWaves - 1) / kWideWaves;

  // staging of chunk ch: element e = tid + 512 i -> row e / kRP, 16-byte part
  // e % kRP of tanh(D); thread tid < NB also stages (F_+, F_-) of row tid for
  // the chunk's RBM into the row's last 16 bytes.  The values sit in named
  // registers (s0..s7, sF) between the loads and the LDS stores; the loads are
  // unconditional (clamped to valid elements).
  static_assert(NSTG <= 8, "staging registers");
  float4 s0, s1, s2, s3, s4, s5, s6, s7, sF;
#define NQS_STG_LD(I, CH)                                                                \
  if constexpr (I < NSTG) {                                                              \
    int e = tid + 64 * kWideWaves * I;                                                   \
    e = e < NB * kRP ? e : 0;                                                            \
    s##I = *reinterpret_cast<const float4*>(Tpm + (size_t)(e / kRP) * 4 * KM +           \
                                            2 * kHC * (CH) + 4 * (e % kRP));             \
  }
#define NQS_STG_ST(I, BUF)                                                               \
  if constexpr (I < NSTG) {                                                              \
    const int e = tid + 64 * kWideWaves * I;                                             \
    if (e < NB * kRP) *reinterpret_cast<float4*>(&Tc[BUF][wrl[e / kRP] + 4 * (e % kRP)]) = s##I; \
  }
#define NQS_STAGE_LOAD(CH)                                                               \
  {                                                                                      \
    NQS_STG_LD(0, CH) NQS_STG_LD(1, CH) NQS_STG_LD(2, CH) NQS_STG_LD(3, CH)              \
    NQS_STG_LD(4, CH) NQS_STG_LD(5, CH) NQS_STG_LD(6, CH) NQS_STG_LD(7, CH)              \
    sF = *reinterpret_cast<const float4*>(F + ((size_t)((CH) / CPR) * NB + (tid < NB ? tid : 0)) * 4); \
  }
#define NQS_STAGE_STORE(BUF)                                                             \
  {                                                                                      \
    NQS_STG_ST(0, BUF) NQS_STG_ST(1, BUF) NQS_STG_ST(2, BUF) NQS_STG_ST(3, BUF)          \
    NQS_STG_ST(4, BUF) NQS_STG_ST(5, BUF) NQS_STG_ST(6, BUF) NQS_STG_ST(7, BUF)          \
    if (tid < NB) *reinterpret_cast<float4*>(&Tc[BUF][wrl[tid] + 2 * kHC]) = sF;         \
  }
  for (int idx = tid; idx < NB; idx += 64 * kWideWaves) wrl[idx] = 4 * wrow[idx];
  __syncthreads();
  NQS_STAGE_LOAD(0)
  NQS_STAGE_STORE(0)
  int gc = 0;                                  // chunks processed by the workgroup so far

  for (int64_t s = blockIdx.x; s < S; s += gridDim.x) {
    const int8_t* srow = spins + s * N;
    __syncthreads();                           // previous sample done with the list
    if (wv == 0) {
      // with a parent bond b1 (s is the exchange neighbour s0^{b1} of a
      // two-hop sum): the unordered-pair list of the second hops (b1 itself
      // excluded, bonds disjoint from b1 only above it, counted twice: flag 0x4000)
      const int b1 = PAIRS ? (int)parent[s] : -1;
      const int i1 = b1 >= 0 ? bonds[2 * b1] : -1, j1 = b1 >= 0 ? bonds[2 * b1 + 1] : -1;
      int n = 0;
      for (int base = 0; base < NB; base += 64) {
        const int b = base + lane;
        bool anti = false, twice = false;
        int sp = 0;
        if (b < NB) {
          const int bi = bonds[2 * b], bj = bonds[2 * b + 1];
          sp = srow[bi];
          anti = sp != srow[bj];
          if (anti && b1 >= 0) {
            const bool shared = bi == i1 || bi == j1 || bj == i1 || bj == j1;
            anti = b != b1 && (shared || b > b1);
            twice = !shared;
          }
        }
        const unsigned long long msk = __ballot(anti);
        const int pos = __popcll(msk & ((1ull << lane) - 1ull));
        if (anti) list[n + pos] = (uint16_t)(b | (sp > 0 ? 0x8000 : 0) | (twice ? 0x4000 : 0));
        n += __popcll(msk);
      }
      if (lane == 0) nc_s = n;
    }
    __syncthreads();
    const int nc = nc_s;
    const int npass = nc > 0 ? (nc + 4 * kWB - 1) / (4 * kWB) : 1;

    for (int rd = 0; rd < rounds; ++rd) {
      const int blk = rd * kWideWaves + wv;
      const bool active = blk < nblk;
      const int g = (active ? blk : 0) * 16 + c;
      const uint8_t* prow = perm + (size_t)g * N;
      typename T::BFrag bx[NK];
      load_bfrag_gather<N, PREC>(srow, prow, q, bx);
      const float ch_g = (float)chi[g];
      double m_item = -INFINITY, Qr = 0.0, Qi = 0.0, denr = 0.0, deni = 0.0;

      for (int pass = 0; pass < npass; ++pass) {
        // this lane's bonds: list entries pass * 4 kWB + q + 4 jb
        int offs[kWB];                  // 2 * (row offset in floats) + (sign < 0)
        uint32_t twice = 0u;                   // bit jb: an unordered pair counted twice
        const int i0 = pass * 4 * kWB + q;
        const int nv = nc > i0 ? min(kWB, (nc - i0 + 3) / 4) : 0;
        // bonds per lane of lane group 0 (the most of any group): a partly
        // filled pass skips the empty pairs of slots
        const int p0 = pass * 4 * kWB;
        const int nvu = __builtin_amdgcn_readfirstlane(
            nc > p0 ? min(kWB, (nc - p0 + 3) / 4) : 0);
#pragma unroll
        for (int jb = 0; jb < kWB; ++jb) {
          const int ii = i0 + 4 * jb;
          const int e = ii < nc ? list[ii] : 0;   // padding entries use bond 0
          offs[jb] = wmap[(size_t)g * NB + (e & 0x3fff)] ^ (e >> 15);
          if (PAIRS && (e & 0x4000)) twice |= 1u << jb;
        }
        float Pr[kWB], Pi[kWB];
        float lpr = 1.f, lpi = 0.f;
        int lpe = 0;
        uint32_t lpar = 0u;
        double sax = 0.0;

        for (int ch = 0; ch < NCH; ++ch, ++gc) {
          const int k = ch / CPR;
          const int buf = gc & 1;
          const int nxt = ch + 1 < NCH ? ch + 1 : 0;
          if (ch % CPR == 0) {                 // RBM start: products begin at F_s
#pragma unroll
            for (int jb = 0; jb < kWB; ++jb) {
              const float* f = Tc[buf] + (offs[jb] >> 1) + 2 * kHC + 2 * (offs[jb] & 1);
              Pr[jb] = f[0];
              Pi[jb] = f[1];
            }
          }
          // theta of the chunk's hidden tiles, epilogue, tanh to LDS
#pragma unroll
          for (int tt = 0; tt < kHC / 8; ++tt) {
            const int ht = (kHC / 8) * ch + tt;
            const int h0 = 8 * ht + 2 * q;
            typename T::Acc acc;
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] = bias[2 * h0 + v];   // start from the biases
#pragma unroll
            for (int kk = 0; kk < NK; ++kk) acc = mfma(wfrag[((size_t)ht * NK + kk) * 64 + lane], bx[kk], acc);
            float axs = 0.f;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
              float tr, ti;
              axs += logcosh_step<float, true>(acc[2 * u], acc[2 * u + 1], lpr, lpi, lpar, tr, ti);
              const int hl = 8 * tt + 2 * q + u;
              tx[wv][c * kXS + 2 * hl] = tr;
              tx[wv][c * kXS + 2 * hl + 1] = ti;
            }
            sax += (double)axs;
          }
          renorm(lpr, lpi, lpe);
          wave_sync_lds();
          float t[2 * kHC];
#pragma unroll
          for (int e = 0; e < kHC / 2; ++e) {
            const float4 v = *reinterpret_cast<const float4*>(&tx[wv][c * kXS + 4 * e]);
            t[4 * e] = v.x; t[4 * e + 1] = v.y; t[4 * e + 2] = v.z; t[4 * e + 3] = v.w;
          }
          NQS_STAGE_LOAD(nxt)                  // lands during the bond products
          // bond products of the chunk, two bonds at a time
#pragma unroll
          for (int jb = 0; jb < kWB; jb += 2) {
            if (jb < nvu) {
            const float* r0 = Tc[buf] + (offs[jb] >> 1);
            const float* r1 = Tc[buf] + (offs[jb + 1] >> 1);
            const float sg0 = (offs[jb] & 1) ? -1.f : 1.f, sg1 = (offs[jb + 1] & 1) ? -1.f : 1.f;
            float ar = Pr[jb], ai = Pi[jb], br = Pr[jb + 1], bi = Pi[jb + 1];
#pragma unroll
            for (int e = 0; e < kHC / 2; ++e) {
              const float4 x0 = *reinterpret_cast<const float4*>(r0 + 4 * e);
              const float4 x1 = *reinterpret_cast<const float4*>(r1 + 4 * e);
#pragma unroll
              for (int hh = 0; hh < 2; ++hh) {
                const float tr = t[4 * e + 2 * hh], ti = t[4 * e + 2 * hh + 1];
                const float T0r = hh ? x0.z : x0.x, T0i = hh ? x0.w : x0.y;
                const float T1r = hh ? x1.z : x1.x, T1i = hh ? x1.w : x1.y;
                float pa = fmaf(tr, T0r, fmaf(-ti, T0i, sg0)), pb = fmaf(tr, T0i, ti * T0r);
                float nr = fmaf(ar, pa, -(ai * pb));
                ai = fmaf(ar, pb, ai * pa);
                ar = nr;
                pa = fmaf(tr, T1r, fmaf(-ti, T1i, sg1));
                pb = fmaf(tr, T1i, ti * T1r);
                nr = fmaf(br, pa, -(bi * pb));
                bi = fmaf(br, pb, bi * pa);
                br = nr;
              }
            }
            Pr[jb] = ar; Pi[jb] = ai; Pr[jb + 1] = br; Pi[jb + 1] = bi;
            }
          }
          if (ch % CPR == CPR - 1) {           // RBM k complete: weight and sum
            apply_parity(lpr, lpi, lpar);
            int E = lpe;
            float pr = lpr, pi = lpi;
            double sx = sax;
#pragma unroll
            for (int o = 16; o <= 32; o <<= 1) {
              const float orr = __shfl_xor(pr, o, 64), oi = __shfl_xor(pi, o, 64);
              const float nr = pr * orr - pi * oi;
              pi = pr * oi + pi * orr;
              pr = nr;
              E += __shfl_xor(E, o, 64);
              sx += __shfl_xor(sx, o, 64);
            }
            double axr = 0.0, axi = 0.0;
            const float* ak = avec + (size_t)k * N * 2;
            for (int jj = q; jj < N; jj += 4) {
              const double xj = 0.5 * (double)srow[prow[jj]];
              axr += xj * (double)ak[2 * jj];
              axi += xj * (double)ak[2 * jj + 1];
            }
            axr += __shfl_xor(axr, 16, 64);
            axi += __shfl_xor(axi, 16, 64);
            axr += __shfl_xor(axr, 32, 64);
            axi += __shfl_xor(axi, 32, 64);
            const double Er = axr + sx + (double)E * 0.69314718055994530942;
            if (WL && pass == 0 && q == 0) {
              // the image's log amplitude L_kg = log(prod_h 2 cosh theta) + a x,
              // unreduced: (Er, a x imaginary part, the joined product P) with
              // L = Er + log|P| + i (Im a x + arg P), for a gradient pass on the
              // same configurations (the log and arg are taken there)
              double* o = &lraw[wv][(k * 16 + c) * 4];
              o[0] = Er;
              o[1] = axi;
              o[2] = (double)pr;
              o[3] = (double)pi;
            }
            const double mk = wave_max(Er);
            if (mk > m_item) {
              const double sc = (double)exp_t((float)(m_item - mk));   // 0 at the first RBM
              Qr *= sc; Qi *= sc; denr *= sc; deni *= sc;
              m_item = mk;
            }
            const float e = ch_g * exp_t((float)(Er - m_item));
            float sn, cs;
            sincos_t((float)axi, &sn, &cs);
            const float ur = e * (pr * cs - pi * sn), ui = e * (pr * sn + pi * cs);
            double sr = 0.0, si = 0.0;
#pragma unroll
            for (int jb = 0; jb < kWB; ++jb) {
              if constexpr (PAIRS) {
                const double wj = ((twice >> jb) & 1u) ? 2.0 : 1.0;
                sr += jb < nv ? wj * (double)Pr[jb] : 0.0;
                si += jb < nv ? wj * (double)Pi[jb] : 0.0;
              } else {
                sr += jb < nv ? (double)Pr[jb] : 0.0;
                si += jb < nv ? (double)Pi[jb] : 0.0;
              }
            }
            Qr += (double)ur * sr - (double)ui * si;
            Qi += (double)ur * si + (double)ui * sr;
            if (pass == 0 && q == 0) {
              denr += (double)ur;
              deni += (double)ui;
            }
            lpr = 1.f; lpi = 0.f; lpe = 0; lpar = 0u; sax = 0.0;
          }
          NQS_STAGE_STORE(gc & 1 ? 0 : 1)
          __syncthreads();
        }
      }
      Qr = wave_sum(Qr);
      Qi = wave_sum(Qi);
      denr = wave_sum(denr);
      deni = wave_sum(deni);
      if (WL && active) {
        // the round's log amplitudes to [S][K][G][4]: 16 images x 4 reals per RBM
        for (int e = lane; e < K * 64; e += 64) {
          const int kk = e >> 6, ci = (e >> 2) & 15, j = e & 3;
          Lout[(((size_t)s * K + kk) * G + blk * 16 + ci) * 4 + j] = lraw[wv][e];
        }
      }
      if (active && lane == 0) {
        double* o = part + ((size_t)s * nblk + blk) * 6;
        o[0] = m_item;
        o[1] = denr;
        o[2] = deni;
        o[3] = Qr;
        o[4] = Qi;
        o[5] = 0.0;
      }
    }
  }
}

#undef NQS_STG_LD
#undef NQS_STG_ST
#undef NQS_STAGE_LOAD
#undef NQS_STAGE_STORE

template <int N, int PREC>
hipError_t run(const nqs_ctx* c, const int8_t* spins, int64_t S, double* part, hipStream_t st,
               const int16_t* parent, double* Lout) {
#define NQS_WIDE_ARGS                                                                     \
  spins, S, c->dev.perm, c->G, c->K, c->M, wf, (const float*)c->par.bias,                 \
      (const float*)c->par.avec, c->dev.bonds, c->dev.wmap, c->dev.wrow, c->dev.chi,      \
      (const float*)c->par.Tpm, (const float*)c->par.F, part
  const int64_t blocks = std::min<int64_t>(S, c->n_cu > 0 ? c->n_cu : 256);
  const auto* wf = (const typename ThetaTraits<PREC>::AFrag*)(PREC == kPrecF32X3 ? c->par.wfrag3
                                                                                 : c->par.wfrag);
  if (parent)
    eloc_wide_kernel<N, PREC, true, false><<<(unsigned)blocks, 64 * kWideWaves, 0, st>>>(
        NQS_WIDE_ARGS, parent, nullptr);
  else if (Lout)
    eloc_wide_kernel<N, PREC, false, true><<<(unsigned)blocks, 64 * kWideWaves, 0, st>>>(
        NQS_WIDE_ARGS, nullptr, Lout);
  else
    eloc_wide_kernel<N, PREC, false, false><<<(unsigned)blocks, 64 * kWideWaves, 0, st>>>(
        NQS_WIDE_ARGS, nullptr, nullptr);
#undef NQS_WIDE_ARGS
  return hipGetLastError();
}

}  // namespace

bool eloc_wide_supported(const nqs_ctx* c) {
  if (c->prec == NQS_FP64 || c->KM <= 128 || c->M % kHC != 0) return false;
  return c->N == 36 || c->N == 64 || c->N == 100;
}

namespace {
hipError_t dispatch(const nqs_ctx* c, const int8_t* spins, int64_t S, const int16_t* parent,
                    double* part, double* Lout, hipStream_t st) {
  if (S <= 0) return hipSuccess;
  const bool bf = c->prec == NQS_BF16X2;
  switch (c->N) {
    case 36: return bf ? run<36, NQS_BF16X2>(c, spins, S, part, st, parent, Lout)
                       : run<36, kPrecF32X3>(c, spins, S, part, st, parent, Lout);
    case 64: return bf ? run<64, NQS_BF16X2>(c, spins, S, part, st, parent, Lout)
                       : run<64, kPrecF32X3>(c, spins, S, part, st, parent, Lout);
    case 100: return bf ? run<100, NQS_BF16X2>(c, spins, S, part, st, parent, Lout)
                        : run<100, kPrecF32X3>(c, spins, S, part, st, parent, Lout);
    default: return hipErrorNotSupported;
  }
}
}  // namespace

hipError_t launch_eloc_wide(const nqs_ctx* c, const int8_t* spins, int64_t S, double* part,
                            hipStream_t st, double* Lout) {
  return dispatch(c, spins, S, nullptr, part, Lout, st);
}

hipError_t launch_eloc_wide_pairs(const nqs_ctx* c, const int8_t* spins, int64_t S,
                                  const int16_t* parent, double* part, hipStream_t st) {
  return dispatch(c, spins, S, parent, part, nullptr, st);
}

}  // namespace nqs
