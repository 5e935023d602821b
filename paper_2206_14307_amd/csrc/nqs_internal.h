// Internal declarations shared by the host API and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/nqs.h"

namespace nqs {

constexpr int kMaxN = 100;          // L <= 10
constexpr int kMaxKM = 4096;

// Geometry of the L x L torus and its space group, built on the host at
// nqs_create (Sec. 3.1).  Bonds: 4N, index b = kind*N + i for the J1 bonds
// (i, i+x), (i, i+y) (kinds 0, 1) and the J2 bonds (i, i+x+y), (i, i+x-y)
// (kinds 2, 3).
struct Geometry {
  int L = 0, N = 0, G = 0, NB = 0;
  std::vector<uint8_t> perm;      // [G][N]  perm_g(i)
  std::vector<int32_t> bond_i, bond_j;
  std::vector<double> bond_J;     // [NB]
  std::vector<int32_t> bmap;      // [G][NB]  2*beta + flip: pre-image of bond b under g
  std::vector<double> chi;        // [G] (real for the supported K and irreps)
};

bool build_geometry(int L, double J1, double J2, int kx, int ky, int irrep, Geometry& geo,
                    std::string& err);

// LDS rows of the fused E_loc kernel: ROW = 2KM + 18K reals per bond, taking
// row16 = ceil(ROW * sizeof(R) / 16) sixteen-byte units; the kernel reserves
// fused_cap16 units.  place_fused_rows returns each bond row's start (units)
// such that every 16-image column block reads distinct bank groups, or an
// empty vector if the packing does not fit in cap16.
constexpr int fused_row16(int K, int M, int real_bytes) {
  return ((2 * K * M + 18 * K) * real_bytes + 15) / 16;
}
constexpr int fused_cap16(int NB, int row16) { return NB * (row16 | 1) + 256; }
std::vector<int> place_fused_rows(const Geometry& geo, int row16, int cap16);
// Rows of the wide E_loc kernel's staged chunk table: 5 sixteen-byte units
// (tanh D of 8 hidden units, then F_+, F_-), placed the same way.
constexpr int kWideRow16 = 5;
constexpr int wide_cap16(int NB) { return NB * kWideRow16 + 256; }
// RBMs whose log amplitudes the wide E_loc kernel can hand to the gradient
constexpr int kWideLrawK = 4;

// Binomial table of the Sz = 0 enumeration; false if C(N, N/2) overflows int64.
bool sz0_binomials(int N, std::vector<uint64_t>& b, int64_t& count);

// Device-side tables owned by the context.
struct DeviceTables {
  uint8_t* perm = nullptr;        // [G][N]
  uint8_t* perminv = nullptr;     // [G][N]  position l with perm_g(l) = site
  int32_t* bonds = nullptr;       // [NB][2]
  double* bond_J = nullptr;       // [NB]
  int32_t* bmap = nullptr;        // [G][NB]
  double* chi = nullptr;          // [G]
  uint64_t* binom = nullptr;      // [N+1][N+1] binomials (Sz = 0 enumeration), if C(N,N/2) fits
  int32_t* fmap = nullptr;        // [G][NB] fused kernel: 2 * (LDS row offset in reals) + flip
  int32_t* frow = nullptr;        // [NB]    fused kernel: LDS row offset in reals
  int32_t* wmap = nullptr;        // [G][NB] wide kernel: 2 * (LDS row offset in floats) + flip
  int32_t* wrow = nullptr;        // [NB]    wide kernel: LDS row start in 16-byte units
};

// Parameter-derived tables (rebuilt by nqs_set_params).  "R" is double for
// NQS_FP64 and float otherwise; complex values are (re, im) pairs of R.
struct ParamTables {
  double* params = nullptr;       // [P] complex double, caller layout
  void* wfrag = nullptr;          // MFMA A-operand fragments of the interleaved W
  void* wfrag3 = nullptr;         // FP32 models: BF16 fragments of [W_hi | W_mid | W_lo | 0]
  void* wfrag_s3 = nullptr;       // FP32 models (N % 4 == 0): site-grouped three-term fragments
  void* bias = nullptr;           // [K*M] complex R (zeros without bias)
  void* avec = nullptr;           // [K][N] complex R
  void* Tpm = nullptr;            // [NB][2][K*M] complex R: +tanh(D), -tanh(D)
  void* F = nullptr;              // [K][NB][2] complex R: (J/2) exp(s A) prod_h cosh D
  void* Tpair = nullptr;          // [N][N][K*M] complex R: tanh(W_h,p - W_h,q) (sampler)
  void* Fpair = nullptr;          // [K][N][N] complex R: exp(-(a_p - a_q)) prod_h cosh(W_h,p - W_h,q)
  void* Tdir = nullptr;           // [NB][2*K*M + 18*K] R: fused-kernel rows, direct form
  void* Urec = nullptr;           // [NB][2*K*M + 18*K] R: fused-kernel rows, reciprocal form
  double* flag = nullptr;         // [2] non-finite detector, reciprocal-form range violation
  bool recip_ok = false;          // Urec usable for the current parameters
};

}  // namespace nqs

namespace nqs {
enum KernelId { K_THETA = 0, K_LSE, K_ELOC, K_ELOC_FIN, K_TWOHOP, K_TWOHOP_FIN, K_MOMENTS,
                K_GRAD, K_SAMPLE, K_SR, K_GRAM, K_CHOL, K_SQ, K_CG, K_HOP3, K_COUNT };
struct Profiler {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[K_COUNT];
  double ms[K_COUNT] = {};
  int64_t n[K_COUNT] = {};
};
}  // namespace nqs

struct nqs_ctx {
  nqs_model_desc d{};
  int L = 0, N = 0, G = 0, NB = 0, K = 0, M = 0, KM = 0, P_rbm = 0;
  int64_t P = 0;
  int prec = 1;
  int64_t sector_count = -1;      // C(N, N/2), -1 if it overflows int64
  bool direct_only = false;       // nqs_set_factor_form: direct exchange-factor forms only
  int n_htiles = 0;               // K*M/8 hidden tiles of 8 units (16 interleaved rows)
  int nk = 0;                     // MFMA K-steps over the site axis
  nqs::Geometry geo;
  nqs::DeviceTables dev;
  nqs::ParamTables par;
  std::string last_error;
  int device = 0;
  int n_cu = 0;                   // compute units of the device (persistent grids)
  mutable nqs::Profiler prof;   // timing only, not model state
};

namespace nqs {
// Bracket one launch with events when profiling is enabled.
inline void prof_begin(const nqs_ctx* c, int k, hipStream_t st) {
  if (!c->prof.on) return;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return;
  if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return; }
  (void)hipEventRecord(a, st);
  c->prof.ev[k].push_back({a, b});
}
inline void prof_end(const nqs_ctx* c, int k, hipStream_t st) {
  if (!c->prof.on || c->prof.ev[k].empty()) return;
  (void)hipEventRecord(c->prof.ev[k].back().second, st);
}
}  // namespace nqs

namespace nqs {

// ----------------------------------------------------------------- launchers
// All launchers enqueue on `st` and return hipGetLastError().
hipError_t launch_prep(const nqs_ctx* c, hipStream_t st);
hipError_t launch_prep_pairs(const nqs_ctx* c, hipStream_t st);
hipError_t launch_check_finite(const double* p, int64_t n, double* flag, hipStream_t st);

// theta = W x + b for every (sample, image), epilogue: per-(k, image)
// L = a.x + sum_h log 2cosh(theta) (complex double [S][K][G]) and, if t_out,
// t = tanh(theta) as complex R in layout [S][n_htiles][G][8].
hipError_t launch_theta(const nqs_ctx* c, const int8_t* spins, int64_t S, double* Lout,
                        void* t_out, hipStream_t st);
// Per sample: log psi = LSE_{k,g}(log chi_g + L), w[s][k][g] = chi_g exp(L - log psi)
// (complex R; skipped if w_out is null).
// raw: L unreduced as the wide E_loc kernel writes it (four reals per image)
hipError_t launch_lse(const nqs_ctx* c, const double* L, int64_t S, double* logpsi_out,
                      void* w_out, hipStream_t st, bool raw = false);
// Bond-exchange sums: partial[s][tile] = sum_{b anti} (J_b/2) sum_{g in tile, k} w R.
hipError_t launch_eloc_bonds(const nqs_ctx* c, const int8_t* spins, int64_t S, const void* t,
                             const void* w, double* partial, hipStream_t st);
hipError_t launch_eloc_bonds_reg(const nqs_ctx* c, const int8_t* spins, int64_t S, const void* t,
                                 const void* w, double* partial, hipStream_t st);
// Fused theta + epilogue + bond exchanges (K*M <= 128 register-resident
// variants); part holds S * (G/16) * 6 doubles.
bool eloc_fused_supported(const nqs_ctx* c);
bool grad_fused_supported(const nqs_ctx* c);
hipError_t launch_enum_sz0(const nqs_ctx* c, int64_t count, int8_t* out, hipStream_t st);
bool eloc_wide_supported(const nqs_ctx* c);
// Lout (optional): the per-image log amplitudes [S][K][G], unreduced (four
// reals each, see launch_lse), for a gradient pass on the same configurations
hipError_t launch_eloc_wide(const nqs_ctx* c, const int8_t* spins, int64_t S, double* part,
                            hipStream_t st, double* Lout = nullptr);
hipError_t launch_fused_finish(const nqs_ctx* c, const int8_t* spins, int64_t S,
                               const double* part, double* logpsi, double* eloc, int eloc_stride,
                               hipStream_t st);
hipError_t launch_grad_fused(const nqs_ctx* c, const int8_t* spins, int64_t S, void* O,
                             double* logpsi, hipStream_t st);
hipError_t launch_eloc_fused(const nqs_ctx* c, const int8_t* spins, int64_t S, double* part,
                             double* logpsi, double* eloc, int eloc_stride, hipStream_t st);
hipError_t launch_eloc_finish(const nqs_ctx* c, const int8_t* spins, int64_t S,
                              const double* partial, double* eloc_out, int eloc_stride,
                              hipStream_t st);
// Two-hop: partial2[s][slot][tile] for e2 (slot = index in the antiparallel list).
hipError_t launch_twohop(const nqs_ctx* c, const int8_t* spins, int64_t S, const void* t,
                         const void* w, double* partial2, hipStream_t st);
hipError_t launch_twohop_reg(const nqs_ctx* c, const int8_t* spins, int64_t S, const void* t,
                             const void* w, double* partial2, hipStream_t st);
hipError_t launch_twohop_finish(const nqs_ctx* c, const int8_t* spins, int64_t S,
                                const double* partial2, double* e1e2, hipStream_t st);
hipError_t launch_moments(const double* e1e2, const double* logpsi, int64_t S, int exact,
                          double* partial, int nblocks, double* result, hipStream_t st);
size_t sample_workspace_bytes(const nqs_ctx* c, int64_t n_chains);
size_t sr_workspace_bytes(const nqs_ctx* c, int64_t S);
size_t sq_workspace_bytes(const nqs_ctx* c, int64_t S);
size_t cg_workspace_bytes(const nqs_ctx* c, int64_t S);
hipError_t launch_energy_stats(const double* eloc, int64_t S, double* stats, hipStream_t st);
hipError_t launch_params_step(const double* params, const double* dtheta, int64_t P, int is_complex,
                              double* next, double* stats, hipStream_t st);
hipError_t launch_sq(const nqs_ctx* c, const int8_t* spins, int64_t S, const double* weights,
                     double* out, void* ws, hipStream_t st);
// Three-hop e3 (p = 2 Lanczos): per-configuration antiparallel-bond counts,
// their exclusive scan (off[n] = total), the neighbour rows, e3 from the
// neighbours' log psi and e2, and the fifth-order moments + 3x3 solve.
hipError_t launch_nb_count(const nqs_ctx* c, const int8_t* spins, int64_t n, int32_t* cnt,
                           hipStream_t st);
hipError_t launch_nb_scan(const int32_t* cnt, int64_t n, int32_t* off, hipStream_t st);
hipError_t launch_nb_write(const nqs_ctx* c, const int8_t* spins, int64_t n, const int32_t* off,
                           int8_t* out, hipStream_t st);
hipError_t launch_e3_combine(const nqs_ctx* c, const int8_t* spins, int64_t n, const int32_t* off,
                             const double* lp, const double* e1e2, const double* lp_nb,
                             const double* e1e2_nb, double* e3, hipStream_t st);
hipError_t launch_moments2(const double* e1e2, const double* e3, const double* logpsi, int64_t S,
                           int exact, double* result, hipStream_t st);
hipError_t launch_grad(const nqs_ctx* c, const int8_t* spins, int64_t S, const void* t,
                       const void* w, void* O_out, hipStream_t st);
// O_k for K*M > 128 (FP32 / split-BF16 theta) from the normalised image
// weights w [S][K][G] (complex float) of launch_lse, theta recomputed in-kernel.
bool grad_wide_supported(const nqs_ctx* c);
hipError_t launch_grad_wide(const nqs_ctx* c, const int8_t* spins, int64_t S, const void* w,
                            void* O_out, hipStream_t st);
// Resolve the current device's copy of the allocation-free entry point's
// scratch array (once per device; the device must be current).
hipError_t noalloc_scratch_init(int device);

}  // namespace nqs
