// C ABI entry points (declared and documented in include/nqs.h): argument
// validation, workspace carving, chunking over samples, kernel launches.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "nqs_internal.h"
#include "hops.h"

using namespace nqs;

namespace {

// Launch with optional event bracketing (nqs_profile_enable).
#define NQS_RUN(ctx, kid, stream, call)   \
  ([&]() -> hipError_t {                  \
    prof_begin((ctx), (kid), (stream));   \
    const hipError_t e_ = (call);         \
    prof_end((ctx), (kid), (stream));     \
    return e_;                            \
  }())

constexpr size_t kChunkBytes = size_t(2) << 30;   // per-chunk working set
constexpr size_t kAlign = 256;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

nqs_status fail(nqs_ctx* c, nqs_status s, const std::string& msg) {
  if (c) c->last_error = msg;
  return s;
}

nqs_status hip_fail(nqs_ctx* c, hipError_t e, const char* where) {
  return fail(c, NQS_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

size_t real_size(const nqs_ctx* c) { return c->prec == NQS_FP64 ? 8 : 4; }

// Per-sample bytes of the chunked intermediates.
struct ChunkSizes {
  size_t L, w, t, partial, partial2;
};
ChunkSizes per_sample(const nqs_ctx* c) {
  ChunkSizes z;
  z.L = (size_t)c->K * c->G * 16;
  z.w = (size_t)c->K * c->G * 2 * real_size(c);
  z.t = (size_t)c->G * c->KM * 2 * real_size(c);
  z.partial = (size_t)(c->G / 32) * 16;
  z.partial2 = (size_t)c->NB * (c->G / 32) * 16;
  return z;
}

// nqs_eloc runs the fused kernel when a register-resident variant covers the model
bool fused_eloc(const nqs_ctx* c, int op) {
  return op == NQS_OP_ELOC && (eloc_fused_supported(c) || eloc_wide_supported(c));
}
bool fused_grad(const nqs_ctx* c, int op) { return op == NQS_OP_GRAD && grad_fused_supported(c); }
// nqs_lanczos_moments forms e2 from the exchange neighbours' E_loc (fused or
// wide kernel) when no register-resident two-hop kernel covers the model
bool composed_moments(const nqs_ctx* c, int op) {
  return op == NQS_OP_MOMENTS && !twohop_reg_supported(c) &&
         (eloc_fused_supported(c) || eloc_wide_supported(c));
}
size_t fused_part_bytes(const nqs_ctx* c) { return (size_t)(c->G / 16) * 6 * 8; }
// nqs_eloc_grad shares the per-image log amplitudes of the wide E_loc kernel
// with the wide gradient kernel (no theta pass of its own)
bool shared_eloc_grad(const nqs_ctx* c) {
  return !eloc_fused_supported(c) && eloc_wide_supported(c) && grad_wide_supported(c) &&
         c->K <= kWideLrawK;
}

size_t chunk_bytes_per_sample(const nqs_ctx* c, int op) {
  const ChunkSizes z = per_sample(c);
  if (fused_eloc(c, op)) return fused_part_bytes(c) + 16;
  if (fused_grad(c, op)) return 0;                 // no workspace
  switch (op) {
    case NQS_OP_LOGPSI: return z.L;
    case NQS_OP_ELOC: return z.L + z.w + z.t + z.partial;
    case NQS_OP_MOMENTS: return z.L + z.w + z.t + z.partial + z.partial2;
    // plus the neighbour row, its log psi and e1, e2
    case NQS_OP_MOMENTS2: return z.L + z.w + z.t + z.partial + z.partial2 + c->N + 48;
    // the wide gradient kernel recomputes tanh(theta): no t buffer
    case NQS_OP_GRAD: return z.L + z.w + (grad_wide_supported(c) ? 16 : z.t);
    // partials, unreduced log amplitudes, weights, two log psi scratch rows
    case NQS_OP_ELOC_GRAD:
      return shared_eloc_grad(c) ? fused_part_bytes(c) + 2 * z.L + z.w + 32 : 0;
    default: return 0;
  }
}

int64_t chunk_of(const nqs_ctx* c, int op, int64_t S) {
  const size_t b = chunk_bytes_per_sample(c, op);
  if (b == 0 || S <= 0) return std::max<int64_t>(S, 1);
  const int64_t ch = (int64_t)std::max<size_t>(1, kChunkBytes / b);
  // the p = 2 moments chunk counts neighbour configurations: at most NB per
  // configuration, and at least one configuration's worth
  if (op == NQS_OP_MOMENTS2) return std::max<int64_t>(std::min<int64_t>(ch, S * c->NB), c->NB);
  return std::min<int64_t>(ch, S);
}

// Carve the workspace: full-S arrays first, then the chunk arrays.
struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* p) : base((char*)p) {}
  void* take(size_t n) {
    void* r = base ? base + off : nullptr;
    off += align_up(n);
    return r;
  }
};

struct Work {
  double* L = nullptr;
  void* w = nullptr;
  void* t = nullptr;
  double* partial = nullptr;
  double* partial2 = nullptr;
  double* e1e2 = nullptr;
  double* logpsi = nullptr;
  double* result = nullptr;
  double* lp = nullptr;            // chunk log psi scratch when the caller wants none
  double* lp2 = nullptr;           // chunk log psi of the weights pass (nqs_eloc_grad)
  double* e3 = nullptr;            // [S] complex (p = 2 moments)
  int8_t* nb_spins = nullptr;      // [chunk][N] neighbour configurations
  double* nb_lp = nullptr;         // [chunk] complex log psi of the neighbours
  double* nb_e1e2 = nullptr;       // [chunk][2] complex e1, e2 of the neighbours
  int32_t* nb_cnt = nullptr;       // [n_out] antiparallel bonds per configuration
  int32_t* nb_off = nullptr;       // [n_out + 1] their exclusive scan
  int16_t* nb_parent = nullptr;    // [chunk] bond exchanged to make each neighbour row
  int64_t n_out = 0;               // configurations per neighbour chunk
  int64_t chunk = 1;
  size_t bytes = 0;
};

Work plan(const nqs_ctx* c, int op, int64_t S, void* ws) {
  Work wk;
  Carve cv(ws);
  const ChunkSizes z = per_sample(c);
  const bool mom = op == NQS_OP_MOMENTS || op == NQS_OP_MOMENTS2;
  if (mom) {
    wk.e1e2 = (double*)cv.take((size_t)std::max<int64_t>(S, 1) * 32);
    wk.logpsi = (double*)cv.take((size_t)std::max<int64_t>(S, 1) * 16);
    wk.result = (double*)cv.take(32 * 8);
  }
  if (op == NQS_OP_MOMENTS2) wk.e3 = (double*)cv.take((size_t)std::max<int64_t>(S, 1) * 16);
  if (composed_moments(c, op)) {
    // chunk = neighbour configurations per E_loc launch (at most NB per configuration)
    const size_t b = fused_part_bytes(c) + c->N + 50;
    int64_t ch = (int64_t)std::max<size_t>(1, kChunkBytes / b);
    ch = std::max<int64_t>(std::min<int64_t>(ch, std::max<int64_t>(S, 1) * c->NB), c->NB);
    wk.chunk = ch;
    wk.n_out = std::max<int64_t>(1, ch / c->NB);
    wk.partial = (double*)cv.take(fused_part_bytes(c) * ch);
    wk.nb_spins = (int8_t*)cv.take((size_t)ch * c->N);
    wk.nb_lp = (double*)cv.take((size_t)ch * 16);
    wk.nb_e1e2 = (double*)cv.take((size_t)ch * 32);
    wk.nb_cnt = (int32_t*)cv.take((size_t)wk.n_out * 4);
    wk.nb_off = (int32_t*)cv.take((size_t)(wk.n_out + 1) * 4);
    wk.nb_parent = (int16_t*)cv.take((size_t)ch * 2);
    wk.bytes = cv.off;
    return wk;
  }
  if (op == NQS_OP_ELOC_GRAD && !shared_eloc_grad(c)) {
    // nqs_eloc, then nqs_grad, in the same workspace
    wk.bytes = std::max(plan(c, NQS_OP_ELOC, S, nullptr).bytes,
                        plan(c, NQS_OP_GRAD, S, nullptr).bytes);
    return wk;
  }
  const int64_t ch = chunk_of(c, op, S);
  wk.chunk = ch;
  if (op == NQS_OP_ELOC_GRAD) {
    wk.partial = (double*)cv.take(fused_part_bytes(c) * ch);
    wk.L = (double*)cv.take(2 * z.L * ch);
    wk.w = cv.take(z.w * ch);
    wk.lp = (double*)cv.take((size_t)16 * ch);
    wk.lp2 = (double*)cv.take((size_t)16 * ch);
    wk.bytes = cv.off;
    return wk;
  }
  if (fused_grad(c, op)) return wk;
  if (fused_eloc(c, op)) {
    wk.partial = (double*)cv.take(fused_part_bytes(c) * ch);
    wk.lp = (double*)cv.take((size_t)16 * ch);
    wk.bytes = cv.off;
    return wk;
  }
  wk.L = (double*)cv.take(z.L * ch);
  if (op != NQS_OP_LOGPSI) {
    wk.w = cv.take(z.w * ch);
    if (!(op == NQS_OP_GRAD && grad_wide_supported(c))) wk.t = cv.take(z.t * ch);
  }
  if (op == NQS_OP_ELOC || mom) wk.partial = (double*)cv.take(z.partial * ch);
  if (op == NQS_OP_ELOC || op == NQS_OP_GRAD) wk.lp = (double*)cv.take((size_t)16 * ch);
  if (mom) wk.partial2 = (double*)cv.take(z.partial2 * ch);
  if (op == NQS_OP_MOMENTS2) {
    wk.n_out = std::max<int64_t>(1, ch / c->NB);
    wk.nb_spins = (int8_t*)cv.take((size_t)ch * c->N);
    wk.nb_lp = (double*)cv.take((size_t)ch * 16);
    wk.nb_e1e2 = (double*)cv.take((size_t)ch * 32);
    wk.nb_cnt = (int32_t*)cv.take((size_t)wk.n_out * 4);
    wk.nb_off = (int32_t*)cv.take((size_t)(wk.n_out + 1) * 4);
  }
  wk.bytes = cv.off;
  return wk;
}

nqs_status check_common(nqs_ctx* c, const int8_t* spins, int64_t S, void* ws, size_t ws_bytes,
                        int op) {
  if (!c) return NQS_ERR_ARG;
  if (S < 0) return fail(c, NQS_ERR_ARG, "S must be >= 0");
  if (S > 0 && !spins) return fail(c, NQS_ERR_ARG, "spins is NULL");
  const size_t need = plan(c, op, S, nullptr).bytes;
  if (S > 0 && need > 0 && (!ws || ws_bytes < need))
    return fail(c, NQS_ERR_ARG, "workspace too small: need " + std::to_string(need) + " bytes");
  return NQS_OK;
}

template <typename T>
nqs_status upload(nqs_ctx* c, T** dst, const std::vector<T>& src) {
  if (hipMalloc((void**)dst, src.size() * sizeof(T)) != hipSuccess)
    return fail(c, NQS_ERR_OOM, "hipMalloc of a geometry table failed");
  if (hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return fail(c, NQS_ERR_DEVICE, "hipMemcpy of a geometry table failed");
  return NQS_OK;
}

// Rebuild the parameter tables and read back whether the reciprocal form of
// the exchange factors is in range for these parameters (synchronous).
hipError_t prep_tables(nqs_ctx* c, hipStream_t st) {
  hipError_t e = hipMemsetAsync(c->par.flag + 1, 0, 8, st);
  if (e == hipSuccess) e = launch_prep(c, st);
  double bad = 1.0;
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, c->par.flag + 1, 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  c->par.recip_ok = e == hipSuccess && bad == 0.0;
  return e;
}

void free_all(nqs_ctx* c) {
  void* ptrs[] = {c->dev.perm, c->dev.perminv, c->dev.bonds, c->dev.bond_J, c->dev.bmap, c->dev.chi,
                  c->dev.fmap, c->dev.frow, c->dev.wmap, c->dev.wrow, c->dev.binom,
                  c->par.params, c->par.wfrag, c->par.wfrag3, c->par.wfrag_s3, c->par.bias, c->par.avec, c->par.Tpm,
                  c->par.F, c->par.Tpair, c->par.Fpair, c->par.Tdir, c->par.Urec, c->par.flag};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
}

}  // namespace

extern "C" {

const char* nqs_status_str(nqs_status s) {
  switch (s) {
    case NQS_OK: return "ok";
    case NQS_ERR_ARG: return "invalid argument";
    case NQS_ERR_DEVICE: return "device error";
    case NQS_ERR_OOM: return "out of device memory";
    case NQS_ERR_NONFINITE: return "non-finite value";
    case NQS_WARN_DEGENERATE: return "degenerate Lanczos step (zero variance)";
    case NQS_ERR_NOT_PD: return "matrix not positive definite";
    case NQS_WARN_NOT_CONVERGED: return "iterative solver stopped above its tolerance";
  }
  return "unknown status";
}

const char* nqs_last_error(const nqs_ctx* c) { return c ? c->last_error.c_str() : "null context"; }

int64_t nqs_num_params(const nqs_ctx* c) { return c ? c->P : -1; }

namespace {
// nqs_vmc_step workspace: E_loc [S], O [S][P], dtheta [P], theta + dtheta [P],
// statistics, then one region shared by the eloc, grad and sr_solve calls.
struct VmcCarve {
  size_t eloc, O, dth, next, stats, sub, bytes;
};
VmcCarve vmc_carve(const nqs_ctx* c, int64_t S) {
  VmcCarve v;
  const size_t osz = c->prec == NQS_FP64 ? 16 : 8;
  size_t off = 0;
  v.eloc = off; off += align_up((size_t)S * 16);
  v.O = off; off += align_up((size_t)S * c->P * osz);
  v.dth = off; off += align_up((size_t)c->P * 16);
  v.next = off; off += align_up((size_t)c->P * 16);
  v.stats = off; off += align_up(8 * 8);
  v.sub = off;
  size_t sub = plan(c, NQS_OP_ELOC_GRAD, S, nullptr).bytes;
  sub = std::max(sub, sr_workspace_bytes(c, S));
  sub = std::max(sub, cg_workspace_bytes(c, S));
  v.bytes = off + align_up(std::max<size_t>(sub, 1));
  return v;
}
size_t vmc_workspace_bytes(const nqs_ctx* c, int64_t S) {
  return vmc_carve(c, std::max<int64_t>(S, 1)).bytes;
}
}  // namespace

size_t nqs_workspace_bytes(const nqs_ctx* c, int op, int64_t S) {
  if (!c || S < 0) return 0;
  if (op == NQS_OP_SR) return sr_workspace_bytes(c, S);
  if (op == NQS_OP_SAMPLE) return sample_workspace_bytes(c, S);
  if (op == NQS_OP_SQ) return sq_workspace_bytes(c, S);
  if (op == NQS_OP_VMC) return vmc_workspace_bytes(c, S);
  if (op == NQS_OP_CG) return cg_workspace_bytes(c, S);
  return plan(c, op, S, nullptr).bytes;
}

nqs_status nqs_create(const nqs_model_desc* d, nqs_ctx** out) {
  if (!d || !out) return NQS_ERR_ARG;
  *out = nullptr;
  nqs_ctx* c = new (std::nothrow) nqs_ctx();
  if (!c) return NQS_ERR_OOM;
  c->d = *d;
  std::string err;
  if (d->n_rbm < 1 || d->n_hidden < 8 || d->n_hidden % 8 != 0 ||
      (int64_t)d->n_rbm * d->n_hidden > kMaxKM || d->precision < 0 || d->precision > 2 ||
      (d->use_bias != 0 && d->use_bias != 1) || !std::isfinite(d->J1) || !std::isfinite(d->J2)) {
    delete c;
    return NQS_ERR_ARG;
  }
  if (!build_geometry(d->L, d->J1, d->J2, d->kx, d->ky, d->irrep, c->geo, err)) {
    delete c;
    return NQS_ERR_ARG;
  }
  c->L = d->L;
  c->N = c->geo.N;
  c->G = c->geo.G;
  c->NB = c->geo.NB;
  c->K = d->n_rbm;
  c->M = d->n_hidden;
  c->KM = c->K * c->M;
  c->P_rbm = c->M * c->N + (d->use_bias ? c->N + c->M : 0);
  c->P = (int64_t)c->K * c->P_rbm;
  c->prec = d->precision;
  c->n_htiles = c->KM / 8;
  c->nk = c->prec == NQS_BF16X2 ? (2 * c->N + 31) / 32 : c->N / 4;
  (void)hipGetDevice(&c->device);
  // the allocation-free entry point's scratch address on this device (if this
  // fails, nqs_eloc_noalloc retries and reports the error)
  (void)noalloc_scratch_init(c->device);
  if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device) !=
      hipSuccess)
    c->n_cu = 256;

  nqs_status st = NQS_OK;
  st = upload(c, &c->dev.perm, c->geo.perm);
  std::vector<uint8_t> inv(c->geo.perm.size());
  for (int g = 0; g < c->G; ++g)
    for (int l = 0; l < c->N; ++l) inv[(size_t)g * c->N + c->geo.perm[(size_t)g * c->N + l]] = l;
  if (st == NQS_OK) st = upload(c, &c->dev.perminv, inv);
  std::vector<int32_t> bonds(2 * c->NB);
  for (int b = 0; b < c->NB; ++b) {
    bonds[2 * b] = c->geo.bond_i[b];
    bonds[2 * b + 1] = c->geo.bond_j[b];
  }
  if (st == NQS_OK) st = upload(c, &c->dev.bonds, bonds);
  if (st == NQS_OK) st = upload(c, &c->dev.bond_J, c->geo.bond_J);
  if (st == NQS_OK) st = upload(c, &c->dev.bmap, c->geo.bmap);
  if (st == NQS_OK) st = upload(c, &c->dev.chi, c->geo.chi);
  {
    std::vector<uint64_t> binom;
    if (nqs::sz0_binomials(c->N, binom, c->sector_count)) {
      if (st == NQS_OK) st = upload(c, &c->dev.binom, binom);
    } else {
      c->sector_count = -1;
    }
  }
  if (st == NQS_OK && eloc_fused_supported(c)) {
    // bank-conflict-free LDS rows for the fused kernel, else plain odd-stride rows
    const int rb = c->prec == NQS_FP64 ? 8 : 4;
    const int row16 = nqs::fused_row16(c->K, c->M, rb);
    std::vector<int> addr = nqs::place_fused_rows(c->geo, row16, nqs::fused_cap16(c->NB, row16));
    if (addr.empty())
      for (int b = 0; b < c->NB; ++b) addr.push_back(b * (row16 | 1));
    std::vector<int32_t> frow(c->NB), fmap((size_t)c->G * c->NB);
    for (int b = 0; b < c->NB; ++b) frow[b] = addr[b] * (16 / rb);
    for (size_t i = 0; i < fmap.size(); ++i)
      fmap[i] = 2 * frow[c->geo.bmap[i] >> 1] + (c->geo.bmap[i] & 1);
    st = upload(c, &c->dev.frow, frow);
    if (st == NQS_OK) st = upload(c, &c->dev.fmap, fmap);
  }
  if (st == NQS_OK && eloc_wide_supported(c)) {
    // wide kernel: chunk rows placed so that 16-image column blocks read
    // (mostly) distinct bank groups
    const int cap = nqs::wide_cap16(c->NB);
    std::vector<int> addr = nqs::place_fused_rows(c->geo, nqs::kWideRow16, cap);
    if (addr.empty())
      for (int b = 0; b < c->NB; ++b) addr.push_back(b * nqs::kWideRow16);
    std::vector<int32_t> wrow(addr.begin(), addr.end()), wmap((size_t)c->G * c->NB);
    for (size_t i = 0; i < wmap.size(); ++i)
      wmap[i] = 2 * (4 * addr[c->geo.bmap[i] >> 1]) + (c->geo.bmap[i] & 1);
    st = upload(c, &c->dev.wrow, wrow);
    if (st == NQS_OK) st = upload(c, &c->dev.wmap, wmap);
  }
  const size_t rs = real_size(c);
  const size_t frag_bytes = (size_t)c->n_htiles * c->nk * 64 * (c->prec == NQS_BF16X2 ? 16 : rs);
  // FP32 models: theta from a three-term BF16 split of W, with the K axis as
  // [W_hi | W_mid | W_lo | 0] (wide E_loc and gradient kernels) and grouped
  // by site (theta kernel, fused E_loc and gradient kernels)
  const size_t frag3_bytes =
      c->prec == NQS_FP32 ? (size_t)c->n_htiles * ((3 * c->N + 31) / 32) * 64 * 16 : 0;
  const size_t frag_s3_bytes = c->prec == NQS_FP32 && c->N % 4 == 0
                                   ? (size_t)c->n_htiles * ((3 * (c->N / 4) + 7) / 8) * 64 * 16
                                   : 0;
  struct {
    void** p;
    size_t n;
  } allocs[] = {{(void**)&c->par.params, (size_t)c->P * 16},
                {&c->par.wfrag, frag_bytes},
                {&c->par.wfrag3, frag3_bytes},
                {&c->par.wfrag_s3, frag_s3_bytes},
                {&c->par.bias, (size_t)c->KM * 2 * rs},
                {&c->par.avec, (size_t)c->K * c->N * 2 * rs},
                {&c->par.Tpm, (size_t)c->NB * 2 * c->KM * 2 * rs},
                {&c->par.F, (size_t)c->K * c->NB * 2 * 2 * rs},
                {&c->par.Tpair, (size_t)c->N * c->N * c->KM * 2 * rs},
                {&c->par.Fpair, (size_t)c->K * c->N * c->N * 2 * rs},
                {&c->par.Tdir, (size_t)c->NB * (2 * c->KM + 18 * c->K) * rs},
                {&c->par.Urec, (size_t)c->NB * (2 * c->KM + 18 * c->K) * rs},
                {(void**)&c->par.flag, 16}};
  for (auto& a : allocs) {
    if (st != NQS_OK) break;
    if (a.n > 0 && hipMalloc(a.p, a.n) != hipSuccess) st = NQS_ERR_OOM;
  }
  if (st == NQS_OK && hipMemset(c->par.params, 0, (size_t)c->P * 16) != hipSuccess)
    st = NQS_ERR_DEVICE;
  if (st == NQS_OK && prep_tables(c, nullptr) != hipSuccess) st = NQS_ERR_DEVICE;
  if (st != NQS_OK) {
    free_all(c);
    delete c;
    return st;
  }
  *out = c;
  return NQS_OK;
}

void nqs_destroy(nqs_ctx* c) {
  if (!c) return;
  for (auto& ev : c->prof.ev)
    for (auto& pr : ev) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  free_all(c);
  delete c;
}

nqs_status nqs_set_params(nqs_ctx* c, const double* params, hipStream_t st) {
  if (!c) return NQS_ERR_ARG;
  if (!params) return fail(c, NQS_ERR_ARG, "params is NULL");
  hipError_t e;
  if ((e = hipMemsetAsync(c->par.flag, 0, 8, st)) != hipSuccess) return hip_fail(c, e, "memset");
  if ((e = launch_check_finite(params, c->P * 2, c->par.flag, st)) != hipSuccess)
    return hip_fail(c, e, "check_finite");
  double flag = 0.0;
  if ((e = hipMemcpyAsync(&flag, c->par.flag, 8, hipMemcpyDeviceToHost, st)) != hipSuccess)
    return hip_fail(c, e, "memcpy");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(c, e, "sync");
  if (flag != 0.0) return fail(c, NQS_ERR_NONFINITE, "parameters contain NaN or Inf");
  if ((e = hipMemcpyAsync(c->par.params, params, (size_t)c->P * 16, hipMemcpyDeviceToDevice, st)) !=
      hipSuccess)
    return hip_fail(c, e, "memcpy params");
  if ((e = prep_tables(c, st)) != hipSuccess) return hip_fail(c, e, "prep");
  return NQS_OK;
}

nqs_status nqs_get_params(nqs_ctx* c, double* params_out, hipStream_t st) {
  if (!c) return NQS_ERR_ARG;
  if (!params_out) return fail(c, NQS_ERR_ARG, "params_out is NULL");
  const hipError_t e = hipMemcpyAsync(params_out, c->par.params, (size_t)c->P * 16,
                                      hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return hip_fail(c, e, "memcpy params");
  return NQS_OK;
}

nqs_status nqs_vmc_step(nqs_ctx* c, const int8_t* spins, int64_t S, double lambda, double dtau,
                        int real_params, int solver, nqs_vmc_stats* out, void* ws,
                        size_t ws_bytes, hipStream_t st) {
  if (!c) return NQS_ERR_ARG;
  if (S < 1 || !spins || !out) return fail(c, NQS_ERR_ARG, "vmc_step: needs S >= 1, spins, out");
  if (solver != 0 && solver != 1) return fail(c, NQS_ERR_ARG, "vmc_step: solver must be 0 or 1");
  const VmcCarve v = vmc_carve(c, S);
  if (!ws || ws_bytes < v.bytes)
    return fail(c, NQS_ERR_ARG, "vmc_step: workspace too small: need " + std::to_string(v.bytes));
  char* base = (char*)ws;
  double* eloc = (double*)(base + v.eloc);
  void* O = base + v.O;
  double* dth = (double*)(base + v.dth);
  double* next = (double*)(base + v.next);
  double* stats = (double*)(base + v.stats);
  void* sub = base + v.sub;
  const size_t sub_bytes = v.bytes - v.sub;
  nqs_status s = nqs_eloc_grad(c, spins, S, nullptr, eloc, O, sub, sub_bytes, st);
  if (s != NQS_OK) return s;
  hipError_t e = launch_energy_stats(eloc, S, stats, st);
  if (e != hipSuccess) return hip_fail(c, e, "energy statistics");
  int iters = 0;
  double resid = 0.0;
  s = solver == 0 ? nqs_sr_solve(c, O, eloc, S, lambda, dtau, dth, sub, sub_bytes, st)
                  : nqs_sr_solve_cg(c, O, eloc, S, lambda, dtau, 1e-8, 2000, dth, &iters, &resid,
                                    sub, sub_bytes, st);
  const bool unconverged = s == NQS_WARN_NOT_CONVERGED;
  if (s != NQS_OK && !unconverged) return s;
  if ((e = launch_params_step(c->par.params, dth, c->P, real_params ? 0 : 1, next, stats, st)) !=
      hipSuccess)
    return hip_fail(c, e, "parameter step");
  double h[5];
  if ((e = hipMemcpyAsync(h, stats, sizeof(h), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return hip_fail(c, e, "memcpy stats");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(c, e, "sync");
  out->n = S;
  out->energy = h[0];
  out->energy_im = h[1];
  out->variance = h[2];
  out->error = std::sqrt(h[2] / (double)S);
  out->dtheta_norm = h[3];
  out->solver_iters = iters;
  out->solver_resid = resid;
  if (h[4] != 0.0) return fail(c, NQS_ERR_NONFINITE, "vmc_step: theta + dtheta is not finite");
  if ((e = hipMemcpyAsync(c->par.params, next, (size_t)c->P * 16, hipMemcpyDeviceToDevice, st)) !=
      hipSuccess)
    return hip_fail(c, e, "memcpy params");
  if ((e = prep_tables(c, st)) != hipSuccess) return hip_fail(c, e, "prep");
  if (unconverged)
    return fail(c, NQS_WARN_NOT_CONVERGED,
                "vmc_step: CG stopped above its tolerance (relative residual " +
                    std::to_string(resid) + "); the update was applied");
  return NQS_OK;
}

nqs_status nqs_structure_factor(nqs_ctx* c, const int8_t* spins, int64_t S, const double* weights,
                                double* out, void* ws, size_t ws_bytes, hipStream_t st) {
  if (!c) return NQS_ERR_ARG;
  if (S < 1) return fail(c, NQS_ERR_ARG, "structure factor needs S >= 1");
  if (!spins || !out) return fail(c, NQS_ERR_ARG, "spins or out is NULL");
  const size_t need = sq_workspace_bytes(c, S);
  if (!ws || ws_bytes < need)
    return fail(c, NQS_ERR_ARG, "workspace too small: need " + std::to_string(need) + " bytes");
  const hipError_t e = NQS_RUN(c, K_SQ, st, launch_sq(c, spins, S, weights, out, ws, st));
  if (e != hipSuccess) return hip_fail(c, e, "structure factor launch");
  return NQS_OK;
}

nqs_status nqs_logpsi(nqs_ctx* c, const int8_t* spins, int64_t S, double* logpsi_out, void* ws,
                      size_t ws_bytes, hipStream_t st) {
  nqs_status s = check_common(c, spins, S, ws, ws_bytes, NQS_OP_LOGPSI);
  if (s != NQS_OK) return s;
  if (S > 0 && !logpsi_out) return fail(c, NQS_ERR_ARG, "logpsi_out is NULL");
  const Work wk = plan(c, NQS_OP_LOGPSI, S, ws);
  for (int64_t s0 = 0; s0 < S; s0 += wk.chunk) {
    const int64_t n = std::min(wk.chunk, S - s0);
    const int8_t* sp = spins + s0 * c->N;
    hipError_t e = NQS_RUN(c, K_THETA, st, launch_theta(c, sp, n, wk.L, nullptr, st));
    if (e == hipSuccess)
      e = NQS_RUN(c, K_LSE, st, launch_lse(c, wk.L, n, logpsi_out + 2 * s0, nullptr, st));
    if (e != hipSuccess) return hip_fail(c, e, "logpsi launch");
  }
  return NQS_OK;
}

namespace {
// log psi and E_loc of n configurations with the fused (K*M <= 128) or wide
// kernel; part holds the per-(configuration, 16-image block) partials.
hipError_t eloc_fused_any(nqs_ctx* c, const int8_t* sp, int64_t n, double* part, double* lp,
                          double* eloc, int eloc_stride, hipStream_t st) {
  if (eloc_fused_supported(c))
    return NQS_RUN(c, K_ELOC, st, launch_eloc_fused(c, sp, n, part, lp, eloc, eloc_stride, st));
  hipError_t e = NQS_RUN(c, K_ELOC, st, launch_eloc_wide(c, sp, n, part, st));
  if (e == hipSuccess)
    e = NQS_RUN(c, K_ELOC_FIN, st, launch_fused_finish(c, sp, n, part, lp, eloc, eloc_stride, st));
  return e;
}

// Neighbour rows of n configurations into wk.nb_spins (bond order; wk.nb_off
// their offsets); *total = their number (reads it back: synchronises).
hipError_t expand_neighbours(nqs_ctx* c, const Work& wk, const int8_t* sp, int64_t n,
                             int32_t* total, hipStream_t st, int16_t* parent = nullptr) {
  *total = 0;
  hipError_t e = NQS_RUN(c, K_HOP3, st, launch_nb_count(c, sp, n, wk.nb_cnt, st));
  if (e == hipSuccess) e = NQS_RUN(c, K_HOP3, st, launch_nb_scan(wk.nb_cnt, n, wk.nb_off, st));
  if (e == hipSuccess) e = hipMemcpyAsync(total, wk.nb_off + n, 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  if (*total < 0 || *total > wk.chunk) return hipErrorInvalidValue;
  if (*total > 0)
    e = NQS_RUN(c, K_HOP3, st,
                parent ? launch_nb_write_parent(c, sp, n, wk.nb_off, wk.nb_spins, parent, st)
                       : launch_nb_write(c, sp, n, wk.nb_off, wk.nb_spins, st));
  return e;
}

// theta (+t) -> LSE (+w) -> bond sums -> E_loc, one chunk.
hipError_t eloc_chunk(nqs_ctx* c, const Work& wk, const int8_t* sp, int64_t n, double* logpsi,
                      double* eloc, int eloc_stride, hipStream_t st) {
  hipError_t e = NQS_RUN(c, K_THETA, st, launch_theta(c, sp, n, wk.L, wk.t, st));
  if (e == hipSuccess) e = NQS_RUN(c, K_LSE, st, launch_lse(c, wk.L, n, logpsi, wk.w, st));
  if (e == hipSuccess)
    e = NQS_RUN(c, K_ELOC, st, launch_eloc_bonds(c, sp, n, wk.t, wk.w, wk.partial, st));
  if (e == hipSuccess)
    e = NQS_RUN(c, K_ELOC_FIN, st,
                launch_eloc_finish(c, sp, n, wk.partial, eloc, eloc_stride, st));
  return e;
}
}  // namespace

nqs_status nqs_eloc(nqs_ctx* c, const int8_t* spins, int64_t S, double* logpsi_out,
                    double* eloc_out, void* ws, size_t ws_bytes, hipStream_t st) {
  nqs_status s = check_common(c, spins, S, ws, ws_bytes, NQS_OP_ELOC);
  if (s != NQS_OK) return s;
  if (S > 0 && !eloc_out) return fail(c, NQS_ERR_ARG, "eloc_out is NULL");
  const Work wk = plan(c, NQS_OP_ELOC, S, ws);
  const bool fused = fused_eloc(c, NQS_OP_ELOC);
  for (int64_t s0 = 0; s0 < S; s0 += wk.chunk) {
    const int64_t n = std::min(wk.chunk, S - s0);
    double* lp = logpsi_out ? logpsi_out + 2 * s0 : wk.lp;
    const int8_t* sp = spins + s0 * c->N;
    hipError_t e;
    if (fused && eloc_fused_supported(c)) {
      e = NQS_RUN(c, K_ELOC, st,
                  launch_eloc_fused(c, sp, n, wk.partial, lp, eloc_out + 2 * s0, 2, st));
    } else if (fused) {
      e = NQS_RUN(c, K_ELOC, st, launch_eloc_wide(c, sp, n, wk.partial, st));
      if (e == hipSuccess)
        e = NQS_RUN(c, K_ELOC_FIN, st,
                    launch_fused_finish(c, sp, n, wk.partial, lp, eloc_out + 2 * s0, 2, st));
    } else {
      e = eloc_chunk(c, wk, sp, n, lp, eloc_out + 2 * s0, 2, st);
    }
    if (e != hipSuccess) return hip_fail(c, e, "eloc launch");
  }
  return NQS_OK;
}

nqs_status nqs_lanczos_moments(nqs_ctx* c, const int8_t* spins, int64_t S, int exact,
                               double* e1e2_out, nqs_moments* out, void* ws, size_t ws_bytes,
                               hipStream_t st) {
  nqs_status s = check_common(c, spins, S, ws, ws_bytes, NQS_OP_MOMENTS);
  if (s != NQS_OK) return s;
  if (!out) return fail(c, NQS_ERR_ARG, "out is NULL");
  if (S <= 0) return fail(c, NQS_ERR_ARG, "moments need S >= 1");
  if (exact != 0 && exact != 1) return fail(c, NQS_ERR_ARG, "exact must be 0 or 1");
  const Work wk = plan(c, NQS_OP_MOMENTS, S, ws);
  hipError_t e = hipSuccess;
  // e2 = H_ss e1 + sum_b (J_b/2) psi(s^b)/psi(s) E_loc(s^b) from the fused / wide kernels
  for (int64_t s0 = 0; composed_moments(c, NQS_OP_MOMENTS) && s0 < S && e == hipSuccess;
       s0 += wk.n_out) {
    const int64_t n = std::min(wk.n_out, S - s0);
    const int8_t* sp = spins + s0 * c->N;
    double* lp = wk.logpsi + 2 * s0;
    double* e12 = wk.e1e2 + 4 * s0;
    // wide models: each neighbour's bond list is its parent's unordered-pair
    // list and the neighbours contribute path sums (no division by their psi)
    const bool pairs = !eloc_fused_supported(c);
    e = eloc_fused_any(c, sp, n, wk.partial, lp, e12, 4, st);
    int32_t total = 0;
    if (e == hipSuccess) e = expand_neighbours(c, wk, sp, n, &total, st, pairs ? wk.nb_parent : nullptr);
    if (e == hipErrorInvalidValue)
      return fail(c, NQS_ERR_DEVICE, "neighbour count " + std::to_string(total) +
                                         " exceeds the chunk " + std::to_string(wk.chunk));
    if (pairs) {
      if (e == hipSuccess && total > 0)
        e = NQS_RUN(c, K_ELOC, st,
                    launch_eloc_wide_pairs(c, wk.nb_spins, total, wk.nb_parent, wk.partial, st));
      if (e == hipSuccess && total > 0)
        e = NQS_RUN(c, K_HOP3, st,
                    launch_pathsum_finish(c, wk.nb_spins, total, wk.partial, wk.nb_lp, st));
      if (e == hipSuccess)
        e = NQS_RUN(c, K_HOP3, st,
                    launch_hop_combine(c, sp, n, wk.nb_off, lp, e12, 4, wk.nb_lp, nullptr, 0,
                                       e12 + 2, 4, st, 1));
    } else {
      if (e == hipSuccess && total > 0)
        e = eloc_fused_any(c, wk.nb_spins, total, wk.partial, wk.nb_lp, wk.nb_e1e2, 4, st);
      if (e == hipSuccess)
        e = NQS_RUN(c, K_HOP3, st,
                    launch_hop_combine(c, sp, n, wk.nb_off, lp, e12, 4, wk.nb_lp, wk.nb_e1e2, 4,
                                       e12 + 2, 4, st));
    }
  }
  for (int64_t s0 = 0; !composed_moments(c, NQS_OP_MOMENTS) && s0 < S && e == hipSuccess;
       s0 += wk.chunk) {
    const int64_t n = std::min(wk.chunk, S - s0);
    const int8_t* sp = spins + s0 * c->N;
    e = eloc_chunk(c, wk, sp, n, wk.logpsi + 2 * s0, wk.e1e2 + 4 * s0, 4, st);
    if (e == hipSuccess)
      e = NQS_RUN(c, K_TWOHOP, st, launch_twohop(c, sp, n, wk.t, wk.w, wk.partial2, st));
    if (e == hipSuccess)
      e = NQS_RUN(c, K_TWOHOP_FIN, st,
                  launch_twohop_finish(c, sp, n, wk.partial2, wk.e1e2 + 4 * s0, st));
  }
  if (e == hipSuccess)
    e = NQS_RUN(c, K_MOMENTS, st,
                launch_moments(wk.e1e2, wk.logpsi, S, exact, nullptr, 0, wk.result, st));
  if (e == hipSuccess && e1e2_out)
    e = hipMemcpyAsync(e1e2_out, wk.e1e2, (size_t)S * 32, hipMemcpyDeviceToDevice, st);
  double r[14];
  if (e == hipSuccess) e = hipMemcpyAsync(r, wk.result, sizeof(r), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(c, e, "moments");
  out->n = (int64_t)r[13];
  out->h1 = r[0];
  out->h1_im = r[1];
  out->h2 = r[2];
  out->h2_alt = r[3];
  out->h3 = r[4];
  out->c2 = r[5];
  out->c3 = r[6];
  out->v = r[7];
  out->r = r[8];
  out->alpha = r[9];
  out->e_p1 = r[10];
  out->h1_err = r[11];
  out->degenerate = r[12] != 0.0;
  for (int j = 0; j < 12; ++j)
    if (!std::isfinite(r[j])) return fail(c, NQS_ERR_NONFINITE, "non-finite moments");
  return out->degenerate ? NQS_WARN_DEGENERATE : NQS_OK;
}

namespace {
// e1 (E_loc) and e2 of n configurations into e1e2 [n][4], log psi into lp.
hipError_t e1e2_chunk(nqs_ctx* c, const Work& wk, const int8_t* sp, int64_t n, double* lp,
                      double* e1e2, hipStream_t st) {
  hipError_t e = eloc_chunk(c, wk, sp, n, lp, e1e2, 4, st);
  if (e == hipSuccess)
    e = NQS_RUN(c, K_TWOHOP, st, launch_twohop(c, sp, n, wk.t, wk.w, wk.partial2, st));
  if (e == hipSuccess)
    e = NQS_RUN(c, K_TWOHOP_FIN, st, launch_twohop_finish(c, sp, n, wk.partial2, e1e2, st));
  return e;
}

void fill_moments(nqs_moments* out, const double* r) {
  out->n = (int64_t)r[13];
  out->h1 = r[0];
  out->h1_im = r[1];
  out->h2 = r[2];
  out->h2_alt = r[3];
  out->h3 = r[4];
  out->c2 = r[5];
  out->c3 = r[6];
  out->v = r[7];
  out->r = r[8];
  out->alpha = r[9];
  out->e_p1 = r[10];
  out->h1_err = r[11];
  out->degenerate = r[12] != 0.0;
}
}  // namespace

nqs_status nqs_lanczos_moments_p2(nqs_ctx* c, const int8_t* spins, int64_t S, int exact,
                                  double* e123_out, nqs_moments2* out, void* ws, size_t ws_bytes,
                                  hipStream_t st) {
  nqs_status s = check_common(c, spins, S, ws, ws_bytes, NQS_OP_MOMENTS2);
  if (s != NQS_OK) return s;
  if (!out) return fail(c, NQS_ERR_ARG, "out is NULL");
  if (S <= 0) return fail(c, NQS_ERR_ARG, "moments need S >= 1");
  if (exact != 0 && exact != 1) return fail(c, NQS_ERR_ARG, "exact must be 0 or 1");
  const Work wk = plan(c, NQS_OP_MOMENTS2, S, ws);
  hipError_t e = hipSuccess;
  // e1, e2 of the configurations
  for (int64_t s0 = 0; s0 < S && e == hipSuccess; s0 += wk.chunk) {
    const int64_t n = std::min(wk.chunk, S - s0);
    e = e1e2_chunk(c, wk, spins + s0 * c->N, n, wk.logpsi + 2 * s0, wk.e1e2 + 4 * s0, st);
  }
  // e3 from the neighbours' log psi and e2, n_out configurations at a time
  for (int64_t s0 = 0; s0 < S && e == hipSuccess; s0 += wk.n_out) {
    const int64_t n = std::min(wk.n_out, S - s0);
    const int8_t* sp = spins + s0 * c->N;
    int32_t total = 0;
    e = expand_neighbours(c, wk, sp, n, &total, st);
    if (e == hipErrorInvalidValue)
      return fail(c, NQS_ERR_DEVICE, "neighbour count " + std::to_string(total) +
                                         " exceeds the chunk " + std::to_string(wk.chunk));
    if (e == hipSuccess && total > 0)
      e = e1e2_chunk(c, wk, wk.nb_spins, total, wk.nb_lp, wk.nb_e1e2, st);
    if (e == hipSuccess)
      e = NQS_RUN(c, K_HOP3, st,
                  launch_e3_combine(c, sp, n, wk.nb_off, wk.logpsi + 2 * s0, wk.e1e2 + 4 * s0,
                                    wk.nb_lp, wk.nb_e1e2, wk.e3 + 2 * s0, st));
  }
  if (e == hipSuccess)
    e = NQS_RUN(c, K_MOMENTS, st,
                launch_moments(wk.e1e2, wk.logpsi, S, exact, nullptr, 0, wk.result, st));
  if (e == hipSuccess)
    e = NQS_RUN(c, K_HOP3, st, launch_moments2(wk.e1e2, wk.e3, wk.logpsi, S, exact, wk.result, st));
  if (e == hipSuccess && e123_out) {
    e = hipMemcpy2DAsync(e123_out, 48, wk.e1e2, 32, 32, (size_t)S, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpy2DAsync((char*)e123_out + 32, 48, wk.e3, 16, 16, (size_t)S,
                           hipMemcpyDeviceToDevice, st);
  }
  double r[24];
  if (e == hipSuccess) e = hipMemcpyAsync(r, wk.result, sizeof(r), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(c, e, "p = 2 moments");
  fill_moments(&out->p1, r);
  out->h4 = r[16];
  out->h5 = r[17];
  out->mu4 = r[18];
  out->mu5 = r[19];
  out->e_p2 = r[20];
  out->beta1 = r[21];
  out->beta2 = r[22];
  out->degenerate = r[23] != 0.0;
  for (int j = 0; j < 23; ++j)
    if ((j < 12 || j >= 16) && !std::isfinite(r[j]))
      return fail(c, NQS_ERR_NONFINITE, "non-finite moments");
  return out->degenerate ? NQS_WARN_DEGENERATE : NQS_OK;
}

nqs_status nqs_grad(nqs_ctx* c, const int8_t* spins, int64_t S, void* O_out, double* logpsi_out,
                    void* ws, size_t ws_bytes, hipStream_t st) {
  nqs_status s = check_common(c, spins, S, ws, ws_bytes, NQS_OP_GRAD);
  if (s != NQS_OK) return s;
  if (S > 0 && !O_out) return fail(c, NQS_ERR_ARG, "O_out is NULL");
  if (fused_grad(c, NQS_OP_GRAD)) {
    const hipError_t e =
        NQS_RUN(c, K_GRAD, st, launch_grad_fused(c, spins, S, O_out, logpsi_out, st));
    return e == hipSuccess ? NQS_OK : hip_fail(c, e, "grad launch");
  }
  const Work wk = plan(c, NQS_OP_GRAD, S, ws);
  const size_t osz = (size_t)c->P * 2 * real_size(c);
  for (int64_t s0 = 0; s0 < S; s0 += wk.chunk) {
    const int64_t n = std::min(wk.chunk, S - s0);
    const int8_t* sp = spins + s0 * c->N;
    double* lp = logpsi_out ? logpsi_out + 2 * s0 : wk.lp;
    // wide models: theta keeps only the per-image log amplitudes (no tanh in
    // HBM); the gradient kernel recomputes theta
    const bool wide = grad_wide_supported(c);
    hipError_t e = NQS_RUN(c, K_THETA, st, launch_theta(c, sp, n, wk.L, wide ? nullptr : wk.t, st));
    if (e == hipSuccess) e = NQS_RUN(c, K_LSE, st, launch_lse(c, wk.L, n, lp, wk.w, st));
    if (e == hipSuccess)
      e = NQS_RUN(c, K_GRAD, st,
                  wide ? launch_grad_wide(c, sp, n, wk.w, (char*)O_out + (size_t)s0 * osz, st)
                       : launch_grad(c, sp, n, wk.t, wk.w, (char*)O_out + (size_t)s0 * osz, st));
    if (e != hipSuccess) return hip_fail(c, e, "grad launch");
  }
  return NQS_OK;
}

nqs_status nqs_eloc_grad(nqs_ctx* c, const int8_t* spins, int64_t S, double* logpsi_out,
                         double* eloc_out, void* O_out, void* ws, size_t ws_bytes,
                         hipStream_t st) {
  nqs_status s = check_common(c, spins, S, ws, ws_bytes, NQS_OP_ELOC_GRAD);
  if (s != NQS_OK) return s;
  if (S > 0 && (!eloc_out || !O_out)) return fail(c, NQS_ERR_ARG, "eloc_out or O_out is NULL");
  if (!shared_eloc_grad(c)) {
    s = nqs_eloc(c, spins, S, logpsi_out, eloc_out, ws, ws_bytes, st);
    return s == NQS_OK ? nqs_grad(c, spins, S, O_out, nullptr, ws, ws_bytes, st) : s;
  }
  const Work wk = plan(c, NQS_OP_ELOC_GRAD, S, ws);
  const size_t osz = (size_t)c->P * 2 * real_size(c);
  for (int64_t s0 = 0; s0 < S; s0 += wk.chunk) {
    const int64_t n = std::min(wk.chunk, S - s0);
    const int8_t* sp = spins + s0 * c->N;
    double* lp = logpsi_out ? logpsi_out + 2 * s0 : wk.lp;
    // E_loc and log psi, the image log amplitudes kept; then the weights and
    // O_k from them
    hipError_t e = NQS_RUN(c, K_ELOC, st, launch_eloc_wide(c, sp, n, wk.partial, st, wk.L));
    if (e == hipSuccess)
      e = NQS_RUN(c, K_ELOC_FIN, st,
                  launch_fused_finish(c, sp, n, wk.partial, lp, eloc_out + 2 * s0, 2, st));
    if (e == hipSuccess)
      e = NQS_RUN(c, K_LSE, st, launch_lse(c, wk.L, n, wk.lp2, wk.w, st, true));
    if (e == hipSuccess)
      e = NQS_RUN(c, K_GRAD, st,
                  launch_grad_wide(c, sp, n, wk.w, (char*)O_out + (size_t)s0 * osz, st));
    if (e != hipSuccess) return hip_fail(c, e, "eloc_grad launch");
  }
  return NQS_OK;
}

nqs_status nqs_enumerate_sz0(nqs_ctx* c, int8_t* spins_out, int64_t cap, int64_t* count,
                             hipStream_t st) {
  if (!c) return NQS_ERR_ARG;
  if (!count) return fail(c, NQS_ERR_ARG, "enumerate_sz0: count is NULL");
  if (c->sector_count < 0) return fail(c, NQS_ERR_ARG, "enumerate_sz0: sector size overflows int64");
  *count = c->sector_count;
  if (!spins_out) return NQS_OK;
  if (c->sector_count > (int64_t)1 << 31)
    return fail(c, NQS_ERR_ARG, "enumerate_sz0: more than 2^31 configurations");
  if (cap < c->sector_count)
    return fail(c, NQS_ERR_ARG, "enumerate_sz0: cap " + std::to_string(cap) + " < " +
                                    std::to_string(c->sector_count));
  const hipError_t e = launch_enum_sz0(c, c->sector_count, spins_out, st);
  return e == hipSuccess ? NQS_OK : hip_fail(c, e, "enumerate_sz0 launch");
}

nqs_status nqs_set_factor_form(nqs_ctx* c, int direct_only) {
  if (!c) return NQS_ERR_ARG;
  if (direct_only != 0 && direct_only != 1)
    return fail(c, NQS_ERR_ARG, "set_factor_form: direct_only must be 0 or 1");
  c->direct_only = direct_only == 1;
  return NQS_OK;
}

nqs_status nqs_profile_enable(nqs_ctx* c, int on) {
  if (!c) return NQS_ERR_ARG;
  c->prof.on = on != 0;
  return NQS_OK;
}

nqs_status nqs_profile_read(nqs_ctx* c, int kernel, double* ms_out, int64_t* launches_out,
                            int reset) {
  if (!c || kernel < 0 || kernel >= K_COUNT) return NQS_ERR_ARG;
  auto& ev = c->prof.ev[kernel];
  for (auto& pr : ev) {
    float ms = 0.f;
    if (hipEventSynchronize(pr.second) != hipSuccess ||
        hipEventElapsedTime(&ms, pr.first, pr.second) != hipSuccess)
      return fail(c, NQS_ERR_DEVICE, "profile event");
    c->prof.ms[kernel] += ms;
    c->prof.n[kernel] += 1;
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  ev.clear();
  if (ms_out) *ms_out = c->prof.ms[kernel];
  if (launches_out) *launches_out = c->prof.n[kernel];
  if (reset) {
    c->prof.ms[kernel] = 0.0;
    c->prof.n[kernel] = 0;
  }
  return NQS_OK;
}

}  // extern "C"
