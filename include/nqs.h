/*
 * nqs.h -- C ABI of the MI355X (gfx950) hot path for symmetry-projected RBM
 * wave functions of the J1-J2 Heisenberg model with a p = 1 Lanczos step
 * (arXiv:2206.14307, "Systematic improvement of neural network quantum
 * states using a Lanczos recursion").
 *
 * Model (Sec. 2.1, Eq. (1)): H = J1 sum_<ij> S_i.S_j + J2 sum_<<ij>> S_i.S_j on
 * the L x L torus, Sz = 0 sector.  Ansatz (Sec. 3.1, Eqs. (2), (6)):
 *   psi(sigma) = sum_{k<K} sum_{g in G} chi(g) psi_s^(k)(g sigma),
 *   psi_s^(k)(x) = exp(sum_j a_j x_j) prod_{h<M} 2 cosh(sum_j W_hj x_j + b_h),
 * G = translations x C4v (8N elements), (g sigma)[i] = sigma[perm_g(i)],
 * perm_g(i) = site(p . r_i + t) for g = (t, p), rotations about site 0,
 * chi(g) = exp(-i K.t) chi_I(p) for K in {(0,0), (pi,pi)} and a 1-D irrep I.
 *
 * Conventions shared by every entry point
 *  - Spins: int8 +1 / -1 encodes sigma = +1/2 / -1/2, row-major [S][N],
 *    site i = x + L*y; rows are taken to hold exactly N/2 entries +1 (the
 *    Sz = 0 sector).  Other rows are not rejected by the evaluation calls:
 *    their results are meaningless, but no access leaves its buffer.
 *  - Complex values are interleaved (re, im) pairs of double unless a
 *    dtype is stated otherwise.
 *  - Ownership: the caller allocates every input, output and workspace
 *    buffer (device memory unless stated); the context owns only its
 *    constant tables and a copy of the parameters.  No entry point
 *    allocates device memory except nqs_create and nqs_set_params.
 *  - Streams: work is enqueued on the given stream and returns without
 *    waiting, except where an entry point says it synchronises.
 *  - Errors: arguments are validated before anything is launched; on an
 *    error nothing is launched and outputs are untouched.  No exception
 *    crosses the ABI.  nqs_last_error() returns a message for the last
 *    failing call on that context.
 *  - Concurrency: calls on one context may be issued from one host thread
 *    at a time; calls that share a workspace must be ordered on one stream.
 */
#ifndef NQS_H
#define NQS_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NQS_OK = 0,
    NQS_ERR_ARG = 1,          /* invalid argument or workspace too small; nothing launched */
    NQS_ERR_DEVICE = 2,       /* a HIP runtime call failed */
    NQS_ERR_OOM = 3,          /* the context could not allocate its tables */
    NQS_ERR_NONFINITE = 4,    /* non-finite parameters or non-finite moments */
    NQS_WARN_DEGENERATE = 5,  /* Lanczos: zero variance (eigenstate); e_p1 = h1, alpha = 0 */
    NQS_ERR_NOT_PD = 6,       /* SR: the Gram matrix is not positive definite */
    NQS_WARN_NOT_CONVERGED = 7 /* CG stopped at max_iter above tol; the result is the last iterate */
} nqs_status;

typedef enum {
    NQS_FP64 = 0,    /* everything in FP64 (theta GEMM on FP64 MFMA) */
    NQS_FP32 = 1,    /* FP32 arithmetic; the theta GEMM and the gradient contraction
                        have FP32 numerics (exact products, FP32 accumulation) and run
                        on BF16 MFMA from an exact three-term BF16 split of the FP32
                        operand where that is faster (x = +-1/2 is exact in BF16),
                        else on FP32 MFMA */
    NQS_BF16X2 = 2   /* theta GEMM on BF16 MFMA with W split into hi + lo BF16 parts,
                        FP32 accumulation; everything else as NQS_FP32 */
} nqs_precision;

typedef enum {
    NQS_OP_LOGPSI = 0, NQS_OP_ELOC = 1, NQS_OP_MOMENTS = 2,
    NQS_OP_GRAD = 3, NQS_OP_SR = 4, NQS_OP_SAMPLE = 5, NQS_OP_SQ = 6, NQS_OP_VMC = 7,
    NQS_OP_CG = 8, NQS_OP_MOMENTS2 = 9, NQS_OP_ELOC_GRAD = 10
} nqs_op;

typedef struct {
    int32_t L;          /* linear size: 4, 6, 8 or 10 (N = L*L sites) */
    double J1, J2;      /* couplings of Eq. (1) */
    int32_t kx, ky;     /* momentum K = 2 pi (kx, ky) / L: (0,0) or (L/2, L/2) */
    int32_t irrep;      /* C4v irrep: 0 A1, 1 A2, 2 B1, 3 B2 (1-D only) */
    int32_t n_rbm;      /* K >= 1: RBMs summed in the linear combination */
    int32_t n_hidden;   /* M per RBM, a multiple of 8, K*M <= 4096 */
    int32_t use_bias;   /* 1: per-RBM parameters [W | a | b]; 0: [W] (bias-free psi_s) */
    int32_t precision;  /* nqs_precision */
} nqs_model_desc;

/* Moments and p = 1 Lanczos energy (Sec. 3.3, Eqs. (13)-(18)).  All FP64.
 * h1 = Re<e1>, h2 = <|e1|^2>, h2_alt = Re<e2>, h3 = Re<conj(e1) e2>,
 * c2 = <|e1-h1|^2>, c3 = Re<conj(e1-h1)(e2 - 2 h1 e1 + h1^2)>,
 * v = sqrt(c2), r = c3 / v^3, alpha = r/2 - sqrt(r^2/4 + 1) (the printed
 * alpha = r - sqrt(r^2+1) lacks the 1/2 of the 2x2 matrix h1 I + v[[0,1],[1,r]]),
 * e_p1 = h1 + v alpha.  h1_err = sqrt(c2 / n) (naive standard error). */
typedef struct {
    int64_t n;
    double h1, h1_im, h2, h2_alt, h3, c2, c3, v, r, alpha, e_p1, h1_err;
    int32_t degenerate;
} nqs_moments;

/* Moments to fifth order and the p = 2 Lanczos energy (Sec. 3.3, Eq. (19)
 * with p = 2).  All FP64.  With d1 = e1 - h1, d2 = e2 - 2 h1 e1 + h1^2,
 * d3 = e3 - 3 h1 e2 + 3 h1^2 e1 - h1^3: h4 = <|e2|^2>, h5 = Re<conj(e2) e3>,
 * mu4 = <|d2|^2>, mu5 = Re<conj(d2) d3>.  e_p2 is the lowest eigenvalue of H
 * in span{psi, H psi, H^2 psi}: the generalised 3x3 Hankel problem
 * A_ij = mu_{i+j+1}/v^{i+j}, B_ij = mu_{i+j}/v^{i+j} (mu_0 = 1, mu_1 = 0,
 * mu_2 = c2, mu_3 = c3), E = h1 + v lambda_min.  Psi_2 = (1 + beta1 H +
 * beta2 H^2) psi is its eigenvector.  degenerate: the scaled Gram determinant
 * mu4/v^4 - r^2 - 1 is <= 64 eps max(mu4/v^4, 1) (Krylov dimension 2, or a
 * Monte-Carlo Hankel matrix that is not positive definite) or the p = 1 step
 * is degenerate: then e_p2 = e_p1, beta2 = 0 (and beta1 is the p = 1 one). */
typedef struct {
    nqs_moments p1;             /* as returned by nqs_lanczos_moments */
    double h4, h5, mu4, mu5;
    double e_p2, beta1, beta2;
    int32_t degenerate;
} nqs_moments2;

/* Statistics of one training step (nqs_vmc_step), all FP64. */
typedef struct {
    int64_t n;                  /* configurations */
    double energy, energy_im;   /* <E_loc>, for the parameters before the update */
    double variance;            /* <|E_loc - <E_loc>|^2> */
    double error;               /* sqrt(variance / n) (no autocorrelation correction) */
    double dtheta_norm;         /* ||dtheta||_2 of the applied update */
    int32_t solver_iters;       /* CG iterations (solver 1), 0 for solver 0 */
    double solver_resid;        /* CG relative residual (solver 1), 0 for solver 0 */
} nqs_vmc_stats;

typedef struct nqs_ctx nqs_ctx;

/* Create a context for one model: builds the lattice, bond and space-group
 * tables (Sec. 3.1) on the current HIP device.  Parameters start at zero.
 * Returns NQS_ERR_ARG for an unsupported description. */
nqs_status nqs_create(const nqs_model_desc* desc, nqs_ctx** out);
void nqs_destroy(nqs_ctx* ctx);

/* Number of complex parameters P = K * (M N + use_bias (N + M)). */
int64_t nqs_num_params(const nqs_ctx* ctx);

/* Bytes of workspace entry point `op` needs for S samples (S = n_chains for
 * NQS_OP_SAMPLE).  Large S is processed in chunks, so the size saturates. */
size_t nqs_workspace_bytes(const nqs_ctx* ctx, int op, int64_t S);

/* Upload parameters: params_dev is device memory holding P complex values
 * (double re, im) in the layout [K][W (M x N, row-major) | a (N) | b (M)].
 * Derives the precision-specific copies and the per-bond tables
 * (tanh and cosh of W_hp - W_hq, Sec. 3.1 applied to bond exchanges).
 * Synchronises the stream.  NQS_ERR_NONFINITE if any value is NaN/Inf. */
nqs_status nqs_set_params(nqs_ctx* ctx, const double* params_dev, hipStream_t stream);

/* log psi(sigma) of Eq. (6) for S configurations: logpsi_out complex [S]
 * (Im in (-pi, pi]).  Workspace: nqs_workspace_bytes(NQS_OP_LOGPSI, S). */
nqs_status nqs_logpsi(nqs_ctx* ctx, const int8_t* spins, int64_t S, double* logpsi_out,
                      void* ws, size_t ws_bytes, hipStream_t stream);

/* Local energies E_loc(sigma) = <sigma|H|psi>/<sigma|psi> (Sec. 3.2, Eq. (10))
 * over the antiparallel J1 and J2 bonds: eloc_out complex [S]; logpsi_out
 * (complex [S]) is written too unless NULL.  Configurations with psi = 0
 * (possible for non-A1 irreps) give non-finite E_loc. */
nqs_status nqs_eloc(nqs_ctx* ctx, const int8_t* spins, int64_t S, double* logpsi_out,
                    double* eloc_out, void* ws, size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid allocation): nqs_eloc without
 * a workspace.  Same results as nqs_eloc (the same kernels); eloc_out and
 * logpsi_out (optional) as there.  The kernels' per-configuration partials,
 * (N/2) x 6 doubles each, live in a 64 MiB device array that the library
 * holds on each GPU it runs on until the process ends, so S is limited to
 * floor(2^26 / (24 N)) configurations (174762 at 4x4, 77672 at 6x6, 43690 at
 * 8x8, 27962 at 10x10): larger S returns NQS_ERR_ARG with nothing launched.
 * Only models with a fused (K*M <= 128) or wide (K*M > 128, FP32 or
 * split-BF16 theta) E_loc kernel are served; others return NQS_ERR_ARG.  The
 * context's device must be current.  Allocates nothing, clears nothing (every
 * partial read is written earlier in the same call) and is asynchronous on
 * the stream.  Calls that overlap on one GPU (other streams or threads) share
 * the array and race: order them on one stream. */
nqs_status nqs_eloc_noalloc(nqs_ctx* ctx, const int8_t* spins, int64_t S, double* logpsi_out,
                            double* eloc_out, hipStream_t stream);

/* e1 = E_loc and e2 = (H^2 psi)/psi per configuration (two-hop connected
 * configurations), then the FP64 moments and p = 1 Lanczos energy
 * (Sec. 3.3).  For models without the register-resident two-hop kernel
 * (K > 1, or K*M beyond its compiled sizes) e2 is formed as
 * H_ss e1 + sum_b (J_b/2) psi(s^b)/psi(s) E_loc(s^b) from the fused / wide
 * E_loc kernels run on the exchange neighbours (the wide kernel on each
 * neighbour's unordered-pair second-hop list, as path sums, with the
 * exchanges there and back added in closed form), which synchronises once
 * per chunk of configurations.  exact = 0: uniform weights (Monte-Carlo samples);
 * exact = 1: Born weights |psi|^2 / sum |psi|^2 (Sec. 3.2, Eq. (9)) over the
 * given configurations (the whole Sz = 0 sector for exact results).
 * e1e2_out (complex [S][2]) is optional.  Writes *out and synchronises the
 * stream.  NQS_WARN_DEGENERATE when c2 <= (8 eps max(|h1|,1))^2. */
nqs_status nqs_lanczos_moments(nqs_ctx* ctx, const int8_t* spins, int64_t S, int exact,
                               double* e1e2_out, nqs_moments* out, void* ws, size_t ws_bytes,
                               hipStream_t stream);

/* e1, e2 and e3 = (H^3 psi)/psi per configuration, then the moments of
 * nqs_moments2 and the p = 2 Lanczos energy (Sec. 3.3, Eq. (19) with p = 2).
 * e3(s) = H_ss e2(s) + sum_b (J_b/2) psi(s^b)/psi(s) e2(s^b): the antiparallel
 * neighbours s^b of each configuration (bond order) are written to the
 * workspace and run through the same logpsi / E_loc / two-hop kernels as the
 * configurations themselves, so the cost is about n_c times that of
 * nqs_lanczos_moments.  exact as for nqs_lanczos_moments.  e123_out (complex
 * [S][3]: e1, e2, e3) is optional.  Workspace:
 * nqs_workspace_bytes(NQS_OP_MOMENTS2, S).  Synchronises the stream (once per
 * chunk of configurations, to size the neighbour launches).  Returns
 * NQS_WARN_DEGENERATE when the p = 2 step is degenerate (see nqs_moments2);
 * NQS_ERR_NONFINITE when a moment is not finite. */
nqs_status nqs_lanczos_moments_p2(nqs_ctx* ctx, const int8_t* spins, int64_t S, int exact,
                                  double* e123_out, nqs_moments2* out, void* ws, size_t ws_bytes,
                                  hipStream_t stream);

/* Log-derivatives O_k = d log psi / d theta_k (Sec. 3.2, below Eq. (12)) for
 * every parameter in the nqs_set_params layout, summed over symmetry images:
 * O_out [S][P] complex, in complex128 for NQS_FP64 and complex64
 * (float re, im) otherwise.  logpsi_out (complex [S]) optional. */
nqs_status nqs_grad(nqs_ctx* ctx, const int8_t* spins, int64_t S, void* O_out, double* logpsi_out,
                    void* ws, size_t ws_bytes, hipStream_t stream);

/* log psi, E_loc and O_k of the same configurations in one call: the outputs of
 * nqs_eloc (logpsi_out optional, eloc_out) and of nqs_grad (O_out), as one
 * VMC step needs them (Sec. 3.2: Eq. (10) and the O_k below Eq. (12)).  For
 * models on the wide E_loc and gradient kernels (K*M > 128) the gradient
 * takes the per-image log amplitudes of psi_s(g sigma) from the E_loc pass
 * instead of a theta pass of its own; other models run nqs_eloc, then
 * nqs_grad.  Results agree with the two separate calls to rounding.
 * Workspace: nqs_workspace_bytes(NQS_OP_ELOC_GRAD, S). */
nqs_status nqs_eloc_grad(nqs_ctx* ctx, const int8_t* spins, int64_t S, double* logpsi_out,
                         double* eloc_out, void* O_out, void* ws, size_t ws_bytes,
                         hipStream_t stream);

/* Stochastic-reconfiguration step of Eq. (12) with ridge lambda (Sec. 3.4),
 * solved in sample space: O_bar = (O - <O>)/sqrt(S), eps = (E_loc - <E>)/sqrt(S),
 * T = O_bar O_bar^H + lambda I (S x S, FP32 MFMA products, FP64 result),
 * FP64 Cholesky T = L L^H, x = T^{-1} eps, dtheta = -dtau O_bar^H x.
 * O: [S][P] as written by nqs_grad; eloc: complex [S]; dtheta_out complex [P].
 * Synchronises the stream; NQS_ERR_NOT_PD if the factorisation fails. */
nqs_status nqs_sr_solve(nqs_ctx* ctx, const void* O, const double* eloc, int64_t S, double lambda,
                        double dtau, double* dtheta_out, void* ws, size_t ws_bytes,
                        hipStream_t stream);

/* The same step of Eq. (12) solved in parameter space by conjugate gradients
 * (Sec. 3.4: CG with the ridge lambda), matrix-free: A v = O_bar^H (O_bar v)
 * + lambda v and b = -dtau O_bar^H eps with O_bar and eps as in
 * nqs_sr_solve, centred on the fly (neither O_bar nor the P x P matrix is
 * formed; each iteration reads O twice).  Starts from dtheta = 0 and stops
 * when ||r|| <= tol ||b|| or after max_iter iterations.  O, eloc and
 * dtheta_out as in nqs_sr_solve; iters_out and resid_out (host, optional)
 * receive the iteration count and ||r|| / ||b||.  Workspace:
 * nqs_workspace_bytes(NQS_OP_CG, S).  Synchronises the stream: iterations
 * are queued four at a time and the residual is read once per four (a
 * device-side flag ends the queued ones after the stop, so the iterates and
 * the count equal a test after every iteration).  NQS_ERR_NOT_PD if
 * p^H A p <= 0; NQS_WARN_NOT_CONVERGED (dtheta_out holds the last iterate)
 * if ||r|| > tol ||b|| after max_iter iterations. */
nqs_status nqs_sr_solve_cg(nqs_ctx* ctx, const void* O, const double* eloc, int64_t S,
                           double lambda, double dtau, double tol, int max_iter,
                           double* dtheta_out, int* iters_out, double* resid_out, void* ws,
                           size_t ws_bytes, hipStream_t stream);

/* The Sz = 0 sector, i.e. all configurations with N/2 up spins (the exact
 * evaluations of Sec. 3.3 run over it on the 4x4 lattice), in colex order of
 * the up-site sets = increasing bit mask sum_{i up} 2^i: row r of
 * spins_out [count][N] int8 (+1 up, -1 down) is the r-th configuration.
 * count (host pointer, required) receives C(N, N/2).  With spins_out = NULL
 * only the count is returned.  NQS_ERR_ARG if cap < count, or if the sector
 * has more than 2^31 configurations (L >= 6; the count is still returned
 * when it fits in int64, i.e. up to L = 8).  Asynchronous on the stream. */
nqs_status nqs_enumerate_sz0(nqs_ctx* ctx, int8_t* spins_out, int64_t cap, int64_t* count,
                             hipStream_t stream);

/* Spin structure factor (Sec. 4, the equation defining S(q), with
 * sigma^z = +-1/2): for every momentum q = 2 pi (kx, ky) / L of the lattice,
 * out[kx + L ky] = sum_s w_s |sum_i sigma_i e^{i q.r_i}|^2 / (N^2 sum_s w_s),
 * the weighted mean over the configurations of the per-configuration
 * (1/N^2) sum_{i,j} sigma_i sigma_j e^{i q.(r_i - r_j)}.  The paper's tables
 * show N S(q).  spins: device int8 [S][N]; weights: device FP64 [S],
 * non-negative (e.g. |psi|^2 for an exact sum over the Sz = 0 sector), or
 * NULL for uniform weights (Monte-Carlo samples); out: device FP64 [N].
 * Workspace: nqs_workspace_bytes(NQS_OP_SQ, S) bytes (per-block partial sums).
 * NQS_ERR_ARG if S < 1 or a pointer is NULL; a zero weight sum gives NaN.
 * Asynchronous on the stream; the result does not depend on the grid (the
 * partial sums are added in a fixed order). */
nqs_status nqs_structure_factor(nqs_ctx* ctx, const int8_t* spins, int64_t S,
                                const double* weights, double* out, void* ws, size_t ws_bytes,
                                hipStream_t stream);

/* Copy the context's current parameters (P complex values, double re, im, in
 * the nqs_set_params layout) to params_out_dev (device memory).  Asynchronous. */
nqs_status nqs_get_params(nqs_ctx* ctx, double* params_out_dev, hipStream_t stream);

/* One stochastic-reconfiguration training step (Sec. 3.2: Eq. (12) and the
 * update theta <- theta + dtheta after it) on S configurations, e.g. from
 * nqs_sample: E_loc (nqs_eloc), their FP64 statistics, O_k (nqs_grad),
 * dtheta from nqs_sr_solve (solver = 0: sample space, Cholesky) or from
 * nqs_sr_solve_cg (solver = 1: parameter-space CG as in Sec. 3.4, relative
 * residual 1e-8, at most 2000 iterations); the context's parameters become
 * theta + dtheta (the imaginary part of dtheta is dropped when
 * real_params = 1, for real RBMs) and the tables are rebuilt.  *out
 * describes the parameters before the update.  Workspace:
 * nqs_workspace_bytes(NQS_OP_VMC, S).  Synchronises the stream.  Errors are
 * those of the three calls; NQS_ERR_NONFINITE (parameters unchanged) if
 * theta + dtheta is not finite.  NQS_WARN_NOT_CONVERGED when CG stopped
 * above its tolerance: the update from its last iterate is still applied
 * and out->solver_resid says how far it got. */
nqs_status nqs_vmc_step(nqs_ctx* ctx, const int8_t* spins, int64_t S, double lambda, double dtau,
                        int real_params, int solver, nqs_vmc_stats* out, void* ws,
                        size_t ws_bytes, hipStream_t stream);

/* Pack initial configurations into chain states: chain_state [n][4] uint64
 * = {spin bits 0..63, spin bits 64..127, proposal counter = 0, chain id}
 * with chain ids first_chain_id + c.  spins: [n][N] int8 (Sz = 0). */
nqs_status nqs_chain_init(nqs_ctx* ctx, const int8_t* spins, int64_t n_chains,
                          uint64_t first_chain_id, uint64_t* chain_state, hipStream_t stream);

/* Exchange Metropolis (Sec. 3.2): proposal n of a chain draws
 * Philox4x64-10(counter (n,0,0,0), key (seed, chain id)) -> (r0, r1, r2, r3);
 * the k-th up site (k = (r0>>11)*(N/2) >> 53) is exchanged with the k'-th
 * down site (from r1); accept iff (r2>>11)*2^-53 < |psi'/psi|^2.  Runs n_burn
 * proposals, then n_per_chain times: n_skip proposals and one kept sample.
 * n_skip = 0 selects N_skip = max(1, ceil(5 P / A)) (capped at 1000) from the
 * A accepted out of P burn-in proposals of all chains (Sec. 3.4, N_skip = 5/r).
 * chain_state [n_chains][4] is read and updated; spins_out [n_chains*n_per_chain][N]
 * (chain-major); acc_rate_out [n_chains] float (sampling phase; NaN for a
 * chain whose state is not in the Sz = 0 sector, which is left unchanged);
 * n_skip_out (device int32, optional) receives the N_skip used.  The chain
 * caches live in the workspace (nqs_workspace_bytes(NQS_OP_SAMPLE, n_chains))
 * and are rebuilt from the spins every 256 proposals.  Synchronises the
 * stream once when n_skip = 0 (to size the sampling phase). */
nqs_status nqs_sample(nqs_ctx* ctx, int64_t n_chains, int64_t n_per_chain, int32_t n_skip,
                      int32_t n_burn, uint64_t seed, uint64_t* chain_state, int8_t* spins_out,
                      float* acc_rate_out, int32_t* n_skip_out, void* ws, size_t ws_bytes,
                      hipStream_t stream);

/* Arithmetic form of the exchange factors (Sec. 3.2 Eq. (10), Sec. 3.3).
 * direct_only = 0 (default): where their range checks pass, the kernels take
 * the one-hop factors s + t T as T (t + s / T) (checked per parameter set)
 * and the two-hop factors s2 A + T2 B as A (s2 + T2 B / A) (checked per
 * first hop and image); direct_only = 1: always the direct products.  Both
 * give the same results within rounding. */
nqs_status nqs_set_factor_form(nqs_ctx* ctx, int direct_only);

/* Per-kernel timing for benchmarks.  While enabled, every kernel launch of
 * this context is bracketed by HIP events on the call's stream.
 * nqs_profile_read synchronises those events and returns, for kernel id
 * `kernel` (0 theta, 1 lse, 2 eloc_bonds, 3 eloc_finish, 4 twohop,
 * 5 twohop_finish, 6 moments, 7 grad, 8 sample, 9 sr (whole nqs_sr_solve),
 * 10 gram (the S x S Gram matrix of nqs_sr_solve), 11 cholesky (its blocked
 * factorisation and the two triangular solves), 12 sq (nqs_structure_factor),
 * 13 cg (nqs_sr_solve_cg), 14 hop3 (the neighbour expansion and combine
 * kernels of nqs_lanczos_moments and nqs_lanczos_moments_p2, and the
 * fifth-order moment kernel)),
 * the summed duration
 * in ms and the launch count since the last reset; reset = 1 clears them. */
nqs_status nqs_profile_enable(nqs_ctx* ctx, int on);
nqs_status nqs_profile_read(nqs_ctx* ctx, int kernel, double* ms_out, int64_t* launches_out,
                            int reset);

const char* nqs_status_str(nqs_status s);
const char* nqs_last_error(const nqs_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* NQS_H */
