// Exchange Metropolis sampler (placeholder until the sampling kernels land).
#include "nqs_internal.h"

extern "C" {

nqs_status nqs_chain_init(nqs_ctx* c, const int8_t* spins, int64_t n_chains,
                          uint64_t first_chain_id, uint64_t* chain_state, hipStream_t st) {
  (void)spins; (void)n_chains; (void)first_chain_id; (void)chain_state; (void)st;
  if (c) c->last_error = "nqs_chain_init is not available in this build";
  return NQS_ERR_ARG;
}

nqs_status nqs_sample(nqs_ctx* c, int64_t n_chains, int64_t n_per_chain, int32_t n_skip,
                      int32_t n_burn, uint64_t seed, uint64_t* chain_state, int8_t* spins_out,
                      float* acc_rate_out, int32_t* n_skip_out, void* ws, size_t ws_bytes,
                      hipStream_t st) {
  (void)n_chains; (void)n_per_chain; (void)n_skip; (void)n_burn; (void)seed; (void)chain_state;
  (void)spins_out; (void)acc_rate_out; (void)n_skip_out; (void)ws; (void)ws_bytes; (void)st;
  if (c) c->last_error = "nqs_sample is not available in this build";
  return NQS_ERR_ARG;
}

}  // extern "C"
