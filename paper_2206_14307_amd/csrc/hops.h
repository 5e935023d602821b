// Declarations shared by the host API and the multi-hop (Lanczos) kernels.
#pragma once

#include "nqs_internal.h"

namespace nqs {

// Whether the register-resident two-hop kernel covers the model (one RBM,
// K*M <= 128 at the compiled sizes).
bool twohop_reg_supported(const nqs_ctx* c);

// out[s] = H_ss eprev[s] + sum_k (J_k/2) exp(lp_nb[k] - lp[s]) enb[k] over the
// neighbour rows k = off[s] .. off[s+1]-1 of configuration s (bond order):
// one more hop of (H^p psi)/psi from the previous order at the configuration
// and its neighbours.  Complex FP64; strides in doubles between configurations.
hipError_t launch_hop_combine(const nqs_ctx* c, const int8_t* spins, int64_t n, const int32_t* off,
                              const double* lp, const double* eprev, int eprev_stride,
                              const double* lp_nb, const double* enb, int enb_stride, double* out,
                              int out_stride, hipStream_t st);

}  // namespace nqs
