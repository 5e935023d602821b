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
// enb = nullptr: every enb[k] is 1 (lp_nb then holds log path sums).  back: add
// sum_b J_b^2 / 4 over the antiparallel bonds (the exchanges there and back,
// which the unordered-pair lists leave out).
hipError_t launch_hop_combine(const nqs_ctx* c, const int8_t* spins, int64_t n, const int32_t* off,
                              const double* lp, const double* eprev, int eprev_stride,
                              const double* lp_nb, const double* enb, int enb_stride, double* out,
                              int out_stride, hipStream_t st, int back = 0);

// Neighbour rows as launch_nb_write, and parent[k] = the bond exchanged to make row k.
hipError_t launch_nb_write_parent(const nqs_ctx* c, const int8_t* spins, int64_t n,
                                  const int32_t* off, int8_t* out, int16_t* parent,
                                  hipStream_t st);

// The wide E_loc kernel on exchange neighbours with parent bonds: each row's
// bond list is the unordered-pair second-hop list of its parent (pair_list.h
// rules); parent = nullptr gives the plain E_loc partials.
hipError_t launch_eloc_wide_pairs(const nqs_ctx* c, const int8_t* spins, int64_t S,
                                  const int16_t* parent, double* part, hipStream_t st);

// out[s] = log of the path sum sum_g chi_g psi_s(g s)(H_ss + sum_b (J_b/2) R_gb)
// from E_loc partials [S][G/16][6] (complex FP64).
hipError_t launch_pathsum_finish(const nqs_ctx* c, const int8_t* spins, int64_t S,
                                 const double* part, double* out, hipStream_t st);

}  // namespace nqs
