// Sample-space stochastic reconfiguration (placeholder until the SR kernels land).
#include "nqs_internal.h"

extern "C" nqs_status nqs_sr_solve(nqs_ctx* c, const void* O, const double* eloc, int64_t S,
                                   double lambda, double dtau, double* dtheta_out, void* ws,
                                   size_t ws_bytes, hipStream_t st) {
  (void)O; (void)eloc; (void)S; (void)lambda; (void)dtau; (void)dtheta_out; (void)ws;
  (void)ws_bytes; (void)st;
  if (c) c->last_error = "nqs_sr_solve is not available in this build";
  return NQS_ERR_ARG;
}
