// Batched Lanczos iteration: placeholder until the block-column path lands.
#include "lanczos_common.h"

void batch_free(rd_graph g) { (void)g; }

extern "C" {

rd_status rd_query_batch(rd_graph g, int32_t, const int32_t *, const int32_t *, double,
                         const rd_options *, rd_result *) {
  if (g) g->err = "rd_query_batch is not available in this build";
  return RD_E_ARG;
}

rd_status rd_grad_edges(rd_graph g, int32_t, const int32_t *, const int32_t *, const double *,
                        double, const rd_options *, rd_result *, float *) {
  if (g) g->err = "rd_grad_edges is not available in this build";
  return RD_E_ARG;
}

}  // extern "C"
