// Learned format selector (paper, Method: predicting optimal configuration
// parameters, multi-class classification over the sparsity features).
#include "common.hpp"

namespace spmv {

spmv_status select_model(spmv_matrix_s *, const float *, spmv_format *, float *, hipStream_t) {
    set_error("no selector weights loaded");
    return SPMV_ERR_NO_MODEL;
}

}  // namespace spmv
