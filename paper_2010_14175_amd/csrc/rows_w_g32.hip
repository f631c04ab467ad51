// Instances of the inverse-factor setup kernel whose gradient reads FP32 values of A.
#include "rows_w_inst.hpp"

namespace afsai {

RowsKernel rows_kernel_w_g32(int mmax, int maxlen, int cap, int lanes, int *gs_out, size_t *lds_out) {
    return winst::rows_kernel_w_t<true>(mmax, maxlen, cap, lanes, gs_out, lds_out);
}

RowsKernel rows_kernel_w_large_g32(int mmax, int cap, size_t *lds_out) {
    return winst::rows_kernel_w_large_t<true>(mmax, cap, lds_out);
}

}  // namespace afsai
