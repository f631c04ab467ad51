// The inverse-factor setup kernel: choice of the instance (FP64-gradient instances here, the
// FP32-gradient ones in rows_w_g32.hip).
#include "rows_w_inst.hpp"

namespace afsai {

RowsKernel rows_kernel_w_g32(int mmax, int maxlen, int cap, int lanes, int *gs_out, size_t *lds_out);
RowsKernel rows_kernel_w_large_g32(int mmax, int cap, size_t *lds_out);

// Kernel for patterns of at most mmax positions over rows of at most maxlen entries with a
// first table of `cap` slots (see rows_w_inst.hpp); g32: the gradient reads FP32 values.
RowsKernel rows_kernel_w(int mmax, int maxlen, int cap, int lanes, bool g32, int *gs_out, size_t *lds_out) {
    return g32 ? rows_kernel_w_g32(mmax, maxlen, cap, lanes, gs_out, lds_out)
               : winst::rows_kernel_w_t<false>(mmax, maxlen, cap, lanes, gs_out, lds_out);
}

RowsKernel rows_kernel_w_large(int mmax, int cap, bool g32, size_t *lds_out) {
    return g32 ? rows_kernel_w_large_g32(mmax, cap, lds_out) : winst::rows_kernel_w_large_t<false>(mmax, cap, lds_out);
}

}  // namespace afsai
