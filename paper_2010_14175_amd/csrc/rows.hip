// Choice of the fused per-row setup kernel instance (instantiated in rows_lds.hip, rows_reg.hip
// and rows_f32.hip, compiled in parallel): pattern capacity 8..64 (LDS sizing of the factor)
// times candidate table 128..8192 slots, with slot lists in LDS or in registers; the
// register-list form also with FP32 arithmetic.
#include "rows.hpp"

namespace afsai {

RowsKernel rows_kernel_lds(int mmax_t, int cap);
RowsKernel rows_kernel_reg(int mmax_t, int cap);
RowsKernel rows_kernel_f32(int mmax_t, int cap);

RowsKernel rows_kernel(int mmax_t, int cap, bool rsl, bool f32) {
    if (f32) return rsl ? rows_kernel_f32(mmax_t, cap) : nullptr;  // FP32: register-list form only
    return rsl ? rows_kernel_reg(mmax_t, cap) : rows_kernel_lds(mmax_t, cap);
}

}  // namespace afsai
