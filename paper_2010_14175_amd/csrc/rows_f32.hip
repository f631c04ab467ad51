// Instantiations of the fused per-row setup kernel, slot lists in registers, FP32 arithmetic.
#include "rows.hpp"

namespace afsai {

RowsKernel rows_kernel_f32(int mmax_t, int cap) {
    switch (mmax_t) {
        case 8: return rows_kernel_cap<8, true, float>(cap);
        case 16: return rows_kernel_cap<16, true, float>(cap);
        case 24: return rows_kernel_cap<24, true, float>(cap);
        case 32: return rows_kernel_cap<32, true, float>(cap);
        case 48: return rows_kernel_cap<48, true, float>(cap);
        case 64: return rows_kernel_cap<64, true, float>(cap);
        default: return nullptr;
    }
}

}  // namespace afsai
