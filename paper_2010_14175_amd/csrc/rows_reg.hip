// Instantiations of the fused per-row setup kernel, slot lists in registers, FP64 arithmetic.
#include "rows.hpp"

namespace afsai {

RowsKernel rows_kernel_reg(int mmax_t, int cap) {
    switch (mmax_t) {
        case 8: return rows_kernel_cap<8, true>(cap);
        case 16: return rows_kernel_cap<16, true>(cap);
        case 24: return rows_kernel_cap<24, true>(cap);
        case 32: return rows_kernel_cap<32, true>(cap);
        case 48: return rows_kernel_cap<48, true>(cap);
        case 64: return rows_kernel_cap<64, true>(cap);
        default: return nullptr;
    }
}

}  // namespace afsai
