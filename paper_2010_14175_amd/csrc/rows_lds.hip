// Instantiations of the fused per-row setup kernel, slot lists in LDS (rows longer than 128
// entries): pattern capacity 8..64 times candidate table 128..8192 slots.
#include "rows.hpp"

namespace afsai {

RowsKernel rows_kernel_lds(int mmax_t, int cap) {
    switch (mmax_t) {
        case 8: return rows_kernel_cap<8, false>(cap);
        case 16: return rows_kernel_cap<16, false>(cap);
        case 24: return rows_kernel_cap<24, false>(cap);
        case 32: return rows_kernel_cap<32, false>(cap);
        case 48: return rows_kernel_cap<48, false>(cap);
        case 64: return rows_kernel_cap<64, false>(cap);
        default: return nullptr;
    }
}

}  // namespace afsai
