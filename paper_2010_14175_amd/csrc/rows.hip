// Instantiations of the fused per-row setup kernel: pattern capacity 8..64 (LDS sizing of the
// factor) times candidate table 128..8192 slots.
#include "rows.hpp"

namespace afsai {

RowsKernel rows_kernel(int mmax_t, int cap) {
    switch (mmax_t) {
        case 8: return rows_kernel_cap<8>(cap);
        case 16: return rows_kernel_cap<16>(cap);
        case 24: return rows_kernel_cap<24>(cap);
        case 32: return rows_kernel_cap<32>(cap);
        case 48: return rows_kernel_cap<48>(cap);
        case 64: return rows_kernel_cap<64>(cap);
        default: return nullptr;
    }
}

}  // namespace afsai
