// Instantiations of the fused per-row setup kernel, LDS form (any pattern up to 64 entries).
#include "rows.hpp"

namespace afsai {

RowsKernel rows_kernel_lds(int mmax_t, int cap) {
    switch (mmax_t) {
        case 8:
        case 16:
        case 24:
        case 32: return rows_kernel_cap<32, false>(cap);
        case 48: return rows_kernel_cap<48, false>(cap);
        case 64: return rows_kernel_cap<64, false>(cap);
        default: return nullptr;
    }
}

}  // namespace afsai
