// Instantiations of the fused per-row setup kernel: pattern capacity 8..64 (LDS sizing of the
// factor) times candidate table 128..8192 slots, with slot lists in LDS or in registers; the
// register-list form also with FP32 arithmetic.
#include "rows.hpp"

namespace afsai {

RowsKernel rows_kernel(int mmax_t, int cap, bool rsl, bool f32) {
    if (f32) {  // FP32 arithmetic: register-list form only
        if (!rsl) return nullptr;
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
    if (rsl) {
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
