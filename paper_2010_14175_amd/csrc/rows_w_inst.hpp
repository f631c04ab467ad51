// Instances of the inverse-factor setup kernel (rows_w.hpp): lanes per row GS, pattern
// capacity MMAX (<= GS), new rows per W block NB, table slots CAP, and the gradient's value
// type (G32: FP32 values of A).  rows_w.hip holds the FP64-gradient instances and the choice,
// rows_w_g32.hip the FP32-gradient ones (compiled in parallel).
#pragma once

#include "rows_w.hpp"

namespace afsai {
namespace winst {

template <bool G32, int GS, int MMAX, int NB>
static RowsKernel w_cap(int cap, int mm, size_t *lds) {
#define AFSAI_W_CASE(C)                                        \
    case C:                                                    \
        *lds = rows_w_lds_bytes<GS, MMAX, C, NB>(mm);          \
        return wform::k_rows_w<GS, MMAX, C, NB, G32>;
    if constexpr (GS <= 16) {
        if (cap == 64) {
            *lds = rows_w_lds_bytes<GS, MMAX, 64, NB>(mm);
            return wform::k_rows_w<GS, MMAX, 64, NB, G32>;
        }
    }
    switch (cap) {
        AFSAI_W_CASE(128)
        AFSAI_W_CASE(256)
        AFSAI_W_CASE(512)
        AFSAI_W_CASE(1024)
        default: return nullptr;
    }
}

// 64 lanes per row with the large tables of a second launch (rows that overflowed the first)
template <bool G32, int MMAX>
static RowsKernel w_cap_large(int cap, int mm, size_t *lds) {
    constexpr int GS = 64, NB = 4;
    switch (cap) {
        AFSAI_W_CASE(128)
        AFSAI_W_CASE(256)
        AFSAI_W_CASE(512)
        AFSAI_W_CASE(1024)
        AFSAI_W_CASE(2048)
        AFSAI_W_CASE(4096)
        AFSAI_W_CASE(8192)
        default: return nullptr;
    }
}
#undef AFSAI_W_CASE

// Kernel for patterns of at most mmax positions over rows of at most maxlen entries with a
// first table of `cap` slots: the fewest lanes per row that hold a position per lane and the
// row entries left of column i in their slot lists.  Returns nullptr when none fits (rows
// longer than 128 entries, or no such table size); *gs_out and *lds_out (dynamic LDS bytes of
// one block) are set on success.
template <bool G32>
RowsKernel rows_kernel_w_t(int mmax, int maxlen, int cap, int lanes, int *gs_out, size_t *lds_out) {
    if (maxlen > 128 || mmax > 64) return nullptr;
    RowsKernel k = nullptr;
    int gs = 0;
    // groups of 8 and 16 lanes only with small tables (a selection pass visits CAP / GS slots
    // per lane); `lanes` asks for at least that many lanes per row
    if (lanes <= 8 && mmax <= 8 && maxlen <= 8 * wform::spw_of(8) && cap <= 128) {
        gs = 8;
        k = w_cap<G32, 8, 8, 1>(cap, mmax, lds_out);
    } else if (lanes <= 16 && mmax <= 16 && maxlen <= 16 * wform::spw_of(16) && cap <= 256) {
        gs = 16;
        k = w_cap<G32, 16, 16, 2>(cap, mmax, lds_out);
    } else if (lanes == 32 && mmax <= 32 && cap >= 128) {
        // two rows per wavefront of 32 lanes each: only when asked for (one row per wavefront
        // of 64 lanes measured faster: more wavefronts resident)
        gs = 32;
        k = mmax <= 24 ? w_cap<G32, 32, 24, 2>(cap, mmax, lds_out) : w_cap<G32, 32, 32, 2>(cap, mmax, lds_out);
    } else if (cap >= 128) {
        gs = 64;
        k = mmax <= 24 ? w_cap<G32, 64, 24, 2>(cap, mmax, lds_out)
                       : (mmax <= 48 ? w_cap<G32, 64, 48, 4>(cap, mmax, lds_out) : w_cap<G32, 64, 64, 4>(cap, mmax, lds_out));
    }
    if (k) *gs_out = gs;
    return k;
}

// The same form with 64 lanes per row and a table of `cap` slots (128..8192), for the rows
// that overflowed the first launch's table.
template <bool G32>
RowsKernel rows_kernel_w_large_t(int mmax, int cap, size_t *lds_out) {
    if (mmax > 64) return nullptr;
    return mmax <= 48 ? w_cap_large<G32, 48>(cap, mmax, lds_out) : w_cap_large<G32, 64>(cap, mmax, lds_out);
}

}  // namespace winst
}  // namespace afsai
