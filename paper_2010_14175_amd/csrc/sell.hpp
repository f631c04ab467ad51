// Sliced ELLPACK with one wavefront-sized slice of 64 rows (SELL-64) for the products of the
// PCG iteration.  Within a slice the entries are stored column by column: entry k of the 64
// rows is contiguous, so one lane per row reads the matrix with fully coalesced 512-byte
// (values) and 256-byte (columns) wave loads, and the x entries of neighbouring rows are read
// together.  Rows shorter than the slice's longest row are padded with (own row, 0.0).
// When that padding would exceed a tenth of the entries (rows of very different lengths, as
// in G^T), rows are first sorted by length inside windows of kSortWindow rows and the slices
// follow that order (SELL-C-sigma, Kreutzer et al. 2014); `perm` then maps slice lanes back
// to rows.
#pragma once

#include "common.hpp"

namespace afsai {

constexpr int kSlice = 64;
constexpr int kSortWindow = 4096;

struct Sell {
    int n = 0;
    int nslices = 0;
    uint32_t *sptr = nullptr;  // [nslices + 1] offsets in 64-entry columns
    int32_t *col = nullptr;    // [sptr[nslices] * 64]
    void *val = nullptr;       // double or float, same layout
    int32_t *perm = nullptr;   // [nslices * 64] row of each slice lane (nullptr: identity)
    bool f32 = false;
    int64_t entries = 0;       // stored entries including padding
};

// SELL-64 copy of a CSR matrix (device arrays); values converted to out_f32 ? float : double.
// Synchronous on s.  On failure nothing is left allocated.
int sell_from_csr(int n, int64_t nnz, const int32_t *rp, const int32_t *ci, const void *val, bool val_f32,
                  bool out_f32, Sell *out, const DeviceInfo &di, hipStream_t s);
// SELL-64 copy of padded row-major per-row results (ell_col/ell_val, ld entries per row, m[i]
// valid): the setup's direct output for G.
int sell_from_ell(int n, int ld, const int32_t *m, const int32_t *ell_col, const double *ell_val, bool out_f32,
                  Sell *out, const DeviceInfo &di, hipStream_t s);
void sell_free(Sell *S);

}  // namespace afsai
