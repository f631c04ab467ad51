// Sliced ELLPACK with one wavefront-sized slice of 64 rows (SELL-64) for the products of the
// PCG iteration.  Within a slice the entries are stored column by column: entry k of the 64
// rows is contiguous, so one lane per row reads the matrix with fully coalesced 512-byte
// (values) and 256-byte (columns) wave loads, and the x entries of neighbouring rows are read
// together.  Rows shorter than the slice's longest row are padded with (own row, 0.0).
//
// When that padding would exceed a tenth of the entries (rows of very different lengths, as
// in G^T), the rows of each window of 4 consecutive slices (256 rows, never across two systems
// of a batch) are ordered by length and dealt to the window's slices (`perm`, with `lens` the
// length of each lane's row; SELL-C-sigma with C = 64, sigma = 256, Kreutzer et al. 2014):
// every lane stops at its own row's length, so the padding is never read, and the slices hold
// rows of similar length.  The four wavefronts of a block multiply one window and return the
// row sums to their natural rows through LDS before they are stored.  The alternative split form
// keeps every row's last w entries in the slices (w chosen from the length histogram) and the
// leading entries of the longer rows in a second SELL matrix (`tail`, in row order; `rowmap`
// maps its rows to rows of the full matrix), multiplied first; the main product then continues
// the sums of the rows marked in `init` from y (or runs them itself, `toff`).  Each row's sum is
// one sequential chain over its entries in stored order in every form, so all layouts give
// bit-identical products.
#pragma once

#include "common.hpp"

namespace afsai {

constexpr int kSlice = 64;
constexpr int kWin = 4;  // slices per window of rows ordered by length (one block of 4 wavefronts)

struct Sell {
    int n = 0;
    int nslices = 0;
    uint32_t *sptr = nullptr;   // [nslices + 1] offsets in 64-entry columns
    int32_t *col = nullptr;     // [sptr[nslices] * 64] (nullptr when col3 holds the columns)
    int32_t *col3 = nullptr;    // column runs: every row stores runs of three consecutive
                                // columns (c, c+1, c+2), so one index per run is kept:
                                // [sptr[nslices] / 3 * 64], run j of a slice at its entry 3j
    void *val = nullptr;        // double or float, same layout
    int32_t *perm = nullptr;    // [nslices * 64] row of each slice lane (nullptr: identity)
    int32_t *lens = nullptr;    // [nslices * 64] entries of each slice lane's row (nullptr: all
                                // lanes run the slice's width; else padding is never read)
    int32_t *wsl = nullptr;     // with lens: [nwin + 1] first slice of each window
    int32_t *wofs = nullptr;    // with lens: [nslices + 1] window of each slice (nwin at the end)
    int nwin = 0;
    int32_t *rowmap = nullptr;  // [n] output row of each row (nullptr: identity)
    uint64_t *init = nullptr;   // [nslices] lanes whose sums continue from y (nullptr: none)
    Sell *tail = nullptr;       // leading entries of the rows longer than the slices hold
    int32_t *toff = nullptr;    // [nslices + 1] with a tail: its first row for each slice (the
                                // rows of a slice marked in init are consecutive tail rows)
    int32_t *srow0 = nullptr;   // [nslices + 1] first row of each slice (nullptr: 64 * slice);
                                // set when slices follow the systems of a batch
    bool f32 = false;
    int64_t entries = 0;        // stored entries including padding (tail included)
    int width_cap = 0;          // entries per row held by the slices (0: all)
};

// Rows of a batch of independent systems: system k owns rows row0[k] .. row0[k+1]-1 (host).
// With nsys > 1 every system starts a new slice, so a slice never holds rows of two systems.
struct Segments {
    int nsys = 1;
    const int32_t *row0 = nullptr;  // host, nsys + 1 entries (nullptr: one system)
};
// slices of each system under a segmentation: slice0[k] .. slice0[k+1]-1 (host, nsys + 1)
void segment_slices(const Segments &seg, int n, int32_t *slice0);

// SELL-64 copy of a CSR matrix (device arrays); values converted to out_f32 ? float : double.
// Synchronous on s.  On failure nothing is left allocated.
int sell_from_csr(int n, int64_t nnz, const int32_t *rp, const int32_t *ci, const void *val, bool val_f32,
                  bool out_f32, Sell *out, const DeviceInfo &di, hipStream_t s, const Segments &seg = Segments());
// SELL-64 copy of padded row-major per-row results (ell_col/ell_val, ld entries per row, m[i]
// valid, nnz in total): the setup's direct output for G.
int sell_from_ell(int n, int64_t nnz, int ld, const int32_t *m, const int32_t *ell_col, const double *ell_val,
                  bool out_f32, Sell *out, const DeviceInfo &di, hipStream_t s, const Segments &seg = Segments());
void sell_free(Sell *S);
// Replace a plain layout's column array (no ordering, split or tail) by one index per run of
// three consecutive columns when every slice's stored entries, padding included, fall into
// such runs (the 3 x 3 blocks of a 3-dof discretisation; padding runs are (r, r, r) with
// zero values and become (c, c+1, c+2) with c <= n - 3).  Values and their order are
// unchanged, so every row's sum is the same chain.  Leaves S as it is when the matrix does
// not qualify.  With keep_col the per-entry columns stay beside the run indices (for kernels
// that read them, such as the block products of a prepared matrix).  Synchronous on s.
int sell_group_runs(Sell *S, const DeviceInfo &di, hipStream_t s, bool keep_col = false);

}  // namespace afsai
