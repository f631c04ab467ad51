// Device scan and the SELL-64 layout used by the PCG products (sell.hpp).
#include <algorithm>
#include <vector>

#include "sell.hpp"

namespace afsai {

// ---------------------------------------------------------------------------------------
// exclusive scan of int32 counts into int32 offsets (three phases; deterministic)
// ---------------------------------------------------------------------------------------
constexpr int kScanThreads = 256, kScanItems = 8, kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t *sh, int64_t &total) {
    // sh: kScanThreads/64 + 1 entries
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) sh[w] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t acc = 0;
        for (int k = 0; k < kScanThreads / 64; ++k) {
            const int64_t t = sh[k];
            sh[k] = acc;
            acc += t;
        }
        sh[kScanThreads / 64] = acc;
    }
    __syncthreads();
    total = sh[kScanThreads / 64];
    const int64_t r = sh[w] + incl - v;
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(int n, const int32_t *__restrict__ cnt,
                                                             int64_t *__restrict__ tile_sum) {
    __shared__ int64_t sh[kScanThreads / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v = 0;
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) v += cnt[base + k];
    int64_t tot;
    block_excl_scan(v, sh, tot);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_sums(int ntiles, int64_t *__restrict__ tile_sum,
                                                            int64_t *__restrict__ total) {
    __shared__ int64_t sh[kScanThreads / 64 + 1];
    const int per = (ntiles + kScanThreads - 1) / kScanThreads;
    const int lo = threadIdx.x * per, hi = min(ntiles, lo + per);
    int64_t v = 0;
    for (int k = lo; k < hi; ++k) v += tile_sum[k];
    int64_t tot;
    int64_t off = block_excl_scan(v, sh, tot);
    for (int k = lo; k < hi; ++k) {
        const int64_t t = tile_sum[k];
        tile_sum[k] = off;
        off += t;
    }
    if (threadIdx.x == 0) *total = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(int n, const int32_t *__restrict__ cnt,
                                                             const int64_t *__restrict__ tile_off,
                                                             int32_t *__restrict__ out /* n+1 */) {
    __shared__ int64_t sh[kScanThreads / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v = 0;
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) v += cnt[base + k];
    int64_t tot;
    int64_t off = block_excl_scan(v, sh, tot) + tile_off[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) {
            out[base + k] = (int32_t)off;
            off += cnt[base + k];
        }
        if (base + k == n - 1) out[n] = (int32_t)off;
    }
}

int scan_counts(int n, const int32_t *cnt, int32_t *out, int64_t *total, const DeviceInfo &di, hipStream_t s) {
    (void)di;
    const int ntiles = (int)(((int64_t)n + kScanTile - 1) / kScanTile);
    DevBuf ts;
    int rc;
    if ((rc = dalloc(ts, sizeof(int64_t) * (size_t)(ntiles + 2), s))) return rc;
    int64_t *tot = ts.as<int64_t>() + ntiles + 1;
    hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(kScanThreads), 0, s, n, cnt, ts.as<int64_t>());
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, s, ntiles, ts.as<int64_t>(), tot);
    hipLaunchKernelGGL(k_scan_apply, dim3(ntiles), dim3(kScanThreads), 0, s, n, cnt, ts.as<int64_t>(), out);
    AFSAI_HIP_TRY(hipMemcpyAsync(total, tot, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    AFSAI_HIP_TRY(hipStreamSynchronize(s));
    return AFSAI_OK;
}

// ---------------------------------------------------------------------------------------
// SELL-64 construction.  Rows come either from a CSR matrix (rp) or from padded per-row
// results (m[r] entries at r * ld).
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ int row_len(const int32_t *rp, const int32_t *m, int r) {
    return rp ? rp[r + 1] - rp[r] : m[r];
}
__device__ __forceinline__ int64_t row_start(const int32_t *rp, int ld, int r) {
    return rp ? (int64_t)rp[r] : (int64_t)r * ld;
}

// rows [r0, r1) of slice sl
__device__ __forceinline__ void slice_rows(const int32_t *srow0, int n, int sl, int &r0, int &r1) {
    if (srow0) {
        r0 = srow0[sl];
        r1 = srow0[sl + 1];
    } else {
        r0 = sl * kSlice;
        r1 = min(n, r0 + kSlice);
    }
}

// rows of each window ordered by length (longest first, ties by row), one block of 256
// threads per window: the window's k-th row goes to lane k % 64 of its slice k / 64 (perm: the
// row, -1 past the window's rows; lens: its length).  A lane then stops at its own row's
// length and the slices of a window hold rows of similar length.
__global__ __launch_bounds__(kWin * kSlice) void k_window_sort(int n, int nwin, const int32_t *__restrict__ wsl,
                                                               const int32_t *__restrict__ rp,
                                                               const int32_t *__restrict__ m,
                                                               const int32_t *__restrict__ srow0,
                                                               int32_t *__restrict__ perm,
                                                               int32_t *__restrict__ lens) {
    __shared__ int32_t wl[kWin * kSlice];
    const int t = threadIdx.x;
    for (int w = blockIdx.x; w < nwin; w += gridDim.x) {
        const int ws = wsl[w], we = wsl[w + 1];
        int wr0, wr1, u0, u1;
        slice_rows(srow0, n, ws, wr0, u0);
        slice_rows(srow0, n, we - 1, u1, wr1);
        const int cnt = wr1 - wr0;  // at most kWin * 64 rows
        const int len = t < cnt ? row_len(rp, m, wr0 + t) : -1;
        wl[t] = len;
        __syncthreads();
        if (t < cnt) {
            int rank = 0;
            for (int j = 0; j < cnt; ++j) {
                const int lj = wl[j];
                rank += (lj > len || (lj == len && j < t)) ? 1 : 0;
            }
            perm[(int64_t)ws * kSlice + rank] = wr0 + t;
            lens[(int64_t)ws * kSlice + rank] = len;
        }
        for (int k = cnt + t; k < (we - ws) * kSlice; k += blockDim.x) {
            perm[(int64_t)ws * kSlice + k] = -1;
            lens[(int64_t)ws * kSlice + k] = 0;
        }
        __syncthreads();
    }
}

// width of each slice = its longest row, capped at `cap` entries (one wavefront per slice)
__global__ __launch_bounds__(256) void k_sell_width(int n, int nslices, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ m, const int32_t *__restrict__ perm,
                                                     const int32_t *__restrict__ srow0, int cap,
                                                     int32_t *__restrict__ width) {
    const int lane = threadIdx.x & 63;
    for (int sl = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; sl < nslices; sl += (gridDim.x * blockDim.x) >> 6) {
        int r0, r1;
        slice_rows(srow0, n, sl, r0, r1);
        int r = r0 + lane;
        if (perm) r = perm[sl * kSlice + lane];
        int len = 0;
        if (r >= 0 && r < (perm ? n : r1)) len = min(row_len(rp, m, r), cap);
        len = wave_max(len);
        if (lane == 0) width[sl] = len;
    }
}

constexpr int kHistBins = 256;

// histogram of row lengths (the last bin holds every longer row)
__global__ __launch_bounds__(256) void k_len_hist(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ m,
                                                   int32_t *__restrict__ hist) {
    __shared__ int32_t h[kHistBins];
    for (int j = threadIdx.x; j < kHistBins; j += blockDim.x) h[j] = 0;
    __syncthreads();
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
        atomicAdd(&h[min(row_len(rp, m, r), kHistBins - 1)], 1);
    __syncthreads();
    for (int j = threadIdx.x; j < kHistBins; j += blockDim.x)
        if (h[j]) atomicAdd(&hist[j], h[j]);
}

// One wavefront per slice; lane = row; the slices hold the last min(len, cap) entries of each
// row; padding entries are (own row, 0).  init[sl] marks the lanes whose rows are longer.
template <typename VI, typename VO>
__global__ __launch_bounds__(256) void k_sell_fill(int n, int nslices, const int32_t *__restrict__ rp,
                                                    const int32_t *__restrict__ m, int ld,
                                                    const int32_t *__restrict__ ci, const VI *__restrict__ val,
                                                    const int32_t *__restrict__ perm,
                                                    const int32_t *__restrict__ srow0,
                                                    const int32_t *__restrict__ sptr, int cap,
                                                    int32_t *__restrict__ col, VO *__restrict__ out,
                                                    uint64_t *__restrict__ init) {
    const int lane = threadIdx.x & 63;
    for (int sl = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; sl < nslices; sl += (gridDim.x * blockDim.x) >> 6) {
        int r0, r1;
        slice_rows(srow0, n, sl, r0, r1);
        int r = r0 + lane;
        if (perm) r = perm[sl * kSlice + lane];
        int len = 0, keep = 0;
        int64_t start = 0;
        const bool valid = r >= 0 && r < (perm ? n : r1);
        if (valid) {
            len = row_len(rp, m, r);
            keep = min(len, cap);
            start = row_start(rp, ld, r) + (len - keep);
        }
        if (init) {
            const uint64_t longer = __ballot(valid && len > cap);
            if (lane == 0) init[sl] = longer;
        }
        const int pad_col = valid ? r : r0;
        const int64_t base = (int64_t)sptr[sl] * kSlice + lane;
        const int width = sptr[sl + 1] - sptr[sl];
        for (int k0 = 0; k0 < width; k0 += 8) {
            int cv[8];
            VO vv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = k0 + u;
                cv[u] = pad_col;
                vv[u] = VO(0);
                if (k < keep) {
                    cv[u] = ci[start + k];
                    vv[u] = (VO)val[start + k];
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (k0 + u < width) {
                    const int64_t d = base + (int64_t)(k0 + u) * kSlice;
                    col[d] = cv[u];
                    out[d] = vv[u];
                }
            }
        }
    }
}

// Orders LDS accesses across the lanes of one wavefront: a wavefront's LDS instructions
// execute in issue order, so only the compiler must keep them on their side of this point.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_wave_barrier();
    __asm__ __volatile__("" ::: "memory");
}

// The same layout for whole rows (no split; rows in row order, or those perm assigns to each
// slice position), staged through LDS: one wavefront per slice takes its 64 rows KF entries
// at a time, reading each row's run of KF consecutive entries with KF lanes (64 / KF rows per
// instruction), then storing each entry position of the slice with one contiguous 64-lane
// store.  KF = 32 for long rows (81-entry rows of the 27-point matrices: A 4.9 -> 4.0 ms at
// 150^3), 16 otherwise (46-entry rows of G: 2.5 ms against 3.8 ms with 32).
template <typename VI, typename VO, int KF>
__global__ __launch_bounds__(256) void k_sell_fill_rows(int n, int nslices, const int32_t *__restrict__ rp,
                                                         const int32_t *__restrict__ m, int ld,
                                                         const int32_t *__restrict__ ci, const VI *__restrict__ val,
                                                         const int32_t *__restrict__ perm,
                                                         const int32_t *__restrict__ srow0,
                                                         const int32_t *__restrict__ sptr, int32_t *__restrict__ col,
                                                         VO *__restrict__ out) {
    constexpr int RPI = 64 / KF;  // rows per read instruction
    __shared__ int32_t lcol[4][KF][kSlice + 1];
    __shared__ VO lval[4][KF][kSlice + 1];
    __shared__ int64_t lstart[4][kSlice];
    __shared__ int32_t llen[4][kSlice], lpad[4][kSlice];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int kk = lane % KF, rq = lane / KF;
    for (int sl = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; sl < nslices; sl += (gridDim.x * blockDim.x) >> 6) {
        int r0, r1;
        slice_rows(srow0, n, sl, r0, r1);
        const int64_t base = (int64_t)sptr[sl] * kSlice;
        const int width = sptr[sl + 1] - sptr[sl];
        {
            // lane = slice position: its row's start, length and padding column
            const int r = perm ? perm[(int64_t)sl * kSlice + lane] : r0 + lane;
            const bool valid = perm ? r >= 0 : r < r1;
            lstart[wv][lane] = valid ? row_start(rp, ld, r) : 0;
            llen[wv][lane] = valid ? row_len(rp, m, r) : 0;
            lpad[wv][lane] = valid ? r : r0;
        }
        wave_lds_sync();
        for (int k0 = 0; k0 < width; k0 += KF) {
            const int k = k0 + kk;
            int c[kSlice / RPI];
            VO v[kSlice / RPI];
#pragma unroll
            for (int j = 0; j < kSlice / RPI; ++j) {
                const int rr = j * RPI + rq;
                c[j] = lpad[wv][rr];
                v[j] = VO(0);
                if (k < llen[wv][rr]) {
                    const int64_t e = lstart[wv][rr] + k;
                    c[j] = ci[e];
                    v[j] = (VO)val[e];
                }
            }
#pragma unroll
            for (int j = 0; j < kSlice / RPI; ++j) {
                lcol[wv][kk][j * RPI + rq] = c[j];
                lval[wv][kk][j * RPI + rq] = v[j];
            }
            wave_lds_sync();
            const int kn = min(KF, width - k0);
            for (int t = 0; t < kn; ++t) {
                const int64_t d = base + (int64_t)(k0 + t) * kSlice + lane;
                col[d] = lcol[wv][t][lane];
                out[d] = lval[wv][t][lane];
            }
            wave_lds_sync();
        }
    }
}

template <typename VI, typename VO>
static void launch_fill_rows(bool wide, int nbs, hipStream_t s, int n, int nslices, const int32_t *rp, const int32_t *m,
                             int ld, const int32_t *ci, const VI *val, const int32_t *perm, const int32_t *srow0,
                             const int32_t *sptr, int32_t *col, VO *out) {
    if (wide)
        hipLaunchKernelGGL((k_sell_fill_rows<VI, VO, 32>), dim3(nbs), dim3(256), 0, s, n, nslices, rp, m, ld, ci, val,
                           perm, srow0, sptr, col, out);
    else
        hipLaunchKernelGGL((k_sell_fill_rows<VI, VO, 16>), dim3(nbs), dim3(256), 0, s, n, nslices, rp, m, ld, ci, val,
                           perm, srow0, sptr, col, out);
}

// leading entries of the rows longer than cap: count per row, and a 0/1 flag per row
__global__ void k_tail_count(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ m, int cap,
                             int32_t *__restrict__ tl, int32_t *__restrict__ flag) {
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        const int t = max(0, row_len(rp, m, r) - cap);
        tl[r] = t;
        flag[r] = t > 0 ? 1 : 0;
    }
}

// the tail as CSR over the longer rows (ascending): row k = rowlist[k], its first len - cap
// entries
template <typename VI>
__global__ void k_tail_fill(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ m, int ld,
                            const int32_t *__restrict__ ci, const VI *__restrict__ val, const int32_t *__restrict__ tl,
                            const int32_t *__restrict__ toff, const int32_t *__restrict__ pos,
                            int32_t *__restrict__ trp, int32_t *__restrict__ tci, VI *__restrict__ tval,
                            int32_t *__restrict__ rowlist) {
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        const int t = tl[r];
        if (t <= 0) continue;
        const int k = pos[r];
        rowlist[k] = r;
        trp[k] = toff[r];
        const int64_t src = row_start(rp, ld, r);
        for (int e = 0; e < t; ++e) {
            tci[toff[r] + e] = ci[src + e];
            tval[toff[r] + e] = val[src + e];
        }
    }
}

__global__ void k_set_i32(int32_t *p, int32_t v) { *p = v; }

// rows of each slice that continue from the tail (count of its init bits)
__global__ void k_init_count(int nslices, const uint64_t *__restrict__ init, int32_t *__restrict__ cnt) {
    for (int sl = blockIdx.x * blockDim.x + threadIdx.x; sl < nslices; sl += gridDim.x * blockDim.x)
        cnt[sl] = __popcll(init[sl]);
}

void sell_free(Sell *S) {
    if (!S) return;
    pool_free(S->sptr);
    pool_free(S->col);
    pool_free(S->col3);
    pool_free(S->val);
    pool_free(S->perm);
    pool_free(S->lens);
    pool_free(S->wsl);
    pool_free(S->wofs);
    pool_free(S->rowmap);
    pool_free(S->init);
    pool_free(S->toff);
    pool_free(S->srow0);
    if (S->tail) {
        sell_free(S->tail);
        delete S->tail;
    }
    *S = Sell();
}

static int sell_build(int n, int64_t nnz, const int32_t *rp, const int32_t *m, int ld, const int32_t *ci,
                      const void *val, bool val_f32, bool out_f32, bool top, Sell *out, const DeviceInfo &di,
                      hipStream_t s, const Segments &seg);

// The tail of a split layout: CSR of the leading entries of the rows longer than cap, then
// a sorted SELL of it whose rows map back to rows of the full matrix.
static int build_tail(int n, const int32_t *rp, const int32_t *m, int ld, const int32_t *ci, const void *val,
                      bool val_f32, bool out_f32, int cap, Sell **out, const DeviceInfo &di, hipStream_t s) {
    DevBuf tl, flag, toff, pos;
    int rc;
    if ((rc = dalloc(tl, sizeof(int32_t) * (size_t)n, s))) return rc;
    if ((rc = dalloc(flag, sizeof(int32_t) * (size_t)n, s))) return rc;
    if ((rc = dalloc(toff, sizeof(int32_t) * (size_t)(n + 1), s))) return rc;
    if ((rc = dalloc(pos, sizeof(int32_t) * (size_t)(n + 1), s))) return rc;
    hipLaunchKernelGGL(k_tail_count, dim3(grid1d(n, di)), dim3(256), 0, s, n, rp, m, cap, tl.as<int32_t>(),
                       flag.as<int32_t>());
    int64_t tnnz = 0, nrows = 0;
    if ((rc = scan_counts(n, tl.as<int32_t>(), toff.as<int32_t>(), &tnnz, di, s))) return rc;
    if ((rc = scan_counts(n, flag.as<int32_t>(), pos.as<int32_t>(), &nrows, di, s))) return rc;
    *out = nullptr;
    if (nrows == 0) return AFSAI_OK;
    const size_t vb = val_f32 ? sizeof(float) : sizeof(double);
    DevBuf trp, tci, tval;
    if ((rc = dalloc(trp, sizeof(int32_t) * (size_t)(nrows + 1), s))) return rc;
    if ((rc = dalloc(tci, sizeof(int32_t) * (size_t)tnnz, s))) return rc;
    if ((rc = dalloc(tval, vb * (size_t)tnnz, s))) return rc;
    int32_t *rowlist = (int32_t *)pool_alloc(sizeof(int32_t) * (size_t)nrows);
    if (!rowlist) AFSAI_FAIL(AFSAI_ERR_NO_MEMORY, "SELL layout: out of device memory");
    if (val_f32)
        hipLaunchKernelGGL(k_tail_fill<float>, dim3(grid1d(n, di)), dim3(256), 0, s, n, rp, m, ld, ci,
                           (const float *)val, tl.as<int32_t>(), toff.as<int32_t>(), pos.as<int32_t>(),
                           trp.as<int32_t>(), tci.as<int32_t>(), tval.as<float>(), rowlist);
    else
        hipLaunchKernelGGL(k_tail_fill<double>, dim3(grid1d(n, di)), dim3(256), 0, s, n, rp, m, ld, ci,
                           (const double *)val, tl.as<int32_t>(), toff.as<int32_t>(), pos.as<int32_t>(),
                           trp.as<int32_t>(), tci.as<int32_t>(), tval.as<double>(), rowlist);
    hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, s, trp.as<int32_t>() + nrows, (int32_t)tnnz);
    Sell *T = new Sell();
    rc = sell_build((int)nrows, tnnz, trp.as<int32_t>(), nullptr, 0, tci.as<int32_t>(), tval.p, val_f32, out_f32,
                    false, T, di, s, Segments());
    if (rc) {
        pool_free(rowlist);
        delete T;
        return rc;
    }
    T->rowmap = rowlist;
    *out = T;
    return AFSAI_OK;
}

// Splitting width: minimises the slice entries (padding included) plus three times the tail
// entries (gathered through a second, sorted layout), from the slice widths and the length
// histogram.  Returns 0 when keeping whole rows is cheapest.
static int choose_cap(const std::vector<int32_t> &width, const std::vector<int32_t> &hist) {
    int maxw = 0;
    for (int w : width) maxw = std::max(maxw, w);
    double best = 0.0;
    for (int w : width) best += (double)w * kSlice;
    int best_cap = 0;
    for (int cap = 1; cap < std::min(maxw, kHistBins - 1); ++cap) {
        double cost = 0.0;
        for (int w : width) cost += (double)std::min(w, cap) * kSlice;
        for (int L = cap + 1; L < kHistBins; ++L) cost += 3.0 * (double)(L - cap) * hist[L];
        if (cost < best) {
            best = cost;
            best_cap = cap;
        }
    }
    return best_cap;
}

void segment_slices(const Segments &seg, int n, int32_t *slice0) {
    slice0[0] = 0;
    if (!seg.row0 || seg.nsys <= 1) {
        slice0[1] = (n + kSlice - 1) / kSlice;
        return;
    }
    for (int k = 0; k < seg.nsys; ++k)
        slice0[k + 1] = slice0[k] + (seg.row0[k + 1] - seg.row0[k] + kSlice - 1) / kSlice;
}

// windows of kWin slices, starting at every system's first slice: first slice of each window
// (nwin + 1 entries) and window of each slice (nslices + 1 entries)
static void make_windows(int nslices, int n, const Segments &seg, std::vector<int32_t> &hw, std::vector<int32_t> &hofs) {
    hw.clear();
    hofs.assign(nslices + 1, 0);
    std::vector<int32_t> s0(2, 0);
    if (seg.row0 && seg.nsys > 1) {
        s0.resize(seg.nsys + 1);
        segment_slices(seg, n, s0.data());
    } else {
        s0[1] = nslices;
    }
    for (size_t k = 0; k + 1 < s0.size(); ++k)
        for (int w = s0[k]; w < s0[k + 1]; w += kWin) {
            for (int j = w; j < std::min(s0[k + 1], w + kWin); ++j) hofs[j] = (int32_t)hw.size();
            hw.push_back(w);
        }
    hofs[nslices] = (int32_t)hw.size();
    hw.push_back(nslices);
}

static int sell_build(int n, int64_t nnz, const int32_t *rp, const int32_t *m, int ld, const int32_t *ci,
                      const void *val, bool val_f32, bool out_f32, bool top, Sell *out, const DeviceInfo &di,
                      hipStream_t s, const Segments &seg) {
    Sell S;
    S.n = n;
    S.f32 = out_f32;
    int rc;
    auto fail = [&](int code) {
        sell_free(&S);
        return code;
    };
    if (seg.row0 && seg.nsys > 1) {
        // every system starts a new slice
        std::vector<int32_t> slice0(seg.nsys + 1);
        segment_slices(seg, n, slice0.data());
        S.nslices = slice0[seg.nsys];
        std::vector<int32_t> h(S.nslices + 1);
        for (int k = 0; k < seg.nsys; ++k)
            for (int j = slice0[k]; j < slice0[k + 1]; ++j) h[j] = seg.row0[k] + (j - slice0[k]) * kSlice;
        h[S.nslices] = n;
        S.srow0 = (int32_t *)pool_alloc(sizeof(int32_t) * h.size());
        if (!S.srow0) return fail(set_error_code(AFSAI_ERR_NO_MEMORY, "SELL layout: out of device memory"));
        if (hipMemcpyAsync(S.srow0, h.data(), sizeof(int32_t) * h.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(set_error_code(AFSAI_ERR_HIP, "SELL layout: copy of the slice rows failed"));
    } else {
        S.nslices = (n + kSlice - 1) / kSlice;
    }
    DevBuf width;
    if ((rc = dalloc(width, sizeof(int32_t) * (size_t)S.nslices, s))) return fail(rc);
    const int nbs = grid1d((int64_t)S.nslices * 64, di);
    S.sptr = (uint32_t *)pool_alloc(sizeof(uint32_t) * (size_t)(S.nslices + 1));
    if (!S.sptr) return fail(set_error_code(AFSAI_ERR_NO_MEMORY, "SELL layout: out of device memory"));
    const int kNoCap = 0x7fffffff;
    hipLaunchKernelGGL(k_sell_width, dim3(nbs), dim3(256), 0, s, n, S.nslices, rp, m, nullptr, S.srow0, kNoCap,
                       width.as<int32_t>());
    int64_t cols = 0;
    if ((rc = scan_counts(S.nslices, width.as<int32_t>(), (int32_t *)S.sptr, &cols, di, s))) return fail(rc);
    int cap = kNoCap;
    const bool padded = cols * kSlice > nnz + nnz / 10 && n > kSlice;
    if (top) {
        const int forced = (int)option(AFSAI_OPT_SELL_WIDTH);
        if (forced > 0) {
            cap = forced;
        } else if (padded && option(AFSAI_OPT_SELL_UNEVEN) != 1) {
            // uneven rows: the rows of each window of slices ordered by length, lanes stop at
            // their own row; windows start at every system's first slice
            std::vector<int32_t> hw, hofs;
            make_windows(S.nslices, n, seg, hw, hofs);
            S.nwin = (int)hw.size() - 1;
            S.perm = (int32_t *)pool_alloc(sizeof(int32_t) * (size_t)S.nslices * kSlice);
            S.lens = (int32_t *)pool_alloc(sizeof(int32_t) * (size_t)S.nslices * kSlice);
            S.wsl = (int32_t *)pool_alloc(sizeof(int32_t) * hw.size());
            S.wofs = (int32_t *)pool_alloc(sizeof(int32_t) * hofs.size());
            if (!S.perm || !S.lens || !S.wsl || !S.wofs)
                return fail(set_error_code(AFSAI_ERR_NO_MEMORY, "SELL layout: out of device memory"));
            if (hipMemcpyAsync(S.wsl, hw.data(), sizeof(int32_t) * hw.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
                hipMemcpyAsync(S.wofs, hofs.data(), sizeof(int32_t) * hofs.size(), hipMemcpyHostToDevice, s) !=
                    hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return fail(set_error_code(AFSAI_ERR_HIP, "SELL layout: copy of the windows failed"));
            hipLaunchKernelGGL(k_window_sort, dim3(std::min(S.nwin, di.num_cus * 16)), dim3(kWin * kSlice), 0, s, n,
                               S.nwin, S.wsl, rp, m, S.srow0, S.perm, S.lens);
            // each slice's width is now its longest ordered row
            hipLaunchKernelGGL(k_sell_width, dim3(nbs), dim3(256), 0, s, n, S.nslices, rp, m, S.perm, S.srow0, kNoCap,
                               width.as<int32_t>());
            if ((rc = scan_counts(S.nslices, width.as<int32_t>(), (int32_t *)S.sptr, &cols, di, s))) return fail(rc);
        } else if (padded) {
            // split at the width that minimises the work (host choice from device statistics)
            DevBuf hist;
            if ((rc = dalloc(hist, sizeof(int32_t) * kHistBins, s))) return fail(rc);
            if (hipMemsetAsync(hist.p, 0, sizeof(int32_t) * kHistBins, s) != hipSuccess)
                return fail(set_error_code(AFSAI_ERR_HIP, "SELL layout: memset failed"));
            hipLaunchKernelGGL(k_len_hist, dim3(grid1d(n, di)), dim3(256), 0, s, n, rp, m, hist.as<int32_t>());
            std::vector<int32_t> hw(S.nslices), hh(kHistBins);
            if (hipMemcpyAsync(hw.data(), width.p, sizeof(int32_t) * S.nslices, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipMemcpyAsync(hh.data(), hist.p, sizeof(int32_t) * kHistBins, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return fail(set_error_code(AFSAI_ERR_HIP, "SELL layout: statistics copy failed"));
            const int c = choose_cap(hw, hh);
            if (c > 0) cap = c;
        }
        if (cap != kNoCap) {
            hipLaunchKernelGGL(k_sell_width, dim3(nbs), dim3(256), 0, s, n, S.nslices, rp, m, nullptr, S.srow0, cap,
                               width.as<int32_t>());
            if ((rc = scan_counts(S.nslices, width.as<int32_t>(), (int32_t *)S.sptr, &cols, di, s))) return fail(rc);
            if ((rc = build_tail(n, rp, m, ld, ci, val, val_f32, out_f32, cap, &S.tail, di, s))) return fail(rc);
            if (S.tail) {
                S.width_cap = cap;
                S.init = (uint64_t *)pool_alloc(sizeof(uint64_t) * (size_t)S.nslices);
                if (!S.init) return fail(set_error_code(AFSAI_ERR_NO_MEMORY, "SELL layout: out of device memory"));
            } else {
                cap = kNoCap;
            }
        }
    }
    if (cols >= ((int64_t)1 << 31))
        return fail(set_error_code(AFSAI_ERR_TOO_LARGE, "SELL layout: %lld columns", (long long)cols));
    S.entries = cols * kSlice + (S.tail ? S.tail->entries : 0);
    S.col = (int32_t *)pool_alloc(sizeof(int32_t) * (size_t)cols * kSlice);
    S.val = pool_alloc((out_f32 ? sizeof(float) : sizeof(double)) * (size_t)cols * kSlice);
    if (!S.col || !S.val) return fail(set_error_code(AFSAI_ERR_NO_MEMORY, "SELL layout: out of device memory"));
    const int32_t *sp = (const int32_t *)S.sptr;
    if (cap == kNoCap && !S.init) {
        // whole rows, staged 32 entries a row at a time for rows of 64 entries or more on average
        const bool wide = nnz >= (int64_t)64 * n;
        if (val_f32) {
            if (out_f32)
                launch_fill_rows<float, float>(wide, nbs, s, n, S.nslices, rp, m, ld, ci, (const float *)val, S.perm,
                                               S.srow0, sp, S.col, (float *)S.val);
            else
                launch_fill_rows<float, double>(wide, nbs, s, n, S.nslices, rp, m, ld, ci, (const float *)val, S.perm,
                                                S.srow0, sp, S.col, (double *)S.val);
        } else {
            if (out_f32)
                launch_fill_rows<double, float>(wide, nbs, s, n, S.nslices, rp, m, ld, ci, (const double *)val,
                                                S.perm, S.srow0, sp, S.col, (float *)S.val);
            else
                launch_fill_rows<double, double>(wide, nbs, s, n, S.nslices, rp, m, ld, ci, (const double *)val,
                                                 S.perm, S.srow0, sp, S.col, (double *)S.val);
        }
    } else if (val_f32) {
        if (out_f32)
            hipLaunchKernelGGL((k_sell_fill<float, float>), dim3(nbs), dim3(256), 0, s, n, S.nslices, rp, m, ld, ci,
                               (const float *)val, S.perm, S.srow0, sp, cap, S.col, (float *)S.val, S.init);
        else
            hipLaunchKernelGGL((k_sell_fill<float, double>), dim3(nbs), dim3(256), 0, s, n, S.nslices, rp, m, ld, ci,
                               (const float *)val, S.perm, S.srow0, sp, cap, S.col, (double *)S.val, S.init);
    } else {
        if (out_f32)
            hipLaunchKernelGGL((k_sell_fill<double, float>), dim3(nbs), dim3(256), 0, s, n, S.nslices, rp, m, ld, ci,
                               (const double *)val, S.perm, S.srow0, sp, cap, S.col, (float *)S.val, S.init);
        else
            hipLaunchKernelGGL((k_sell_fill<double, double>), dim3(nbs), dim3(256), 0, s, n, S.nslices, rp, m, ld,
                               ci, (const double *)val, S.perm, S.srow0, sp, cap, S.col, (double *)S.val, S.init);
    }
    if (hipGetLastError() != hipSuccess) return fail(set_error_code(AFSAI_ERR_HIP, "SELL layout: launch failed"));
    if (S.tail) {
        // first tail row of each slice, so that a slice's product can run its rows' tails itself
        DevBuf icnt;
        int64_t ntail = 0;
        if ((rc = dalloc(icnt, sizeof(int32_t) * (size_t)S.nslices, s))) return fail(rc);
        S.toff = (int32_t *)pool_alloc(sizeof(int32_t) * (size_t)(S.nslices + 1));
        if (!S.toff) return fail(set_error_code(AFSAI_ERR_NO_MEMORY, "SELL layout: out of device memory"));
        hipLaunchKernelGGL(k_init_count, dim3(grid1d(S.nslices, di)), dim3(256), 0, s, S.nslices, S.init,
                           icnt.as<int32_t>());
        if ((rc = scan_counts(S.nslices, icnt.as<int32_t>(), S.toff, &ntail, di, s))) return fail(rc);
        if (ntail != S.tail->n)
            return fail(set_error_code(AFSAI_ERR_HIP, "SELL layout: %lld split rows against %d tail rows",
                                       (long long)ntail, S.tail->n));
    }
    *out = S;
    return AFSAI_OK;
}

// slices whose width is not a multiple of three (their runs would cross slices)
__global__ __launch_bounds__(256) void k_runs_widths(int nslices, const uint32_t *__restrict__ sptr,
                                                     int32_t *__restrict__ bad) {
    for (int sl = blockIdx.x * blockDim.x + threadIdx.x; sl < nslices; sl += gridDim.x * blockDim.x)
        if ((sptr[sl + 1] - sptr[sl]) % 3u) atomicOr(bad, 1);
}

// one index per run: entries 3j, 3j+1, 3j+2 of a lane either hold consecutive columns (a run)
// or are padding (one column three times, zero values); anything else marks the matrix
template <typename VT>
__global__ __launch_bounds__(256) void k_sell_runs(int n, int64_t nruns, const int32_t *__restrict__ col,
                                                   const VT *__restrict__ val, int32_t *__restrict__ col3,
                                                   int32_t *__restrict__ bad) {
    bool err = false;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nruns * kSlice;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = t / kSlice, lane = t % kSlice;
        const int64_t e = 3 * j * kSlice + lane;
        const int c0 = col[e], c1 = col[e + kSlice], c2 = col[e + 2 * kSlice];
        int c = c0;
        if (c1 == c0 + 1 && c2 == c0 + 2) {
            if (c0 < 0 || c2 >= n) err = true;
        } else if (c0 == c1 && c1 == c2 && val[e] == VT(0) && val[e + kSlice] == VT(0) &&
                   val[e + 2 * kSlice] == VT(0)) {
            c = max(0, min(c0, n - 3));
        } else {
            err = true;
        }
        col3[t] = c;
    }
    if (err) atomicOr(bad, 1);
}

int sell_group_runs(Sell *S, const DeviceInfo &di, hipStream_t s, bool keep_col) {
    if (S->col3 || !S->col || S->perm || S->lens || S->tail || S->init || S->rowmap || S->n < 3 || S->nslices < 1)
        return AFSAI_OK;
    uint32_t cols = 0;
    if (hipMemcpyAsync(&cols, S->sptr + S->nslices, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return set_error_code(AFSAI_ERR_HIP, "SELL runs: copy of the column count failed");
    if (cols % 3u) return AFSAI_OK;
    const int64_t nruns = cols / 3u;
    DevBuf flag;
    int rc;
    if ((rc = dalloc(flag, sizeof(int32_t), s))) return rc;
    int32_t *c3 = (int32_t *)pool_alloc(sizeof(int32_t) * (size_t)(nruns > 0 ? nruns : 1) * kSlice);
    if (!c3) return set_error_code(AFSAI_ERR_NO_MEMORY, "SELL runs: out of device memory");
    int32_t hbad = 1;
    if (hipMemsetAsync(flag.p, 0, sizeof(int32_t), s) == hipSuccess) {
        hipLaunchKernelGGL(k_runs_widths, dim3(grid1d(S->nslices, di)), dim3(256), 0, s, S->nslices, S->sptr,
                           flag.as<int32_t>());
        if (S->f32)
            hipLaunchKernelGGL((k_sell_runs<float>), dim3(grid1d(nruns * kSlice, di)), dim3(256), 0, s, S->n, nruns,
                               S->col, (const float *)S->val, c3, flag.as<int32_t>());
        else
            hipLaunchKernelGGL((k_sell_runs<double>), dim3(grid1d(nruns * kSlice, di)), dim3(256), 0, s, S->n, nruns,
                               S->col, (const double *)S->val, c3, flag.as<int32_t>());
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(&hbad, flag.p, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            pool_free(c3);
            return set_error_code(AFSAI_ERR_HIP, "SELL runs: conversion failed");
        }
    }
    if (hbad) {
        pool_free(c3);
        return AFSAI_OK;
    }
    if (!keep_col) {
        pool_free(S->col);
        S->col = nullptr;
    }
    S->col3 = c3;
    return AFSAI_OK;
}

int sell_from_csr(int n, int64_t nnz, const int32_t *rp, const int32_t *ci, const void *val, bool val_f32,
                  bool out_f32, Sell *out, const DeviceInfo &di, hipStream_t s, const Segments &seg) {
    return sell_build(n, nnz, rp, nullptr, 0, ci, val, val_f32, out_f32, true, out, di, s, seg);
}

int sell_from_ell(int n, int64_t nnz, int ld, const int32_t *m, const int32_t *ell_col, const double *ell_val,
                  bool out_f32, Sell *out, const DeviceInfo &di, hipStream_t s, const Segments &seg) {
    return sell_build(n, nnz, nullptr, m, ld, ell_col, ell_val, false, out_f32, true, out, di, s, seg);
}

}  // namespace afsai
