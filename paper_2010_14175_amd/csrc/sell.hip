// Device scan and the SELL-64 layout used by the PCG products (sell.hpp).
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
// SELL-64 construction
// ---------------------------------------------------------------------------------------
// rows sorted by length (longest first, ties by row index) inside windows of kSortWindow rows;
// one block per window, bitonic sort of (length, row) keys in LDS
__global__ __launch_bounds__(1024) void k_sell_sort(int n, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ m, int32_t *__restrict__ perm) {
    __shared__ unsigned long long key[kSortWindow];
    const int w0 = blockIdx.x * kSortWindow;
    for (int j = threadIdx.x; j < kSortWindow; j += blockDim.x) {
        const int r = w0 + j;
        unsigned long long k = ~0ull;
        if (r < n) {
            const uint32_t len = (uint32_t)(rp ? rp[r + 1] - rp[r] : m[r]);
            k = ((unsigned long long)(0xFFFFFFFFu - len) << 32) | (uint32_t)j;
        }
        key[j] = k;
    }
    __syncthreads();
    for (int size = 2; size <= kSortWindow; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < kSortWindow / 2; t += blockDim.x) {
                const int lo = 2 * t - (t & (stride - 1));
                const int hi = lo + stride;
                const bool up = ((lo & size) == 0);
                const unsigned long long a = key[lo], b = key[hi];
                if ((a > b) == up) {
                    key[lo] = b;
                    key[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    for (int j = threadIdx.x; j < kSortWindow; j += blockDim.x) {
        const unsigned long long k = key[j];
        const int r = w0 + j;
        if (r < ((n + kSlice - 1) / kSlice) * kSlice)
            perm[r] = (k == ~0ull) ? -1 : w0 + (int)(k & 0xFFFFFFFFu);
    }
}

// width of each slice = longest row in it (one wavefront per slice)
__global__ __launch_bounds__(256) void k_sell_width(int n, int nslices, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ m, const int32_t *__restrict__ perm,
                                                     int32_t *__restrict__ width) {
    const int lane = threadIdx.x & 63;
    for (int sl = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; sl < nslices; sl += (gridDim.x * blockDim.x) >> 6) {
        int r = sl * kSlice + lane;
        if (perm) r = perm[r];
        int len = 0;
        if (r >= 0 && r < n) len = rp ? rp[r + 1] - rp[r] : m[r];
        len = wave_max(len);
        if (lane == 0) width[sl] = len;
    }
}

// one wavefront per slice; lane = row; padding entries are (own row, 0)
template <typename VI, typename VO>
__global__ __launch_bounds__(256) void k_sell_fill(int n, int nslices, const int32_t *__restrict__ rp,
                                                    const int32_t *__restrict__ m, int ld,
                                                    const int32_t *__restrict__ ci, const VI *__restrict__ val,
                                                    const int32_t *__restrict__ perm,
                                                    const int32_t *__restrict__ sptr, int32_t *__restrict__ col,
                                                    VO *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    for (int sl = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; sl < nslices; sl += (gridDim.x * blockDim.x) >> 6) {
        int r = sl * kSlice + lane;
        if (perm) r = perm[r];
        int len = 0;
        int64_t start = 0;
        const bool valid = r >= 0 && r < n;
        if (valid) {
            if (rp) {
                start = rp[r];
                len = rp[r + 1] - rp[r];
            } else {
                start = (int64_t)r * ld;
                len = m[r];
            }
        }
        const int pad_col = valid ? r : n - 1;
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
                if (k < len) {
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

void sell_free(Sell *S) {
    if (!S) return;
    pool_free(S->sptr);
    pool_free(S->col);
    pool_free(S->val);
    pool_free(S->perm);
    *S = Sell();
}

static int sell_build(int n, int64_t nnz_in, const int32_t *rp, const int32_t *m, int ld, const int32_t *ci,
                      const void *val, bool val_f32, bool out_f32, Sell *out, const DeviceInfo &di, hipStream_t s) {
    Sell S;
    S.n = n;
    S.nslices = (n + kSlice - 1) / kSlice;
    S.f32 = out_f32;
    DevBuf width;
    int rc;
    if ((rc = dalloc(width, sizeof(int32_t) * (size_t)S.nslices, s))) return rc;
    const int nbs = grid1d((int64_t)S.nslices * 64, di);
    S.sptr = (uint32_t *)pool_alloc(sizeof(uint32_t) * (size_t)(S.nslices + 1));
    if (!S.sptr) AFSAI_FAIL(AFSAI_ERR_NO_MEMORY, "SELL layout: out of device memory");
    // stored entries of the plain layout
    hipLaunchKernelGGL(k_sell_width, dim3(nbs), dim3(256), 0, s, n, S.nslices, rp, m, nullptr, width.as<int32_t>());
    int64_t cols = 0;
    if ((rc = scan_counts(S.nslices, width.as<int32_t>(), (int32_t *)S.sptr, &cols, di, s))) {
        sell_free(&S);
        return rc;
    }
    // per-row results (rp == nullptr) have rows of nearly equal length: never sorted
    const int64_t nnz = rp ? nnz_in : cols * kSlice;
    if (cols * kSlice > nnz + nnz / 10 && n > kSlice) {
        // rows of very different lengths: sort by length inside windows, then re-measure
        S.perm = (int32_t *)pool_alloc(sizeof(int32_t) * (size_t)S.nslices * kSlice);
        if (!S.perm) {
            sell_free(&S);
            AFSAI_FAIL(AFSAI_ERR_NO_MEMORY, "SELL layout: out of device memory");
        }
        const int nwin = (n + kSortWindow - 1) / kSortWindow;
        hipLaunchKernelGGL(k_sell_sort, dim3(nwin), dim3(1024), 0, s, n, rp, m, S.perm);
        hipLaunchKernelGGL(k_sell_width, dim3(nbs), dim3(256), 0, s, n, S.nslices, rp, m, S.perm,
                           width.as<int32_t>());
        if ((rc = scan_counts(S.nslices, width.as<int32_t>(), (int32_t *)S.sptr, &cols, di, s))) {
            sell_free(&S);
            return rc;
        }
    }
    if (cols >= ((int64_t)1 << 31)) {
        sell_free(&S);
        AFSAI_FAIL(AFSAI_ERR_TOO_LARGE, "SELL layout: %lld columns", (long long)cols);
    }
    S.entries = cols * kSlice;
    S.col = (int32_t *)pool_alloc(sizeof(int32_t) * (size_t)S.entries);
    S.val = pool_alloc((out_f32 ? sizeof(float) : sizeof(double)) * (size_t)S.entries);
    if (!S.col || !S.val) {
        sell_free(&S);
        AFSAI_FAIL(AFSAI_ERR_NO_MEMORY, "SELL layout: out of device memory");
    }
    const int32_t *sp = (const int32_t *)S.sptr;
    if (val_f32) {
        if (out_f32)
            hipLaunchKernelGGL((k_sell_fill<float, float>), dim3(nbs), dim3(256), 0, s, n, S.nslices, rp, m, ld, ci,
                               (const float *)val, S.perm, sp, S.col, (float *)S.val);
        else
            hipLaunchKernelGGL((k_sell_fill<float, double>), dim3(nbs), dim3(256), 0, s, n, S.nslices, rp, m, ld, ci,
                               (const float *)val, S.perm, sp, S.col, (double *)S.val);
    } else {
        if (out_f32)
            hipLaunchKernelGGL((k_sell_fill<double, float>), dim3(nbs), dim3(256), 0, s, n, S.nslices, rp, m, ld, ci,
                               (const double *)val, S.perm, sp, S.col, (float *)S.val);
        else
            hipLaunchKernelGGL((k_sell_fill<double, double>), dim3(nbs), dim3(256), 0, s, n, S.nslices, rp, m, ld,
                               ci, (const double *)val, S.perm, sp, S.col, (double *)S.val);
    }
    if (hipGetLastError() != hipSuccess) {
        sell_free(&S);
        AFSAI_FAIL(AFSAI_ERR_HIP, "SELL layout: launch failed");
    }
    *out = S;
    return AFSAI_OK;
}

int sell_from_csr(int n, int64_t nnz, const int32_t *rp, const int32_t *ci, const void *val, bool val_f32,
                  bool out_f32, Sell *out, const DeviceInfo &di, hipStream_t s) {
    return sell_build(n, nnz, rp, nullptr, 0, ci, val, val_f32, out_f32, out, di, s);
}

int sell_from_ell(int n, int ld, const int32_t *m, const int32_t *ell_col, const double *ell_val, bool out_f32,
                  Sell *out, const DeviceInfo &di, hipStream_t s) {
    return sell_build(n, 0, nullptr, m, ld, ell_col, ell_val, false, out_f32, out, di, s);
}

}  // namespace afsai
