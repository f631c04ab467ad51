// Host side of the adaptive FSAI setup: row statistics and validation, the launches of the fused
// per-row kernel (rows.hpp), and the assembly of G and G^T as CSR from its padded per-row
// results.  Rows are taken from per-XCD work counters (dynamic scheduling inside one
// contiguous range of rows per XCD).  A row whose candidate set overflows its on-chip table is
// reported and redone by a second launch with a table large enough for any pattern.
#include <cmath>
#include <vector>

#include "common.hpp"

#include "rows.hpp"

namespace afsai {

// ---------------------------------------------------------------------------------------
// row statistics (max row length) and optional structural / symmetry validation
// ---------------------------------------------------------------------------------------
struct ScanOut {
    int32_t maxlen;
    int32_t bad;       // structural problem found
    int32_t asym;      // asymmetric pair found
    int32_t nodiag;    // rows without a diagonal entry
};

// max row length, diagonal of every row (binary search in the ascending row) and, when
// validating, structure and exact symmetry
__global__ void k_row_scan(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                           const double *__restrict__ av, int validate, double *__restrict__ diag, ScanOut *out) {
    int lmax = 0, nodiag = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int a = rp[i], b = rp[i + 1];
        lmax = max(lmax, b - a);
        {
            int lo = a, hi = b - 1;
            double d = 0.0;
            bool found = false;
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                const int cm = ci[mid];
                if (cm == i) {
                    d = av[mid];
                    found = true;
                    break;
                }
                if (cm < i) lo = mid + 1; else hi = mid - 1;
            }
            diag[i] = d;
            nodiag += found ? 0 : 1;
        }
        if (!validate) continue;
        if (b < a) {
            atomicOr(&out->bad, 1);
            continue;
        }
        for (int e = a; e < b; ++e) {
            const int c = ci[e];
            if (c < 0 || c >= n || (e > a && c <= ci[e - 1])) {
                atomicOr(&out->bad, 1);
                break;
            }
            // symmetry: a_ci must exist and equal a_ic bit for bit
            int lo = rp[c], hi = rp[c + 1] - 1;
            bool ok = false;
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                const int cm = ci[mid];
                if (cm == i) {
                    ok = (__double_as_longlong(av[mid]) == __double_as_longlong(av[e]));
                    break;
                }
                if (cm < i) lo = mid + 1; else hi = mid - 1;
            }
            if (!ok) atomicOr(&out->asym, 1);
        }
    }
    lmax = wave_max(lmax);
    nodiag = wave_sum(nodiag);
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&out->maxlen, lmax);
        if (nodiag) atomicAdd(&out->nodiag, nodiag);
    }
}

__global__ void k_row_ptr_check(int n, const int32_t *__restrict__ rp, int nnz, ScanOut *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && (rp[0] != 0 || rp[n] != nnz)) atomicOr(&out->bad, 1);
    if (i < n && rp[i + 1] < rp[i]) atomicOr(&out->bad, 1);
}

// ---------------------------------------------------------------------------------------
// per-row status summary
// ---------------------------------------------------------------------------------------
struct Summary {
    int64_t nnz;
    int32_t nbad, nnotspd, novf;
    int32_t stop[3];
    double sumlog;  // not deterministic in order; diagnostics only
};

__global__ void k_summary(int n, const int32_t *__restrict__ m, const int8_t *__restrict__ st,
                          const int32_t *__restrict__ reason, const double *__restrict__ psi, Summary *out) {
    int64_t nnz = 0;
    int c_bad = 0, c_spd = 0, c_ovf = 0, c0 = 0, c1 = 0, c2 = 0;
    double sl = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        nnz += m[i];
        const int8_t s = st[i];
        c_bad += (s == ROW_BAD);
        c_spd += (s == ROW_NOT_SPD);
        c_ovf += (s == ROW_OVERFLOW);
        const int r = reason[i];
        c0 += (r == STOP_KMAX);
        c1 += (r == STOP_EPS);
        c2 += (r == STOP_NOCAND);
        if (s == ROW_OK) sl += log(psi[i]);
    }
    nnz = wave_sum(nnz);
    c_bad = wave_sum(c_bad);
    c_spd = wave_sum(c_spd);
    c_ovf = wave_sum(c_ovf);
    c0 = wave_sum(c0);
    c1 = wave_sum(c1);
    c2 = wave_sum(c2);
    sl = wave_sum(sl);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd((unsigned long long *)&out->nnz, (unsigned long long)nnz);
        atomicAdd(&out->nbad, c_bad);
        atomicAdd(&out->nnotspd, c_spd);
        atomicAdd(&out->novf, c_ovf);
        atomicAdd(&out->stop[0], c0);
        atomicAdd(&out->stop[1], c1);
        atomicAdd(&out->stop[2], c2);
        atomicAdd(&out->sumlog, sl);
    }
}

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

// ---------------------------------------------------------------------------------------
// assembly of G (CSR) from the padded per-row results, and of G^T
// ---------------------------------------------------------------------------------------
template <typename VT>
__global__ void k_fill_g(int n, int ldell, const int32_t *__restrict__ m, const int32_t *__restrict__ ell_col,
                         const double *__restrict__ ell_val, const int32_t *__restrict__ g_rp,
                         int32_t *__restrict__ g_ci, VT *__restrict__ g_val) {
    const int64_t total = (int64_t)n * ldell;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(k / ldell), t = (int)(k - (int64_t)i * ldell);
        if (t < m[i]) {
            const int64_t d = (int64_t)g_rp[i] + t;
            g_ci[d] = ell_col[k];
            g_val[d] = (VT)ell_val[k];
        }
    }
}

__global__ void k_count_cols(int nnz, const int32_t *__restrict__ ci, int32_t *__restrict__ cnt) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += gridDim.x * blockDim.x) atomicAdd(&cnt[ci[e]], 1);
}

template <typename VT>
__global__ void k_transpose_fill(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                 const VT *__restrict__ val, const int32_t *__restrict__ t_rp,
                                 int32_t *__restrict__ fill, int32_t *__restrict__ t_ci, VT *__restrict__ t_val) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            const int c = ci[e];
            const int d = t_rp[c] + atomicAdd(&fill[c], 1);
            t_ci[d] = i;
            t_val[d] = val[e];
        }
}

// each row of G^T sorted by column (= row of G): the atomic fill order is not deterministic
template <typename VT>
__global__ void k_sort_rows(int n, const int32_t *__restrict__ rp, int32_t *__restrict__ ci, VT *__restrict__ val) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int a = rp[i], b = rp[i + 1];
        for (int e = a + 1; e < b; ++e) {
            const int c = ci[e];
            const VT v = val[e];
            int f = e - 1;
            while (f >= a && ci[f] > c) {
                ci[f + 1] = ci[f];
                val[f + 1] = val[f];
                --f;
            }
            ci[f + 1] = c;
            val[f + 1] = v;
        }
    }
}

template <typename VT>
__global__ void k_widen(int64_t nnz, const VT *__restrict__ in, double *__restrict__ out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = (double)in[e];
}

__global__ void k_copy_i32(int64_t n, const int32_t *__restrict__ in, int32_t *__restrict__ out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = in[e];
}

template <typename VT>
__global__ void k_narrow(int64_t nnz, const double *__restrict__ in, VT *__restrict__ out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = (VT)in[e];
}

__global__ void k_fill_i32(int64_t n, int32_t *__restrict__ p, int32_t v) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) p[e] = v;
}

__global__ void k_row_counts(int n, const int32_t *__restrict__ rp, int32_t *__restrict__ cnt) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) cnt[i] = rp[i + 1] - rp[i];
}

// ---------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------
struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    template <typename T>
    T *as() { return (T *)p; }
    void *release() {
        void *q = p;
        p = nullptr;
        return q;
    }
};

static int dalloc(DevBuf &b, size_t bytes) {
    AFSAI_HIP_TRY(hipMalloc(&b.p, bytes ? bytes : 16));
    return AFSAI_OK;
}

static int grid1d(int64_t work, const DeviceInfo &di, int threads = 256) {
    int64_t b = (work + threads - 1) / threads;
    const int64_t cap = (int64_t)di.num_cus * 16;
    if (b > cap) b = cap;
    return (int)(b < 1 ? 1 : b);
}

// exclusive scan cnt[0..n) -> out[0..n]; returns the total through *total (host)
static int scan_counts(int n, const int32_t *cnt, int32_t *out, int64_t *total, const DeviceInfo &di,
                       hipStream_t s) {
    (void)di;
    const int ntiles = (int)(((int64_t)n + kScanTile - 1) / kScanTile);
    DevBuf ts, tot;
    int rc;
    if ((rc = dalloc(ts, sizeof(int64_t) * (size_t)(ntiles + 1)))) return rc;
    if ((rc = dalloc(tot, sizeof(int64_t)))) return rc;
    hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(kScanThreads), 0, s, n, cnt, ts.as<int64_t>());
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, s, ntiles, ts.as<int64_t>(), tot.as<int64_t>());
    hipLaunchKernelGGL(k_scan_apply, dim3(ntiles), dim3(kScanThreads), 0, s, n, cnt, ts.as<int64_t>(), out);
    AFSAI_HIP_TRY(hipMemcpyAsync(total, tot.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    AFSAI_HIP_TRY(hipStreamSynchronize(s));
    return AFSAI_OK;
}

// fused per-row kernels, instantiated in rows_reg.hip and rows_lds.hip
RowsKernel rows_kernel_reg(int mmax_t, int cap);
RowsKernel rows_kernel_lds(int mmax_t, int cap);

// register form for patterns of at most 32 entries and s <= kRegSMax; LDS form otherwise
static RowsKernel rows_kernel(int mmax_t, int cap, bool reg) {
    return reg ? rows_kernel_reg(mmax_t, cap) : rows_kernel_lds(mmax_t, cap);
}

static int pow2ceil(int64_t v) {
    int64_t p = 1;
    while (p < v) p <<= 1;
    return (int)p;
}

static size_t rows_lds_bytes(int mmax_t, int cap, bool reg) {
    const size_t tri = (size_t)mmax_t * (mmax_t + 1) / 2;
    return (size_t)cap * 12 + tri * 8 * (reg ? 1 : 2) + (reg ? (size_t)kRegSMax * mmax_t * 8 : 0) +
           (size_t)mmax_t * 32 + 65 * 4 + 64 * 16 + 16;
}

static int launch_rows(RowsKernel kern, int mmax_t, int cap, bool reg, const afsai_csr *A, const double *diag,
                       const afsai_params *p, const int32_t *list, int nlist, int32_t *counters, int ldell,
                       int32_t *ell_col, double *ell_val, int32_t *m, double *psi, int32_t *steps, int32_t *reason,
                       int8_t *st, int32_t *ovf_count, int32_t *ovf_list, const DeviceInfo &di, hipStream_t s) {
    const size_t lds = rows_lds_bytes(mmax_t, cap, reg);
    int per_cu = (int)((160 * 1024) / (lds + 256));
    if (per_cu > 32) per_cu = 32;
    if (per_cu < 1) per_cu = 1;
    int64_t nb = (int64_t)di.num_cus * per_cu;
    if (nb > nlist) nb = nlist;
    const int nx = di.num_xcds;
    nb = ((nb + nx - 1) / nx) * nx;
    if (nb < nx) nb = nx;
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, (int64_t)nx, counters, 0);
    {
        ProfScope ps("afsai_rows", s);
        hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(64), 0, s, A->n, A->row_ptr, A->col_idx, A->val, diag,
                           p->kmax, p->s, p->eps, p->tie_rtol, list, nlist, counters, nx, ell_col, ell_val, ldell, m,
                           psi, steps, reason, st, ovf_count, ovf_list);
    }
    AFSAI_HIP_TRY(hipGetLastError());
    return AFSAI_OK;
}

// builds G^T (CSR, rows sorted) from G
template <typename VT>
static int build_transpose(afsai_precond_s *P, const DeviceInfo &di, hipStream_t s) {
    const int n = P->n;
    const int64_t nnz = P->nnz_g;
    DevBuf cnt, rp, ci, val;
    int rc;
    if ((rc = dalloc(cnt, sizeof(int32_t) * (size_t)n))) return rc;
    if ((rc = dalloc(rp, sizeof(int32_t) * (size_t)(n + 1)))) return rc;
    if ((rc = dalloc(ci, sizeof(int32_t) * (size_t)nnz))) return rc;
    if ((rc = dalloc(val, sizeof(VT) * (size_t)nnz))) return rc;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid1d(n, di)), dim3(256), 0, s, (int64_t)n, cnt.as<int32_t>(), 0);
    hipLaunchKernelGGL(k_count_cols, dim3(grid1d(nnz, di)), dim3(256), 0, s, (int)nnz, P->g_ci, cnt.as<int32_t>());
    int64_t tot = 0;
    if ((rc = scan_counts(n, cnt.as<int32_t>(), rp.as<int32_t>(), &tot, di, s))) return rc;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid1d(n, di)), dim3(256), 0, s, (int64_t)n, cnt.as<int32_t>(), 0);
    hipLaunchKernelGGL((k_transpose_fill<VT>), dim3(grid1d(n, di)), dim3(256), 0, s, n, P->g_rp, P->g_ci,
                       (const VT *)P->g_val, rp.as<int32_t>(), cnt.as<int32_t>(), ci.as<int32_t>(), val.as<VT>());
    hipLaunchKernelGGL((k_sort_rows<VT>), dim3(grid1d(n, di)), dim3(256), 0, s, n, rp.as<int32_t>(), ci.as<int32_t>(),
                       val.as<VT>());
    AFSAI_HIP_TRY(hipGetLastError());
    P->gt_rp = (int32_t *)rp.release();
    P->gt_ci = (int32_t *)ci.release();
    P->gt_val = val.release();
    return AFSAI_OK;
}

static void free_handle(afsai_precond_s *P) {
    if (!P) return;
    (void)hipFree(P->g_rp);
    (void)hipFree(P->g_ci);
    (void)hipFree(P->g_val);
    (void)hipFree(P->gt_rp);
    (void)hipFree(P->gt_ci);
    (void)hipFree(P->gt_val);
    (void)hipFree(P->psi);
    (void)hipFree(P->steps);
    (void)hipFree(P->reason);
    (void)hipFree(P->work);
    delete P;
}

static int alloc_workspace(afsai_precond_s *P, const DeviceInfo &di) {
    // PCG: r, z, p, q, t (n each) + partial sums + scalars (must cover the solver's layout)
    const size_t np = (size_t)2 * di.num_cus * 8 + 64;
    P->work_elems = (size_t)5 * P->n + np + 16;
    AFSAI_HIP_TRY(hipMalloc(&P->work, P->work_elems * sizeof(double)));
    return AFSAI_OK;
}

}  // namespace afsai

using namespace afsai;

extern "C" {

int afsai_setup(const afsai_csr *A, const afsai_params *p, void *stream, afsai_precond *out) {
    clear_error();
    if (out) *out = nullptr;
    if (!A || !p || !out) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_setup: null argument");
    if (A->n <= 0 || A->nnz < A->n) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_setup: n = %d, nnz = %d", A->n, A->nnz);
    if (!A->row_ptr || !A->col_idx || !A->val) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_setup: null CSR array");
    if (p->kmax < 0 || (p->kmax > 0 && p->s < 1) || !(p->eps >= 0.0) || !(p->tie_rtol >= 0.0 && p->tie_rtol < 1.0) ||
        (p->g_prec != AFSAI_F64 && p->g_prec != AFSAI_F32) || (p->flags & ~AFSAI_VALIDATE))
        AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_setup: bad parameters (kmax=%d s=%d eps=%g tie_rtol=%g g_prec=%d)",
                   p->kmax, p->s, p->eps, p->tie_rtol, p->g_prec);
    const int64_t mmax64 = 1 + (int64_t)p->kmax * (p->kmax > 0 ? p->s : 0);
    if (mmax64 > 64) AFSAI_FAIL(AFSAI_ERR_TOO_LARGE, "afsai_setup: 1 + kmax*s = %lld exceeds 64", (long long)mmax64);
    const int mmax = (int)mmax64;
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t t0, t1;
    AFSAI_HIP_TRY(hipEventCreate(&t0));
    AFSAI_HIP_TRY(hipEventCreate(&t1));
    AFSAI_HIP_TRY(hipEventRecord(t0, s));
    const int n = A->n;

    // ---- row statistics / validation
    DevBuf scanb;
    if ((rc = dalloc(scanb, sizeof(ScanOut)))) return rc;
    AFSAI_HIP_TRY(hipMemsetAsync(scanb.p, 0, sizeof(ScanOut), s));
    const int validate = (p->flags & AFSAI_VALIDATE) ? 1 : 0;
    if (validate)
        hipLaunchKernelGGL(k_row_ptr_check, dim3((n + 256) / 256), dim3(256), 0, s, n, A->row_ptr, A->nnz,
                           scanb.as<ScanOut>());
    ScanOut so{};
    if (validate) {
        // row pointers must be sane before rows are scanned
        AFSAI_HIP_TRY(hipMemcpyAsync(&so, scanb.p, sizeof so, hipMemcpyDeviceToHost, s));
        AFSAI_HIP_TRY(hipStreamSynchronize(s));
        if (so.bad) AFSAI_FAIL(AFSAI_ERR_BAD_MATRIX, "afsai_setup: row pointers are not monotone from 0 to nnz");
    }
    DevBuf diagb;
    if ((rc = dalloc(diagb, sizeof(double) * (size_t)n))) return rc;
    hipLaunchKernelGGL(k_row_scan, dim3(grid1d(n, di)), dim3(256), 0, s, n, A->row_ptr, A->col_idx, A->val, validate,
                       diagb.as<double>(), scanb.as<ScanOut>());
    AFSAI_HIP_TRY(hipMemcpyAsync(&so, scanb.p, sizeof so, hipMemcpyDeviceToHost, s));
    AFSAI_HIP_TRY(hipStreamSynchronize(s));
    AFSAI_HIP_TRY(hipGetLastError());
    if (so.bad) AFSAI_FAIL(AFSAI_ERR_BAD_MATRIX, "afsai_setup: CSR structure invalid (columns unsorted, duplicate, out of range, or a missing diagonal)");
    if (so.asym) AFSAI_FAIL(AFSAI_ERR_BAD_MATRIX, "afsai_setup: matrix is not exactly symmetric");
    if (so.nodiag) AFSAI_FAIL(AFSAI_ERR_BAD_MATRIX, "afsai_setup: %d rows without a diagonal entry (or unsorted columns)", so.nodiag);
    const int maxlen = so.maxlen > 0 ? so.maxlen : 1;

    // ---- kernel shape: pattern capacity and candidate table size
    int mmax_t = 8;
    for (int c : {8, 16, 24, 32, 48, 64})
        if (c >= mmax) {
            mmax_t = c;
            break;
        }
    const bool reg = mmax <= 32 && (p->kmax == 0 || p->s <= kRegSMax) && !option(AFSAI_OPT_SETUP_FORM_LDS);
    // distinct columns one step can touch: at most every entry of the m pattern rows
    const int64_t bound = (int64_t)mmax * maxlen + mmax;
    // first table: about twice the distinct columns a step typically touches on stencil-like
    // matrices (an eighth of the bound), 128..1024 slots; rows that overflow it are redone with
    // a table larger than the bound (up to 8192 slots)
    int cap1 = pow2ceil(bound / 4 + 1);
    if (option(AFSAI_OPT_SETUP_TABLE) > 0) cap1 = pow2ceil(option(AFSAI_OPT_SETUP_TABLE));
    if (cap1 < 128) cap1 = 128;
    if (cap1 > 1024) cap1 = 1024;
    int cap2 = pow2ceil(bound + 1);
    if (cap2 < cap1) cap2 = cap1;
    if (cap2 > 8192) cap2 = 8192;

    // ---- per-row results (padded) and diagnostics
    const int ldell = mmax;
    DevBuf ell_col, ell_val, mcnt, psi, steps, reason, st, ctr, ovf;
    if ((rc = dalloc(ell_col, sizeof(int32_t) * (size_t)n * ldell))) return rc;
    if ((rc = dalloc(ell_val, sizeof(double) * (size_t)n * ldell))) return rc;
    if ((rc = dalloc(mcnt, sizeof(int32_t) * (size_t)n))) return rc;
    if ((rc = dalloc(psi, sizeof(double) * (size_t)n))) return rc;
    if ((rc = dalloc(steps, sizeof(int32_t) * (size_t)n))) return rc;
    if ((rc = dalloc(reason, sizeof(int32_t) * (size_t)n))) return rc;
    if ((rc = dalloc(st, sizeof(int8_t) * (size_t)n))) return rc;
    if ((rc = dalloc(ctr, sizeof(int32_t) * 16))) return rc;
    if ((rc = dalloc(ovf, sizeof(int32_t) * ((size_t)n + 1)))) return rc;
    int32_t *ovf_count = ovf.as<int32_t>() + n;
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, (int64_t)1, ovf_count, 0);

    RowsKernel k1 = rows_kernel(mmax_t, cap1, reg);
    if (!k1) AFSAI_FAIL(AFSAI_ERR_TOO_LARGE, "afsai_setup: no kernel for pattern %d / table %d", mmax_t, cap1);
    if ((rc = launch_rows(k1, mmax_t, cap1, reg, A, diagb.as<double>(), p, nullptr, n, ctr.as<int32_t>(), ldell, ell_col.as<int32_t>(),
                          ell_val.as<double>(), mcnt.as<int32_t>(), psi.as<double>(), steps.as<int32_t>(),
                          reason.as<int32_t>(), st.as<int8_t>(), ovf_count, ovf.as<int32_t>(), di, s)))
        return rc;
    int32_t novf = 0;
    AFSAI_HIP_TRY(hipMemcpyAsync(&novf, ovf_count, sizeof novf, hipMemcpyDeviceToHost, s));
    AFSAI_HIP_TRY(hipStreamSynchronize(s));
    int32_t retried = 0;
    if (novf > 0 && cap2 > cap1) {
        retried = novf;
        DevBuf list2;
        if ((rc = dalloc(list2, sizeof(int32_t) * ((size_t)novf + 1)))) return rc;
        hipLaunchKernelGGL(k_copy_i32, dim3(grid1d(novf, di)), dim3(256), 0, s, (int64_t)novf, ovf.as<int32_t>(),
                           list2.as<int32_t>());
        int32_t *cnt2 = list2.as<int32_t>() + novf;
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, (int64_t)1, cnt2, 0);
        RowsKernel k2 = rows_kernel(mmax_t, cap2, reg);
        if (!k2) AFSAI_FAIL(AFSAI_ERR_TOO_LARGE, "afsai_setup: no kernel for table %d", cap2);
        if ((rc = launch_rows(k2, mmax_t, cap2, reg, A, diagb.as<double>(), p, list2.as<int32_t>(), novf, ctr.as<int32_t>(), ldell,
                              ell_col.as<int32_t>(), ell_val.as<double>(), mcnt.as<int32_t>(), psi.as<double>(),
                              steps.as<int32_t>(), reason.as<int32_t>(), st.as<int8_t>(), cnt2, ovf.as<int32_t>(), di, s)))
            return rc;
        AFSAI_HIP_TRY(hipStreamSynchronize(s));
    }

    // ---- status summary
    DevBuf sumb;
    if ((rc = dalloc(sumb, sizeof(Summary)))) return rc;
    AFSAI_HIP_TRY(hipMemsetAsync(sumb.p, 0, sizeof(Summary), s));
    hipLaunchKernelGGL(k_summary, dim3(grid1d(n, di)), dim3(256), 0, s, n, mcnt.as<int32_t>(), st.as<int8_t>(),
                       reason.as<int32_t>(), psi.as<double>(), sumb.as<Summary>());
    Summary sm{};
    AFSAI_HIP_TRY(hipMemcpyAsync(&sm, sumb.p, sizeof sm, hipMemcpyDeviceToHost, s));
    AFSAI_HIP_TRY(hipStreamSynchronize(s));
    AFSAI_HIP_TRY(hipGetLastError());
    if (sm.nbad) AFSAI_FAIL(AFSAI_ERR_BAD_MATRIX, "afsai_setup: %d rows without a diagonal entry", sm.nbad);
    if (sm.nnotspd) AFSAI_FAIL(AFSAI_ERR_NOT_SPD, "afsai_setup: %d rows met a non-positive pivot (A not SPD)", sm.nnotspd);
    if (sm.novf) AFSAI_FAIL(AFSAI_ERR_TOO_LARGE, "afsai_setup: %d rows touch more candidate columns than fit on chip", sm.novf);
    if (sm.nnz >= ((int64_t)1 << 31)) AFSAI_FAIL(AFSAI_ERR_TOO_LARGE, "afsai_setup: nnz(G) = %lld exceeds int32", (long long)sm.nnz);

    // ---- G as CSR
    afsai_precond_s *P = new afsai_precond_s();
    P->device = di.device;
    P->n = n;
    P->mmax = mmax;
    P->g_prec = p->g_prec;
    auto fail = [&](int code) {
        free_handle(P);
        return code;
    };
    if (hipMalloc(&P->g_rp, sizeof(int32_t) * (size_t)(n + 1)) != hipSuccess) {
        set_error("afsai_setup: out of device memory");
        return fail(AFSAI_ERR_NO_MEMORY);
    }
    int64_t nnz = 0;
    if ((rc = scan_counts(n, mcnt.as<int32_t>(), P->g_rp, &nnz, di, s))) return fail(rc);
    P->nnz_g = nnz;
    const size_t vsz = (p->g_prec == AFSAI_F32) ? sizeof(float) : sizeof(double);
    if (hipMalloc(&P->g_ci, sizeof(int32_t) * (size_t)nnz) != hipSuccess ||
        hipMalloc(&P->g_val, vsz * (size_t)nnz) != hipSuccess) {
        set_error("afsai_setup: out of device memory for G");
        return fail(AFSAI_ERR_NO_MEMORY);
    }
    if (p->g_prec == AFSAI_F32)
        hipLaunchKernelGGL((k_fill_g<float>), dim3(grid1d((int64_t)n * ldell, di)), dim3(256), 0, s, n, ldell,
                           mcnt.as<int32_t>(), ell_col.as<int32_t>(), ell_val.as<double>(), P->g_rp, P->g_ci,
                           (float *)P->g_val);
    else
        hipLaunchKernelGGL((k_fill_g<double>), dim3(grid1d((int64_t)n * ldell, di)), dim3(256), 0, s, n, ldell,
                           mcnt.as<int32_t>(), ell_col.as<int32_t>(), ell_val.as<double>(), P->g_rp, P->g_ci,
                           (double *)P->g_val);
    AFSAI_HIP_TRY(hipGetLastError());
    rc = (p->g_prec == AFSAI_F32) ? build_transpose<float>(P, di, s) : build_transpose<double>(P, di, s);
    if (rc) return fail(rc);
    P->psi = (double *)psi.release();
    P->steps = (int32_t *)steps.release();
    P->reason = (int32_t *)reason.release();
    if ((rc = alloc_workspace(P, di))) return fail(rc);
    AFSAI_HIP_TRY(hipEventRecord(t1, s));
    AFSAI_HIP_TRY(hipStreamSynchronize(s));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, t0, t1);
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    prof_flush();

    afsai_setup_info &inf = P->info;
    inf.n = n;
    inf.mmax = mmax;
    inf.nnz_g = nnz;
    inf.g_prec = p->g_prec;
    inf.rows_stop_kmax = sm.stop[0];
    inf.rows_stop_eps = sm.stop[1];
    inf.rows_stop_nocand = sm.stop[2];
    inf.rows_retried = retried;
    inf.sum_log_psi = sm.sumlog;
    inf.ms = ms;
    *out = P;
    return AFSAI_OK;
}

int afsai_get_setup_info(afsai_precond P, afsai_setup_info *info) {
    if (!P || !info) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_get_setup_info: null argument");
    *info = P->info;
    return AFSAI_OK;
}

int afsai_export(afsai_precond P, int32_t *row_ptr, int32_t *col, double *val, void *stream) {
    if (!P) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_export: null handle");
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (row_ptr) AFSAI_HIP_TRY(hipMemcpyAsync(row_ptr, P->g_rp, sizeof(int32_t) * (size_t)(P->n + 1), hipMemcpyDeviceToDevice, s));
    if (col) AFSAI_HIP_TRY(hipMemcpyAsync(col, P->g_ci, sizeof(int32_t) * (size_t)P->nnz_g, hipMemcpyDeviceToDevice, s));
    if (val) {
        if (P->g_prec == AFSAI_F32)
            hipLaunchKernelGGL((k_widen<float>), dim3(grid1d(P->nnz_g, di)), dim3(256), 0, s, P->nnz_g,
                               (const float *)P->g_val, val);
        else
            AFSAI_HIP_TRY(hipMemcpyAsync(val, P->g_val, sizeof(double) * (size_t)P->nnz_g, hipMemcpyDeviceToDevice, s));
    }
    AFSAI_HIP_TRY(hipGetLastError());
    AFSAI_HIP_TRY(hipStreamSynchronize(s));
    return AFSAI_OK;
}

int afsai_export_rows(afsai_precond P, double *psi, int32_t *steps, int32_t *reason, void *stream) {
    if (!P) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_export_rows: null handle");
    if (!P->psi && (psi || steps || reason))
        AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_export_rows: imported preconditioners carry no row diagnostics");
    hipStream_t s = (hipStream_t)stream;
    if (psi) AFSAI_HIP_TRY(hipMemcpyAsync(psi, P->psi, sizeof(double) * (size_t)P->n, hipMemcpyDeviceToDevice, s));
    if (steps) AFSAI_HIP_TRY(hipMemcpyAsync(steps, P->steps, sizeof(int32_t) * (size_t)P->n, hipMemcpyDeviceToDevice, s));
    if (reason) AFSAI_HIP_TRY(hipMemcpyAsync(reason, P->reason, sizeof(int32_t) * (size_t)P->n, hipMemcpyDeviceToDevice, s));
    AFSAI_HIP_TRY(hipStreamSynchronize(s));
    return AFSAI_OK;
}

int afsai_import(const afsai_csr *G, int32_t g_prec, void *stream, afsai_precond *out) {
    clear_error();
    if (out) *out = nullptr;
    if (!G || !out) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_import: null argument");
    if (G->n <= 0 || G->nnz < 0 || !G->row_ptr || !G->col_idx || !G->val)
        AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_import: bad CSR");
    if (g_prec != AFSAI_F64 && g_prec != AFSAI_F32) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_import: bad g_prec");
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    afsai_precond_s *P = new afsai_precond_s();
    P->device = di.device;
    P->n = G->n;
    P->nnz_g = G->nnz;
    P->g_prec = g_prec;
    auto fail = [&](int code) {
        free_handle(P);
        return code;
    };
    const size_t vsz = (g_prec == AFSAI_F32) ? sizeof(float) : sizeof(double);
    if (hipMalloc(&P->g_rp, sizeof(int32_t) * (size_t)(G->n + 1)) != hipSuccess ||
        hipMalloc(&P->g_ci, sizeof(int32_t) * (size_t)(G->nnz ? G->nnz : 1)) != hipSuccess ||
        hipMalloc(&P->g_val, vsz * (size_t)(G->nnz ? G->nnz : 1)) != hipSuccess) {
        set_error("afsai_import: out of device memory");
        return fail(AFSAI_ERR_NO_MEMORY);
    }
    if (hipMemcpyAsync(P->g_rp, G->row_ptr, sizeof(int32_t) * (size_t)(G->n + 1), hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(P->g_ci, G->col_idx, sizeof(int32_t) * (size_t)G->nnz, hipMemcpyDeviceToDevice, s) != hipSuccess) {
        set_error("afsai_import: copy failed");
        return fail(AFSAI_ERR_HIP);
    }
    if (g_prec == AFSAI_F32)
        hipLaunchKernelGGL((k_narrow<float>), dim3(grid1d(G->nnz, di)), dim3(256), 0, s, (int64_t)G->nnz, G->val,
                           (float *)P->g_val);
    else if (hipMemcpyAsync(P->g_val, G->val, sizeof(double) * (size_t)G->nnz, hipMemcpyDeviceToDevice, s) != hipSuccess) {
        set_error("afsai_import: copy failed");
        return fail(AFSAI_ERR_HIP);
    }
    rc = (g_prec == AFSAI_F32) ? build_transpose<float>(P, di, s) : build_transpose<double>(P, di, s);
    if (rc) return fail(rc);
    if ((rc = alloc_workspace(P, di))) return fail(rc);
    if (hipStreamSynchronize(s) != hipSuccess) {
        set_error("afsai_import: synchronisation failed");
        return fail(AFSAI_ERR_HIP);
    }
    P->mmax = 0;
    P->info.n = P->n;
    P->info.nnz_g = P->nnz_g;
    P->info.g_prec = g_prec;
    *out = P;
    return AFSAI_OK;
}

void afsai_destroy(afsai_precond P) {
    if (!P) return;
    (void)hipDeviceSynchronize();
    free_handle(P);
}

}  // extern "C"
