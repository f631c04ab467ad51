// Host side of the adaptive FSAI setup: row statistics and validation, the launches of the fused
// per-row kernel (rows.hpp), and the assembly of G and G^T as CSR from its padded per-row
// results.  Rows are taken from per-XCD work counters (dynamic scheduling inside one
// contiguous range of rows per XCD).  A row whose candidate set overflows its on-chip table is
// reported and redone by a second launch with a table large enough for any pattern.
#include <cmath>
#include <vector>

#include "handle.hpp"
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

// max row length, diagonal of every row and the number of entries left of it (binary search
// in the ascending row) and, when validating, structure and exact symmetry
__global__ void k_row_scan(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                           const double *__restrict__ av, int validate, double *__restrict__ diag,
                           int32_t *__restrict__ dlo, ScanOut *out) {
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
                    lo = mid;
                    break;
                }
                if (cm < i) lo = mid + 1; else hi = mid - 1;
            }
            diag[i] = d;
            dlo[i] = found ? lo - a : 0;
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
// per-row status summary (two stages, fixed order: deterministic)
// ---------------------------------------------------------------------------------------
struct Summary {
    int64_t nnz;
    int64_t nbad, nnotspd, novf;
    int64_t stop[3];
    double sumlog;
};

__device__ __forceinline__ void summary_add(Summary &a, const Summary &b) {
    a.nnz += b.nnz;
    a.nbad += b.nbad;
    a.nnotspd += b.nnotspd;
    a.novf += b.novf;
    for (int k = 0; k < 3; ++k) a.stop[k] += b.stop[k];
    a.sumlog += b.sumlog;
}

__device__ Summary block_summary(Summary v) {
    __shared__ Summary sh[4];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        v.nnz += __shfl_xor(v.nnz, off, 64);
        v.nbad += __shfl_xor(v.nbad, off, 64);
        v.nnotspd += __shfl_xor(v.nnotspd, off, 64);
        v.novf += __shfl_xor(v.novf, off, 64);
        for (int k = 0; k < 3; ++k) v.stop[k] += __shfl_xor(v.stop[k], off, 64);
        v.sumlog += __shfl_xor(v.sumlog, off, 64);
    }
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    Summary t{};
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) summary_add(t, sh[w]);
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(256) void k_summary(int n, const int32_t *__restrict__ m, const int8_t *__restrict__ st,
                                                 const int32_t *__restrict__ reason, const double *__restrict__ psi,
                                                 Summary *part) {
    Summary v{};
    const int64_t per = ((int64_t)n + gridDim.x - 1) / gridDim.x;
    const int i0 = (int)min<int64_t>(n, per * blockIdx.x), i1 = (int)min<int64_t>(n, per * (blockIdx.x + 1));
    for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        v.nnz += m[i];
        const int8_t s = st[i];
        v.nbad += (s == ROW_BAD);
        v.nnotspd += (s == ROW_NOT_SPD);
        v.novf += (s == ROW_OVERFLOW);
        const int r = reason[i];
        v.stop[0] += (r == STOP_KMAX);
        v.stop[1] += (r == STOP_EPS);
        v.stop[2] += (r == STOP_NOCAND);
        if (s == ROW_OK) v.sumlog += log(psi[i]);
    }
    Summary t = block_summary(v);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// sums the block partials: thread t adds a contiguous run in order, then the runs are added
// in thread order (fixed shape: deterministic)
__global__ __launch_bounds__(256) void k_summary_final(int nparts, const Summary *__restrict__ part, Summary *out) {
    const int per = (nparts + 255) / 256;
    const int lo = threadIdx.x * per, hi = min(nparts, lo + per);
    Summary v{};
    for (int k = lo; k < hi; ++k) summary_add(v, part[k]);
    Summary t = block_summary(v);
    if (threadIdx.x == 0) *out = t;
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

// entry (i, c) of G goes to row c of G^T at a slot taken with an atomic counter (the order
// within a row is fixed afterwards by k_sort_rows); one wavefront per row of G, one lane per entry
template <typename VT>
__global__ __launch_bounds__(256) void k_transpose_fill(int n, const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ ci, const VT *__restrict__ val,
                                                        const int32_t *__restrict__ t_rp, int32_t *__restrict__ fill,
                                                        int32_t *__restrict__ t_ci, VT *__restrict__ t_val) {
    const int lane = threadIdx.x & 63;
    for (int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < n; i += (gridDim.x * blockDim.x) >> 6) {
        const int a = rp[i], b = rp[i + 1];
        for (int e = a + lane; e < b; e += 64) {
            const int c = ci[e];
            const int d = t_rp[c] + atomicAdd(&fill[c], 1);
            t_ci[d] = i;
            t_val[d] = val[e];
        }
    }
}

// An entry of G^T as the fill leaves it: (row of G, value) in one 8- or 16-byte word, so that
// each entry is one scattered store instead of two
template <typename VT>
struct TPair;
template <>
struct alignas(8) TPair<float> {
    int32_t i;
    float v;
};
template <>
struct alignas(16) TPair<double> {
    int32_t i, pad;
    double v;
};

// The same from the padded per-row results (ld slots per row, m[i] valid): one thread per slot,
// so every entry's slot reservation is independent of the others (the row is slot / ld); the
// entries go to `pr` as pairs, which k_sort_rows splits into columns and values
template <typename VT>
__global__ __launch_bounds__(256) void k_transpose_fill_ell(int n, int ld, const int32_t *__restrict__ m,
                                                            const int32_t *__restrict__ ell_col,
                                                            const double *__restrict__ ell_val,
                                                            const int32_t *__restrict__ t_rp,
                                                            int32_t *__restrict__ fill, TPair<VT> *__restrict__ pr) {
    const int64_t total = (int64_t)n * ld;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(k / ld), t = (int)(k - (int64_t)i * ld);
        if (t < m[i]) {
            const int c = ell_col[k];
            const int d = t_rp[c] + atomicAdd(&fill[c], 1);
            TPair<VT> e;
            if constexpr (sizeof(VT) == 8) e.pad = 0;
            e.i = i;
            e.v = (VT)ell_val[k];
            pr[d] = e;
        }
    }
}

// entry e of a row of G^T before sorting: from the pairs of the fill when given, else in place
template <typename VT>
__device__ __forceinline__ void sort_load(const int32_t *ci, const VT *val, const TPair<VT> *pr, int64_t e, int &k,
                                          VT &v) {
    if (pr) {
        const TPair<VT> q = pr[e];
        k = q.i;
        v = q.v;
    } else {
        k = ci[e];
        v = val[e];
    }
}

// Sorts every row of G^T by column (= row of G), reading the rows from the fill's pairs (pr)
// or in place (pr null).  One wavefront per row: rows of up to 256 entries are ranked in
// registers (each lane counts the smaller keys, one, two or four keys per lane); longer rows
// fall back to an insertion sort by one lane.
template <typename VT>
__global__ __launch_bounds__(256) void k_sort_rows(int n, const int32_t *__restrict__ rp, int32_t *__restrict__ ci,
                                                   VT *__restrict__ val, const TPair<VT> *__restrict__ pr) {
    const int lane = threadIdx.x & 63;
    for (int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < n; i += (gridDim.x * blockDim.x) >> 6) {
        const int a = rp[i], b = rp[i + 1], len = b - a;
        if (len <= 64) {
            int key = 0x7fffffff;
            VT v = VT(0);
            if (lane < len) sort_load(ci, val, pr, a + lane, key, v);
            int rank = 0;
            for (int t = 0; t < len; ++t) rank += (__shfl(key, t, 64) < key) ? 1 : 0;
            if (lane < len) {
                ci[a + rank] = key;
                val[a + rank] = v;
            }
        } else if (len <= 128) {
            // two keys per lane (the columns of a row are distinct, so the ranks are too)
            int k0, k1 = 0x7fffffff;
            VT v0, v1 = VT(0);
            sort_load(ci, val, pr, a + lane, k0, v0);
            if (lane + 64 < len) sort_load(ci, val, pr, a + 64 + lane, k1, v1);
            int r0 = 0, r1 = 0;
            for (int t = 0; t < 64; ++t) {
                const int kt = __shfl(k0, t, 64);
                r0 += (kt < k0) ? 1 : 0;
                r1 += (kt < k1) ? 1 : 0;
            }
            for (int t = 0; t < len - 64; ++t) {
                const int kt = __shfl(k1, t, 64);
                r0 += (kt < k0) ? 1 : 0;
                r1 += (kt < k1) ? 1 : 0;
            }
            ci[a + r0] = k0;
            val[a + r0] = v0;
            if (lane + 64 < len) {
                ci[a + r1] = k1;
                val[a + r1] = v1;
            }
        } else if (len <= 256) {
            // four keys per lane (rows of G^T past 128 entries: columns chosen by many rows)
            int k[4];
            VT v[4];
            int r[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int o = lane + 64 * j;
                k[j] = 0x7fffffff;
                v[j] = VT(0);
                r[j] = 0;
                if (o < len) sort_load(ci, val, pr, a + o, k[j], v[j]);
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int lim = min(64, len - 64 * c);
                for (int t = 0; t < lim; ++t) {
                    const int kt = __shfl(k[c], t, 64);
#pragma unroll
                    for (int j = 0; j < 4; ++j) r[j] += (kt < k[j]) ? 1 : 0;
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (lane + 64 * j < len) {
                    ci[a + r[j]] = k[j];
                    val[a + r[j]] = v[j];
                }
        } else if (lane == 0) {
            if (pr)
                for (int e = a; e < b; ++e) sort_load(ci, val, pr, e, ci[e], val[e]);
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

// batches: every row's first and last column lie inside its own system (rows ascending), so
// the matrix is block diagonal
__global__ void k_block_check(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, int nsys,
                              const int32_t *__restrict__ row0, ScanOut *out) {
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        int lo = 0, hi = nsys - 1;  // system k with row0[k] <= r < row0[k+1]
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (row0[mid] <= r) lo = mid; else hi = mid - 1;
        }
        const int a = rp[r], b = rp[r + 1];
        if (b > a && (ci[a] < row0[lo] || ci[b - 1] >= row0[lo + 1])) atomicOr(&out->bad, 1);
    }
}

// ---------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------
// fused per-row kernels, instantiated in rows.hip (Cholesky form) and rows_w.hip (inverse-factor form)
RowsKernel rows_kernel(int mmax_t, int cap, bool rsl, bool f32);
RowsKernel rows_kernel_w(int mmax, int maxlen, int cap, int lanes, bool g32, int *gs_out, size_t *lds_out);
RowsKernel rows_kernel_w_large(int mmax, int cap, bool g32, size_t *lds_out);

// Launch of a per-row kernel over `nlist` rows.  Inverse-factor form: wdyn > 0 is its dynamic
// LDS per block and rpw its rows per wavefront; the Cholesky form sizes its LDS from the
// pattern and table (wdyn = 0).
static int launch_rows(const char *prof_name, RowsKernel kern, size_t wdyn, int rpw, int mmax_t, int mmax, int64_t row_work, int cap, bool rsl, int tb, int gmax, const afsai_csr *A, const float *av32, const double *diag,
                       const int32_t *dlo, const afsai_params *p, const int32_t *list, int nlist, int32_t *counters,
                       int ldell, int32_t *ell_col, double *ell_val, int32_t *m, double *psi, int32_t *steps,
                       int32_t *reason, int8_t *st, int32_t *ovf_count, int32_t *ovf_list, const DeviceInfo &di,
                       hipStream_t s) {
    // resident rows per CU: the runtime's occupancy for this kernel (registers and LDS, with
    // its dynamic LDS), else from the LDS bytes (512-byte granules)
    const size_t lds = ((wdyn ? wdyn + 16 : rows_lds_bytes(mmax_t, mmax, cap, rsl, tb)) + 511) / 512 * 512;
    const size_t dyn = wdyn ? wdyn : rows_lds_dyn_bytes(mmax, rsl, tb);
    int per_cu = (int)((160 * 1024) / lds);
    if (dyn > 48 * 1024)
        AFSAI_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
    {
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void *>(kern), 64, dyn) ==
                hipSuccess &&
            occ > 0)
            per_cu = std::min(per_cu, occ);
        else
            (void)hipGetLastError();
    }
    if (per_cu > 32) per_cu = 32;
    if (per_cu < 1) per_cu = 1;
    int64_t nb = (int64_t)di.num_cus * per_cu;
    if (nb > (nlist + rpw - 1) / rpw) nb = (nlist + rpw - 1) / rpw;
    const int nx = di.num_xcds;
    nb = ((nb + nx - 1) / nx) * nx;
    if (nb < nx) nb = nx;
    // rows per claim (one atomic on the XCD's counter each): enough rows for about 4,000 table
    // entries of work, 1..16, and at most a quarter of a resident row-slot's share (short tail)
    // (claims are counted in wavefronts' worth of rows: rpw rows each)
    int64_t claim64 = (4000 + row_work * rpw - 1) / std::max<int64_t>(1, row_work * rpw);
    claim64 = std::min<int64_t>(claim64, std::max<int64_t>(1, nlist / ((int64_t)rpw * nb * 4)));
    int claim = (int)std::min<int64_t>(16, std::max<int64_t>(1, claim64));
    if (option(AFSAI_OPT_SETUP_CLAIM) > 0) claim = (int)option(AFSAI_OPT_SETUP_CLAIM);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, (int64_t)nx, counters, 0);
    {
        ProfScope ps(prof_name, s);
        hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(64), dyn, s, A->n, A->row_ptr, A->col_idx, A->val, av32, diag, dlo,
                           p->kmax, p->s, p->eps, p->tie_rtol, gmax, list, nlist, counters, nx, claim, ell_col, ell_val,
                           ldell, m, psi, steps, reason, st, ovf_count, ovf_list);
    }
    AFSAI_HIP_TRY(hipGetLastError());
    return AFSAI_OK;
}

static void free_handle(afsai_precond_s *P) {
    if (!P) return;
    pool_free(P->g_rp);
    pool_free(P->g_ci);
    pool_free(P->g_val);
    sell_free(&P->sg);
    sell_free(&P->sgt);
    pool_free(P->psi);
    pool_free(P->steps);
    pool_free(P->reason);
    pool_free(P->work);
    delete P;
}

// G^T as SELL-64, built from the CSR G of the handle (count, scan, fill, sort, convert); the
// fill reads the padded per-row results when given (ld slots per row, m[i] valid)
template <typename VT>
static int build_transpose(afsai_precond_s *P, const DeviceInfo &di, hipStream_t s, const Segments &seg,
                           int ld = 0, const int32_t *m = nullptr, const int32_t *ell_col = nullptr,
                           const double *ell_val = nullptr) {
    const int n = P->n;
    const int64_t nnz = P->nnz_g;
    DevBuf cnt, rp, ci, val;
    int rc;
    if ((rc = dalloc(cnt, sizeof(int32_t) * (size_t)n, s))) return rc;
    if ((rc = dalloc(rp, sizeof(int32_t) * (size_t)(n + 1), s))) return rc;
    if ((rc = dalloc(ci, sizeof(int32_t) * (size_t)nnz, s))) return rc;
    if ((rc = dalloc(val, sizeof(VT) * (size_t)nnz, s))) return rc;
    {
        ProfScope ps("transpose", s);
        hipLaunchKernelGGL(k_fill_i32, dim3(grid1d(n, di)), dim3(256), 0, s, (int64_t)n, cnt.as<int32_t>(), 0);
        hipLaunchKernelGGL(k_count_cols, dim3(grid1d(nnz, di)), dim3(256), 0, s, (int)nnz, P->g_ci, cnt.as<int32_t>());
    }
    int64_t tot = 0;
    if ((rc = scan_counts(n, cnt.as<int32_t>(), rp.as<int32_t>(), &tot, di, s))) return rc;
    {
        // the fill's pairs, released (after the sort) before the SELL layout takes its memory
        DevBuf pairs;
        if (ell_col && (rc = dalloc(pairs, sizeof(TPair<VT>) * (size_t)nnz, s))) return rc;
        ProfScope ps("transpose", s);
        hipLaunchKernelGGL(k_fill_i32, dim3(grid1d(n, di)), dim3(256), 0, s, (int64_t)n, cnt.as<int32_t>(), 0);
        if (ell_col)
            hipLaunchKernelGGL((k_transpose_fill_ell<VT>), dim3(grid1d((int64_t)n * ld, di)), dim3(256), 0, s, n, ld,
                               m, ell_col, ell_val, rp.as<int32_t>(), cnt.as<int32_t>(), (TPair<VT> *)pairs.p);
        else
            hipLaunchKernelGGL((k_transpose_fill<VT>), dim3(grid1d((int64_t)n * 64, di)), dim3(256), 0, s, n,
                               P->g_rp, P->g_ci, (const VT *)P->g_val, rp.as<int32_t>(), cnt.as<int32_t>(),
                               ci.as<int32_t>(), val.as<VT>());
        hipLaunchKernelGGL((k_sort_rows<VT>), dim3(grid1d((int64_t)n * 64, di)), dim3(256), 0, s, n, rp.as<int32_t>(),
                           ci.as<int32_t>(), val.as<VT>(), (const TPair<VT> *)pairs.p);
    }
    AFSAI_HIP_TRY(hipGetLastError());
    const bool f32 = sizeof(VT) == 4;
    ProfScope ps("sell_GT", s);
    return sell_from_csr(n, nnz, rp.as<int32_t>(), ci.as<int32_t>(), val.p, f32, f32, &P->sgt, di, s, seg);
}

static int alloc_workspace(afsai_precond_s *P, const DeviceInfo &di) {
    // PCG: r, r', z, p, p', q, t (n each) + partial sums + scalars (the solver's layout)
    const size_t np = (size_t)2 * di.num_cus * 16 + 64;
    P->work_elems = (size_t)7 * P->n + np + 16;
    P->work = (double *)pool_alloc(P->work_elems * sizeof(double));
    if (!P->work) AFSAI_FAIL(AFSAI_ERR_NO_MEMORY, "out of device memory for the solver workspace");
    return AFSAI_OK;
}

}  // namespace afsai

using namespace afsai;

extern "C" {

// The adaptive setup of A; a batch (nsys > 1, row0: host, nsys + 1 entries) must be block
// diagonal, and its G and G^T layouts then follow the systems.
static int setup_core(const afsai_csr *A, const afsai_params *p, int nsys, const int32_t *row0, void *stream,
                      afsai_precond *out) {
    if (out) *out = nullptr;
    if (!A || !p || !out) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_setup: null argument");
    if (A->n <= 0 || A->nnz < A->n) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_setup: n = %d, nnz = %d", A->n, A->nnz);
    if (!A->row_ptr || !A->col_idx || !A->val) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_setup: null CSR array");
    if (p->kmax < 0 || (p->kmax > 0 && p->s < 1) || !(p->eps >= 0.0) || !(p->tie_rtol >= 0.0 && p->tie_rtol < 1.0) ||
        (p->g_prec != AFSAI_F64 && p->g_prec != AFSAI_F32) ||
        (p->flags & ~(AFSAI_VALIDATE | AFSAI_SETUP_F32 | AFSAI_GRAD_F32)) ||
        ((p->flags & AFSAI_SETUP_F32) && (p->flags & AFSAI_GRAD_F32)))
        AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_setup: bad parameters (kmax=%d s=%d eps=%g tie_rtol=%g g_prec=%d)",
                   p->kmax, p->s, p->eps, p->tie_rtol, p->g_prec);
    const int64_t mmax64 = 1 + (int64_t)p->kmax * (p->kmax > 0 ? p->s : 0);
    if (mmax64 > 64) AFSAI_FAIL(AFSAI_ERR_TOO_LARGE, "afsai_setup: 1 + kmax*s = %lld exceeds 64", (long long)mmax64);
    const int mmax = (int)mmax64;
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    // the two timing events are destroyed on every return path
    struct Events {
        hipEvent_t e[2] = {nullptr, nullptr};
        ~Events() {
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } ev;
    AFSAI_HIP_TRY(hipEventCreate(&ev.e[0]));
    AFSAI_HIP_TRY(hipEventCreate(&ev.e[1]));
    hipEvent_t t0 = ev.e[0], t1 = ev.e[1];
    AFSAI_HIP_TRY(hipEventRecord(t0, s));
    const int n = A->n;
    const bool f32 = (p->g_prec == AFSAI_F32);

    // ---- row statistics / validation
    DevBuf scanb, diagb, dlob;
    if ((rc = dalloc(scanb, sizeof(ScanOut), s))) return rc;
    if ((rc = dalloc(diagb, sizeof(double) * (size_t)n, s))) return rc;
    if ((rc = dalloc(dlob, sizeof(int32_t) * (size_t)n, s))) return rc;
    AFSAI_HIP_TRY(hipMemsetAsync(scanb.p, 0, sizeof(ScanOut), s));
    const int validate = (p->flags & AFSAI_VALIDATE) ? 1 : 0;
    ScanOut so{};
    if (validate) {
        // row pointers must be sane before rows are scanned
        hipLaunchKernelGGL(k_row_ptr_check, dim3((n + 256) / 256), dim3(256), 0, s, n, A->row_ptr, A->nnz,
                           scanb.as<ScanOut>());
        AFSAI_HIP_TRY(hipMemcpyAsync(&so, scanb.p, sizeof so, hipMemcpyDeviceToHost, s));
        AFSAI_HIP_TRY(hipStreamSynchronize(s));
        if (so.bad) AFSAI_FAIL(AFSAI_ERR_BAD_MATRIX, "afsai_setup: row pointers are not monotone from 0 to nnz");
    }
    {
        ProfScope ps("row_scan", s);
        hipLaunchKernelGGL(k_row_scan, dim3(grid1d(n, di)), dim3(256), 0, s, n, A->row_ptr, A->col_idx, A->val,
                           validate, diagb.as<double>(), dlob.as<int32_t>(), scanb.as<ScanOut>());
    }
    AFSAI_HIP_TRY(hipMemcpyAsync(&so, scanb.p, sizeof so, hipMemcpyDeviceToHost, s));
    AFSAI_HIP_TRY(hipStreamSynchronize(s));
    AFSAI_HIP_TRY(hipGetLastError());
    if (so.bad) AFSAI_FAIL(AFSAI_ERR_BAD_MATRIX, "afsai_setup: CSR structure invalid (columns unsorted, duplicate or out of range)");
    if (so.asym) AFSAI_FAIL(AFSAI_ERR_BAD_MATRIX, "afsai_setup: matrix is not exactly symmetric");
    if (so.nodiag) AFSAI_FAIL(AFSAI_ERR_BAD_MATRIX, "afsai_setup: %d rows without a diagonal entry (or unsorted columns)", so.nodiag);
    Segments seg;
    if (nsys > 1) {
        seg.nsys = nsys;
        seg.row0 = row0;
        DevBuf r0b;
        if ((rc = dalloc(r0b, sizeof(int32_t) * (size_t)(nsys + 1), s))) return rc;
        AFSAI_HIP_TRY(hipMemcpyAsync(r0b.p, row0, sizeof(int32_t) * (size_t)(nsys + 1), hipMemcpyHostToDevice, s));
        // a result of its own: the row scan's (longest row) stays in `so`
        ScanOut sb{};
        AFSAI_HIP_TRY(hipMemsetAsync(scanb.p, 0, sizeof(ScanOut), s));
        hipLaunchKernelGGL(k_block_check, dim3(grid1d(n, di)), dim3(256), 0, s, n, A->row_ptr, A->col_idx, nsys,
                           r0b.as<int32_t>(), scanb.as<ScanOut>());
        AFSAI_HIP_TRY(hipMemcpyAsync(&sb, scanb.p, sizeof sb, hipMemcpyDeviceToHost, s));
        AFSAI_HIP_TRY(hipStreamSynchronize(s));
        if (sb.bad) AFSAI_FAIL(AFSAI_ERR_BAD_MATRIX, "afsai_setup_batched: a row has entries outside its system");
    }
    const int maxlen = so.maxlen > 0 ? so.maxlen : 1;

    // ---- kernel shape: pattern capacity and candidate table size
    int mmax_t = 8;
    for (int c : {8, 16, 24, 32, 48, 64})
        if (c >= mmax) {
            mmax_t = c;
            break;
        }
    const int gmax = option(AFSAI_OPT_SETUP_GROUP) > 0 ? (int)option(AFSAI_OPT_SETUP_GROUP) : kGMax;
    // distinct columns one step can touch: at most every entry of the m pattern rows
    const int64_t bound = (int64_t)mmax * maxlen + mmax;
    // First table: a quarter of the bound (about twice the distinct columns a row's steps touch
    // on stencil-like matrices), 128..1024 slots; rows that overflow it are redone with a table
    // larger than the bound (up to 8192 slots).  Slot lists in registers where every row has at
    // most 128 entries (more rows resident per CU), else in LDS.
    const int64_t slopt = option(AFSAI_OPT_SETUP_SLOTS);
    const bool rsl = slopt == 1 ? false : (maxlen <= 128 && n <= (1 << 24));
    // with rows of at most 128 entries (stencil-like) the first table stops at 512 slots: the
    // 150^3 27-point workload (46 positions) then retries 129 of 10.1M rows and its setup takes
    // 1.81 s instead of 2.32 s with 1,024 slots (fewer rows resident per CU)
    int cap1 = pow2ceil(bound / 4 + 1);
    if (cap1 < 128) cap1 = 128;
    if (cap1 > (maxlen <= 128 ? 512 : 1024)) cap1 = maxlen <= 128 ? 512 : 1024;
    if (option(AFSAI_OPT_SETUP_TABLE) > 0) cap1 = std::max(128, std::min(8192, pow2ceil(option(AFSAI_OPT_SETUP_TABLE))));
    if (slopt == 2 && !rsl)
        AFSAI_FAIL(AFSAI_ERR_INVALID_ARG,
                   "afsai_setup: register slot lists need rows of at most 128 entries and n <= 2^24");
    // FP32 setup arithmetic: register-list form only
    const bool sf32 = (p->flags & AFSAI_SETUP_F32) != 0;
    if (sf32 && !rsl)
        AFSAI_FAIL(AFSAI_ERR_INVALID_ARG,
                   "afsai_setup: FP32 setup arithmetic needs rows of at most 128 entries and n <= 2^24 "
                   "(and register slot lists)");
    const int tb = sf32 ? 4 : 8;
    int cap2 = pow2ceil(bound + 1);
    if (cap2 < cap1) cap2 = cap1;
    if (cap2 > 8192) cap2 = 8192;

    // ---- per-row results (padded) and diagnostics
    const int ldell = mmax;
    DevBuf ell_col, ell_val, mcnt, psi, steps, reason, st, ctr, ovf;
    if ((rc = dalloc(ell_col, sizeof(int32_t) * (size_t)n * ldell, s))) return rc;
    if ((rc = dalloc(ell_val, sizeof(double) * (size_t)n * ldell, s))) return rc;
    if ((rc = dalloc(mcnt, sizeof(int32_t) * (size_t)n, s))) return rc;
    if ((rc = dalloc(psi, sizeof(double) * (size_t)n, s))) return rc;
    if ((rc = dalloc(steps, sizeof(int32_t) * (size_t)n, s))) return rc;
    if ((rc = dalloc(reason, sizeof(int32_t) * (size_t)n, s))) return rc;
    if ((rc = dalloc(st, sizeof(int8_t) * (size_t)n, s))) return rc;
    if ((rc = dalloc(ctr, sizeof(int32_t) * 16, s))) return rc;
    if ((rc = dalloc(ovf, sizeof(int32_t) * ((size_t)n + 1), s))) return rc;
    int32_t *ovf_count = ovf.as<int32_t>() + n;
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, (int64_t)1, ovf_count, 0);

    // inverse-factor form where it applies (FP64 arithmetic, register slot lists), its first
    // table from 64 slots; rows that overflow it are redone by the Cholesky form below
    const int64_t form = option(AFSAI_OPT_SETUP_FORM);
    RowsKernel k1 = nullptr;
    size_t wdyn = 0;
    int wrpw = 1;
    if (form != 1 && !sf32 && rsl) {
        int wcap = pow2ceil(bound / 4 + 1);
        if (wcap < 64) wcap = 64;
        if (wcap > 512) wcap = 512;
        if (option(AFSAI_OPT_SETUP_TABLE) > 0) wcap = (int)std::max<int64_t>(64, std::min<int64_t>(1024, pow2ceil(option(AFSAI_OPT_SETUP_TABLE))));
        const int lanes = (int)option(AFSAI_OPT_SETUP_LANES);
        // groups of 32 and 64 lanes take tables from 128 slots
        if (wcap < 128 && (lanes >= 32 || mmax > 16 || maxlen > 64)) wcap = 128;
        int gs = 64;
        k1 = rows_kernel_w(mmax, maxlen, wcap, lanes, (p->flags & AFSAI_GRAD_F32) != 0, &gs, &wdyn);
        if (k1) {
            wrpw = 64 / gs;
            cap1 = wcap;
            if (cap2 < cap1) cap2 = cap1;
        }
    }
    const bool gf32 = (p->flags & AFSAI_GRAD_F32) != 0;
    if ((form == 2 || gf32) && !k1)
        AFSAI_FAIL(AFSAI_ERR_INVALID_ARG,
                   "afsai_setup: the inverse-factor form needs FP64 setup arithmetic, rows of at most 128 entries "
                   "and n <= 2^24");
    if (!k1) k1 = rows_kernel(mmax_t, cap1, rsl, sf32);
    if (!k1) AFSAI_FAIL(AFSAI_ERR_TOO_LARGE, "afsai_setup: no kernel for pattern %d / table %d", mmax_t, cap1);
    // table entries one row touches over its steps (bound per step times k_max, plus its own row)
    const int64_t row_work = (int64_t)p->kmax * bound + maxlen;
    // the precision form's gradient values: A's values rounded to FP32, for this call
    DevBuf av32b;
    if (gf32) {
        if ((rc = dalloc(av32b, sizeof(float) * (size_t)A->nnz, s))) return rc;
        hipLaunchKernelGGL((k_narrow<float>), dim3(grid1d(A->nnz, di)), dim3(256), 0, s, (int64_t)A->nnz, A->val,
                           av32b.as<float>());
    }
    const float *av32 = gf32 ? av32b.as<float>() : nullptr;
    if ((rc = launch_rows("afsai_rows", k1, wdyn, wrpw, mmax_t, mmax, row_work, cap1, rsl, tb, gmax, A, av32, diagb.as<double>(), dlob.as<int32_t>(), p, nullptr, n, ctr.as<int32_t>(), ldell,
                          ell_col.as<int32_t>(), ell_val.as<double>(), mcnt.as<int32_t>(), psi.as<double>(),
                          steps.as<int32_t>(), reason.as<int32_t>(), st.as<int8_t>(), ovf_count, ovf.as<int32_t>(), di,
                          s)))
        return rc;
    int32_t novf = 0;
    AFSAI_HIP_TRY(hipMemcpyAsync(&novf, ovf_count, sizeof novf, hipMemcpyDeviceToHost, s));
    AFSAI_HIP_TRY(hipStreamSynchronize(s));
    int32_t retried = 0;
    if (novf > 0 && cap2 > cap1) {
        retried = novf;
        DevBuf list2;
        if ((rc = dalloc(list2, sizeof(int32_t) * ((size_t)novf + 1), s))) return rc;
        hipLaunchKernelGGL(k_copy_i32, dim3(grid1d(novf, di)), dim3(256), 0, s, (int64_t)novf, ovf.as<int32_t>(),
                           list2.as<int32_t>());
        int32_t *cnt2 = list2.as<int32_t>() + novf;
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, (int64_t)1, cnt2, 0);
        // the same form as the first launch, with the larger table
        size_t wdyn2 = 0;
        RowsKernel k2 = wdyn ? rows_kernel_w_large(mmax, cap2, (p->flags & AFSAI_GRAD_F32) != 0, &wdyn2) : rows_kernel(mmax_t, cap2, rsl, sf32);
        if (!k2) AFSAI_FAIL(AFSAI_ERR_TOO_LARGE, "afsai_setup: no kernel for table %d", cap2);
        if ((rc = launch_rows("afsai_rows_retry", k2, wdyn2, 1, mmax_t, mmax, row_work, cap2, rsl, tb, gmax, A, av32, diagb.as<double>(), dlob.as<int32_t>(), p, list2.as<int32_t>(), novf,
                              ctr.as<int32_t>(), ldell, ell_col.as<int32_t>(), ell_val.as<double>(), mcnt.as<int32_t>(),
                              psi.as<double>(), steps.as<int32_t>(), reason.as<int32_t>(), st.as<int8_t>(), cnt2,
                              ovf.as<int32_t>(), di, s)))
            return rc;
        AFSAI_HIP_TRY(hipStreamSynchronize(s));
    }

    // ---- status summary
    const int nsb = grid1d(n, di);
    DevBuf sumb;
    if ((rc = dalloc(sumb, sizeof(Summary) * (size_t)(nsb + 1), s))) return rc;
    Summary *sum_out = sumb.as<Summary>() + nsb;
    {
        ProfScope ps("summary", s);
        hipLaunchKernelGGL(k_summary, dim3(nsb), dim3(256), 0, s, n, mcnt.as<int32_t>(), st.as<int8_t>(),
                           reason.as<int32_t>(), psi.as<double>(), sumb.as<Summary>());
        hipLaunchKernelGGL(k_summary_final, dim3(1), dim3(256), 0, s, nsb, sumb.as<Summary>(), sum_out);
    }
    Summary sm{};
    AFSAI_HIP_TRY(hipMemcpyAsync(&sm, sum_out, sizeof sm, hipMemcpyDeviceToHost, s));
    AFSAI_HIP_TRY(hipStreamSynchronize(s));
    AFSAI_HIP_TRY(hipGetLastError());
    if (sm.nbad) AFSAI_FAIL(AFSAI_ERR_BAD_MATRIX, "afsai_setup: %lld rows without a diagonal entry", (long long)sm.nbad);
    if (sm.nnotspd)
        AFSAI_FAIL(AFSAI_ERR_NOT_SPD, "afsai_setup: %lld rows met a non-positive pivot (A not SPD)", (long long)sm.nnotspd);
    if (sm.novf)
        AFSAI_FAIL(AFSAI_ERR_TOO_LARGE, "afsai_setup: %lld rows touch more candidate columns than fit on chip",
                   (long long)sm.novf);
    if (sm.nnz >= ((int64_t)1 << 31))
        AFSAI_FAIL(AFSAI_ERR_TOO_LARGE, "afsai_setup: nnz(G) = %lld exceeds int32", (long long)sm.nnz);

    // ---- G as CSR (export) and SELL-64 (products); G^T as SELL-64
    afsai_precond_s *P = new afsai_precond_s();
    P->device = di.device;
    P->n = n;
    P->mmax = mmax;
    P->g_prec = p->g_prec;
    auto fail = [&](int code) {
        (void)hipStreamSynchronize(s);
        free_handle(P);
        return code;
    };
    P->g_rp = (int32_t *)pool_alloc(sizeof(int32_t) * (size_t)(n + 1));
    if (!P->g_rp) {
        set_error("afsai_setup: out of device memory");
        return fail(AFSAI_ERR_NO_MEMORY);
    }
    int64_t nnz = 0;
    if ((rc = scan_counts(n, mcnt.as<int32_t>(), P->g_rp, &nnz, di, s))) return fail(rc);
    P->nnz_g = nnz;
    const size_t vsz = f32 ? sizeof(float) : sizeof(double);
    P->g_ci = (int32_t *)pool_alloc(sizeof(int32_t) * (size_t)nnz);
    P->g_val = pool_alloc(vsz * (size_t)nnz);
    if (!P->g_ci || !P->g_val) {
        set_error("afsai_setup: out of device memory for G");
        return fail(AFSAI_ERR_NO_MEMORY);
    }
    {
        ProfScope ps("assemble_G", s);
        if (f32)
            hipLaunchKernelGGL((k_fill_g<float>), dim3(grid1d((int64_t)n * ldell, di)), dim3(256), 0, s, n, ldell,
                               mcnt.as<int32_t>(), ell_col.as<int32_t>(), ell_val.as<double>(), P->g_rp, P->g_ci,
                               (float *)P->g_val);
        else
            hipLaunchKernelGGL((k_fill_g<double>), dim3(grid1d((int64_t)n * ldell, di)), dim3(256), 0, s, n, ldell,
                               mcnt.as<int32_t>(), ell_col.as<int32_t>(), ell_val.as<double>(), P->g_rp, P->g_ci,
                               (double *)P->g_val);
    }
    if (hipError_t e = hipGetLastError(); e != hipSuccess) {
        set_error("afsai_setup: assembly of G: %s", hipGetErrorString(e));
        return fail(AFSAI_ERR_HIP);
    }
    {
        ProfScope ps("sell_G", s);
        if ((rc = sell_from_ell(n, P->nnz_g, ldell, mcnt.as<int32_t>(), ell_col.as<int32_t>(), ell_val.as<double>(), f32, &P->sg,
                                di, s, seg)))
            return fail(rc);
    }
    if (nsys > 1) P->seg_row0.assign(row0, row0 + nsys + 1);
    rc = f32 ? build_transpose<float>(P, di, s, seg, ldell, mcnt.as<int32_t>(), ell_col.as<int32_t>(),
                                      ell_val.as<double>())
             : build_transpose<double>(P, di, s, seg, ldell, mcnt.as<int32_t>(), ell_col.as<int32_t>(),
                                       ell_val.as<double>());
    if (rc) return fail(rc);
    P->psi = (double *)psi.release();
    P->steps = (int32_t *)steps.release();
    P->reason = (int32_t *)reason.release();
    if ((rc = alloc_workspace(P, di))) return fail(rc);
    {
        hipError_t e = hipEventRecord(t1, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            set_error("afsai_setup: %s", hipGetErrorString(e));
            return fail(AFSAI_ERR_HIP);
        }
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, t0, t1);
    prof_flush();

    afsai_setup_info &inf = P->info;
    inf.n = n;
    inf.mmax = mmax;
    inf.nnz_g = nnz;
    inf.g_prec = p->g_prec;
    inf.rows_stop_kmax = (int32_t)sm.stop[0];
    inf.rows_stop_eps = (int32_t)sm.stop[1];
    inf.rows_stop_nocand = (int32_t)sm.stop[2];
    inf.rows_retried = retried;
    inf.sum_log_psi = sm.sumlog;
    inf.ms = ms;
    *out = P;
    return AFSAI_OK;
}

int afsai_setup(const afsai_csr *A, const afsai_params *p, void *stream, afsai_precond *out) {
    clear_error();
    return setup_core(A, p, 1, nullptr, stream, out);
}

int afsai_setup_batched(const afsai_csr *A, int32_t nsys, const int32_t *offsets, const afsai_params *p, void *stream,
                        afsai_precond *out) {
    clear_error();
    if (out) *out = nullptr;
    if (!A || !offsets || nsys < 1) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_setup_batched: null argument or nsys < 1");
    if (offsets[0] != 0 || offsets[nsys] != A->n)
        AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_setup_batched: offsets must run from 0 to n = %d", A->n);
    for (int k = 0; k < nsys; ++k)
        if (offsets[k + 1] <= offsets[k])
            AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_setup_batched: system %d is empty or offsets decrease", k);
    return setup_core(A, p, nsys, offsets, stream, out);
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
    const bool f32 = (g_prec == AFSAI_F32);
    auto fail = [&](int code) {
        (void)hipStreamSynchronize(s);
        free_handle(P);
        return code;
    };
    const size_t vsz = f32 ? sizeof(float) : sizeof(double);
    P->g_rp = (int32_t *)pool_alloc(sizeof(int32_t) * (size_t)(G->n + 1));
    P->g_ci = (int32_t *)pool_alloc(sizeof(int32_t) * (size_t)(G->nnz ? G->nnz : 1));
    P->g_val = pool_alloc(vsz * (size_t)(G->nnz ? G->nnz : 1));
    if (!P->g_rp || !P->g_ci || !P->g_val) {
        set_error("afsai_import: out of device memory");
        return fail(AFSAI_ERR_NO_MEMORY);
    }
    if (hipMemcpyAsync(P->g_rp, G->row_ptr, sizeof(int32_t) * (size_t)(G->n + 1), hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(P->g_ci, G->col_idx, sizeof(int32_t) * (size_t)G->nnz, hipMemcpyDeviceToDevice, s) != hipSuccess) {
        set_error("afsai_import: copy failed");
        return fail(AFSAI_ERR_HIP);
    }
    if (f32)
        hipLaunchKernelGGL((k_narrow<float>), dim3(grid1d(G->nnz, di)), dim3(256), 0, s, (int64_t)G->nnz, G->val,
                           (float *)P->g_val);
    else if (hipMemcpyAsync(P->g_val, G->val, sizeof(double) * (size_t)G->nnz, hipMemcpyDeviceToDevice, s) != hipSuccess) {
        set_error("afsai_import: copy failed");
        return fail(AFSAI_ERR_HIP);
    }
    if ((rc = sell_from_csr(P->n, P->nnz_g, P->g_rp, P->g_ci, P->g_val, f32, f32, &P->sg, di, s))) return fail(rc);
    rc = f32 ? build_transpose<float>(P, di, s, Segments()) : build_transpose<double>(P, di, s, Segments());
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
