// Adaptive FSAI setup on gfx950 (Sec. 2 method; Sec. 3 kernels: Kaporin gradient and
// selection, systems gather, batched Cholesky), plus the assembly of G and G^T.
//
// One 64-lane wavefront owns one row i for all of its growth steps, so the pattern P_i, the
// scaled row g_i, the candidate table and the dense block A[P_i,P_i] never leave LDS (the
// paper's three kernels each wrote their results to memory between steps).  Per step:
//
//  1. product pass over the rows r in P_i: every stored entry a_rc with c <= i is looked up in
//     an LDS open-addressing table.  Columns already in P_i were entered first, tagged with
//     their position, and their entries fill A[P,P] (lower part, row r being the larger
//     index).  Any other column is a candidate and accumulates v_c += a_rc g_r, which is
//     (A g)_c by symmetry, the Kaporin gradient of eq. grapsi up to a positive factor.
//  2. selection: the largest |v_c| over the candidates, then s rounds of "largest |v|, ties
//     within the relative band tie_rtol go to the smallest column" with 64-lane reductions.
//  3. gather: A[P,P] is re-indexed to the enlarged pattern and only the s new rows are read.
//  4. Cholesky A[P,P] = L L^T and g = L^-T e_m (eq. DensSys with the scaling of eq.
//     diagScal), psi = L_mm^2, all in FP64 in LDS.
//  5. exit test psi / psi_0 <= eps (eq. exit_crit).
//
// The Cholesky factorisation and the back substitution use the same operation order as a
// column-by-column textbook factorisation with products and sums rounded separately (no
// contraction), so G is reproducible bit for bit.  The gradient accumulation uses LDS atomics
// (order not fixed); it only ranks candidates, and the tie band absorbs rounding noise.
//
// Rows are taken from per-XCD work counters (dynamic scheduling inside one contiguous range
// of rows per XCD).  A row whose candidate set overflows its LDS table is reported and redone
// by a second launch with a table large enough for any pattern.
#include <cmath>
#include <vector>

#include "common.hpp"

#pragma clang fp contract(off)

namespace afsai {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint32_t kPBit = 0x80000000u;

enum : int8_t { ROW_OK = 0, ROW_OVERFLOW = 1, ROW_BAD = 2, ROW_NOT_SPD = 3 };
enum : int32_t { STOP_KMAX = 0, STOP_EPS = 1, STOP_NOCAND = 2 };

__device__ __forceinline__ int tri(int p, int q) { return ((p * (p + 1)) >> 1) + q; }  // q <= p

template <int CAP>
__device__ __forceinline__ uint32_t hash0(uint32_t c) {
    constexpr int B = __builtin_ctz(CAP);
    return (c * 2654435761u) >> (32 - B);
}

// Finds column c in the table; inserts `ins` (c, possibly tagged) when absent and `insert` is
// set.  Returns the slot, -1 if absent (lookup only) or -2 if the table is full.
template <int CAP>
__device__ __forceinline__ int table_find(uint32_t *hkey, uint32_t c, uint32_t ins, bool insert,
                                          bool &tagged) {
    uint32_t slot = hash0<CAP>(c);
    for (int probe = 0; probe < CAP; ++probe) {
        uint32_t k = __hip_atomic_load(&hkey[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (k == kEmpty) {
            if (!insert) return -1;
            uint32_t old = atomicCAS(&hkey[slot], kEmpty, ins);
            if (old == kEmpty) {
                tagged = (ins & kPBit) != 0;
                return (int)slot;
            }
            k = old;
        }
        if ((k & ~kPBit) == c) {
            tagged = (k & kPBit) != 0;
            return (int)slot;
        }
        slot = (slot + 1) & (CAP - 1);
    }
    return -2;
}

// position t of the concatenated entry e: largest t < cnt with off[t] <= e
__device__ __forceinline__ int seg_of(const int32_t *off, int cnt, int e) {
    int lo = 0, hi = cnt - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= e) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Offsets of the concatenation of rows list[0..cnt) (cnt <= 64); returns the total length.
__device__ __forceinline__ int stage_rows(const int32_t *__restrict__ rp, const int32_t *list, int cnt,
                                          int32_t *off, int32_t *beg) {
    const int lane = threadIdx.x;
    int len = 0;
    if (lane < cnt) {
        const int r = list[lane];
        const int b = rp[r];
        len = rp[r + 1] - b;
        beg[lane] = b;
    }
    const int incl = wave_incl_scan(len);
    if (lane < cnt) off[lane] = incl - len;
    const int total = __shfl(incl, cnt - 1, 64);
    __syncthreads();
    return total;
}

constexpr int kUnroll = 4;

template <int MMAX, int CAP>
__global__ __launch_bounds__(64) void k_afsai_rows(
    int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, const double *__restrict__ av,
    int kmax, int s, double eps, double tau, const int32_t *__restrict__ list, int nlist,
    int32_t *__restrict__ counters, int nxcd, int32_t *__restrict__ ell_col, double *__restrict__ ell_val,
    int ldell, int32_t *__restrict__ m_out, double *__restrict__ psi_out, int32_t *__restrict__ steps_out,
    int32_t *__restrict__ reason_out, int8_t *__restrict__ status_out, int32_t *__restrict__ ovf_count,
    int32_t *__restrict__ ovf_list) {
    constexpr int TRI = MMAX * (MMAX + 1) / 2;
    __shared__ uint32_t hkey[CAP];
    __shared__ double hval[CAP];
    __shared__ double X[TRI];
    __shared__ double Y[TRI];
    __shared__ int32_t Pl[MMAX];      // pattern, ascending
    __shared__ int32_t Pn[MMAX];      // enlarged pattern
    __shared__ int32_t pslot[MMAX];   // table slot of each member of Pl
    __shared__ int32_t nslot[MMAX];   // table slot of each member of Pn
    __shared__ int32_t npos[MMAX];    // new position of old member t
    __shared__ double gl[MMAX];       // scaled row on Pl
    __shared__ int32_t off[64], beg[64];
    __shared__ int32_t sel[64], selslot[64], selpos[64];
    __shared__ int32_t s_row, s_flag;

    const int lane = threadIdx.x;
    const int x = blockIdx.x % nxcd;
    const int64_t per = ((int64_t)nlist + nxcd - 1) / nxcd;
    const int q0 = (int)min<int64_t>(nlist, per * x), q1 = (int)min<int64_t>(nlist, per * (x + 1));

    for (;;) {
        if (lane == 0) s_row = q0 + atomicAdd(&counters[x], 1);
        __syncthreads();
        const int q = s_row;
        __syncthreads();
        if (q >= q1) break;
        const int i = list ? list[q] : q;

        // ---- G_0 = I scaled: P = {i}, g = a_ii^-1/2, psi_0 = a_ii
        const int a0 = rp[i], a1 = rp[i + 1];
        double aii = 0.0;
        bool found = false;
        for (int e = a0 + lane; e < a1; e += 64)
            if (ci[e] == i) {
                aii = av[e];
                found = true;
            }
        const unsigned long long bal = __ballot(found);
        int8_t status = ROW_OK;
        int m = 1, steps = 0;
        int32_t reason = STOP_KMAX;
        double psi = 0.0;
        if (bal == 0ull) {
            status = ROW_BAD;
        } else {
            aii = __shfl(aii, __ffsll((long long)bal) - 1, 64);
            if (!(aii > 0.0) || !isfinite(aii)) status = ROW_NOT_SPD;
        }
        if (status == ROW_OK) {
            if (lane == 0) {
                Pl[0] = i;
                gl[0] = 1.0 / sqrt(aii);
            }
            psi = aii;
            __syncthreads();
        }
        const double psi0 = aii;

        for (int k = 1; k <= kmax && status == ROW_OK; ++k) {
            // ---- 1. product pass: gradient on candidates, A[P,P] from the rows of P
            for (int j = lane; j < CAP; j += 64) {
                hkey[j] = kEmpty;
                hval[j] = 0.0;
            }
            const int ntri = (m * (m + 1)) >> 1;
            for (int j = lane; j < ntri; j += 64) X[j] = 0.0;
            if (lane == 0) s_flag = 0;
            __syncthreads();
            if (lane < m) {
                bool tg;
                const uint32_t c = (uint32_t)Pl[lane];
                const int slot = table_find<CAP>(hkey, c, c | kPBit, true, tg);
                pslot[lane] = slot;
                if (slot >= 0) hval[slot] = (double)lane;  // position tag
                else s_flag = 1;
            }
            const int total = stage_rows(rp, Pl, m, off, beg);
            for (int base = 0; base < total; base += 64 * kUnroll) {
                int cc[kUnroll], tt[kUnroll];
                double vv[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const int e = base + u * 64 + lane;
                    cc[u] = -1;
                    tt[u] = 0;
                    vv[u] = 0.0;
                    if (e < total) {
                        const int t = seg_of(off, m, e);
                        const int idx = beg[t] + (e - off[t]);
                        tt[u] = t;
                        cc[u] = __builtin_nontemporal_load(&ci[idx]);
                        vv[u] = __builtin_nontemporal_load(&av[idx]);
                    }
                }
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const int c = cc[u];
                    if (c >= 0 && c <= i) {
                        bool tg = false;
                        const int slot = table_find<CAP>(hkey, (uint32_t)c, (uint32_t)c, true, tg);
                        if (slot < 0) {
                            s_flag = 1;
                        } else if (tg) {
                            const int pc = (int)hval[slot];
                            if (pc <= tt[u]) X[tri(tt[u], pc)] = vv[u];
                        } else {
                            __hip_atomic_fetch_add(&hval[slot], vv[u] * gl[tt[u]], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                        }
                    }
                }
            }
            __syncthreads();
            if (s_flag) {
                status = ROW_OVERFLOW;
                break;
            }

            // ---- 2. selection (top-s of |v| over the candidates, tie band, smallest column)
            double lmax = 0.0;
            for (int j = lane; j < CAP; j += 64) {
                const uint32_t kk = hkey[j];
                if (kk != kEmpty && !(kk & kPBit)) lmax = fmax(lmax, fabs(hval[j]));
            }
            const double M = wave_max(lmax);
            int ns = 0;
            if (M > 0.0) {
                const double thr = 0x1.0p-40 * M;
                for (int round = 0; round < s; ++round) {
                    double l = 0.0;
                    for (int j = lane; j < CAP; j += 64) {
                        const uint32_t kk = hkey[j];
                        if (kk != kEmpty && !(kk & kPBit)) {
                            const double a = fabs(hval[j]);
                            if (a > thr) l = fmax(l, a);
                        }
                    }
                    const double Mp = wave_max(l);
                    if (!(Mp > 0.0)) break;
                    const double band = (1.0 - tau) * Mp;
                    uint32_t lb = kEmpty;
                    for (int j = lane; j < CAP; j += 64) {
                        const uint32_t kk = hkey[j];
                        if (kk != kEmpty && !(kk & kPBit)) {
                            const double a = fabs(hval[j]);
                            if (a > thr && a >= band && kk < lb) lb = kk;
                        }
                    }
                    const uint32_t js = wave_min(lb);
                    for (int j = lane; j < CAP; j += 64)
                        if (hkey[j] == js) {
                            hkey[j] = js | kPBit;
                            selslot[ns] = j;
                        }
                    if (lane == 0) sel[ns] = (int32_t)js;
                    ++ns;
                    __syncthreads();
                }
            }
            if (ns == 0) {
                reason = STOP_NOCAND;
                break;
            }

            // ---- 3. enlarged pattern, positions, gather of A[Pn,Pn]
            const int mn = m + ns;
            if (lane < m) {
                const int c = Pl[lane];
                int add = 0;
                for (int u = 0; u < ns; ++u) add += (sel[u] < c);
                const int p = lane + add;
                npos[lane] = p;
                Pn[p] = c;
                nslot[p] = pslot[lane];
                hval[pslot[lane]] = (double)p;
            } else if (lane < m + ns) {
                const int u = lane - m;
                const int c = sel[u];
                int lo = 0, hi = m;  // number of old members below c
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (Pl[mid] < c) lo = mid + 1; else hi = mid;
                }
                int add = 0;
                for (int v = 0; v < ns; ++v) add += (sel[v] < c);
                const int p = lo + add;
                selpos[u] = p;
                Pn[p] = c;
                nslot[p] = selslot[u];
                hval[selslot[u]] = (double)p;
            }
            const int ntn = (mn * (mn + 1)) >> 1;
            for (int j = lane; j < ntn; j += 64) Y[j] = 0.0;
            __syncthreads();
            {
                const float invm = 1.0f / (float)m;
                for (int e = lane; e < m * m; e += 64) {
                    const int a = (int)(((float)e + 0.5f) * invm);
                    const int b = e - a * m;
                    if (b <= a) Y[tri(npos[a], npos[b])] = X[tri(a, b)];
                }
            }
            const int tot2 = stage_rows(rp, sel, ns, off, beg);
            for (int e = lane; e < tot2; e += 64) {
                const int u = seg_of(off, ns, e);
                const int idx = beg[u] + (e - off[u]);
                const int c = ci[idx];
                if (c <= i) {
                    bool tg = false;
                    const int slot = table_find<CAP>(hkey, (uint32_t)c, 0u, false, tg);
                    if (slot >= 0 && tg) {
                        const int pc = (int)hval[slot];
                        const int pn = selpos[u];
                        Y[pc <= pn ? tri(pn, pc) : tri(pc, pn)] = av[idx];
                    }
                }
            }
            __syncthreads();
            if (lane < mn) {
                Pl[lane] = Pn[lane];
                pslot[lane] = nslot[lane];
            }

            // ---- 4. Cholesky A[P,P] = L L^T (right-looking; same rounding sequence as the
            //         column-oriented textbook form) and g = L^-T e_m
            bool spd = true;
            for (int kk = 0; kk < mn; ++kk) {
                const double d2 = Y[tri(kk, kk)];
                if (!(d2 > 0.0) || !isfinite(d2)) {
                    spd = false;
                    break;
                }
                const double d = sqrt(d2);
                const int R = mn - kk - 1;
                __syncthreads();
                if (lane < R) {
                    const int r = kk + 1 + lane;
                    Y[tri(r, kk)] = Y[tri(r, kk)] / d;
                }
                if (lane == 0) Y[tri(kk, kk)] = d;
                __syncthreads();
                if (R > 0) {
                    const float invR = 1.0f / (float)R;
                    for (int e = lane; e < R * R; e += 64) {
                        const int tr = (int)(((float)e + 0.5f) * invR);
                        const int tc = e - tr * R;
                        if (tc <= tr) {
                            const int r = kk + 1 + tr, c = kk + 1 + tc;
                            Y[tri(r, c)] = Y[tri(r, c)] - Y[tri(r, kk)] * Y[tri(c, kk)];
                        }
                    }
                }
                __syncthreads();
            }
            if (!spd) {
                status = ROW_NOT_SPD;
                break;
            }
            double acc = 0.0, gx = 0.0;
            for (int l = mn - 1; l >= 0; --l) {
                const double Lll = Y[tri(l, l)];
                const double accl = __shfl(acc, l, 64);
                const double xl = (l == mn - 1) ? 1.0 / Lll : -(accl / Lll);
                if (lane == l) gx = xl;
                if (lane < l) acc = acc + Y[tri(l, lane)] * xl;
            }
            if (lane < mn) gl[lane] = gx;
            const double lmm = Y[tri(mn - 1, mn - 1)];
            psi = lmm * lmm;
            m = mn;
            steps = k;
            __syncthreads();
            // ---- 5. exit test (eq. exit_crit)
            if (psi <= eps * psi0) {
                reason = STOP_EPS;
                break;
            }
        }

        // ---- outputs
        if (status == ROW_OK) {
            if (lane < m) {
                ell_col[(size_t)i * ldell + lane] = Pl[lane];
                ell_val[(size_t)i * ldell + lane] = gl[lane];
            }
        }
        if (lane == 0) {
            m_out[i] = (status == ROW_OK) ? m : 0;
            psi_out[i] = psi;
            steps_out[i] = steps;
            reason_out[i] = reason;
            status_out[i] = status;
            if (status == ROW_OVERFLOW) {
                const int pos = atomicAdd(ovf_count, 1);
                ovf_list[pos] = i;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------
// row statistics (max row length) and optional structural / symmetry validation
// ---------------------------------------------------------------------------------------
struct ScanOut {
    int32_t maxlen;
    int32_t bad;       // structural problem found
    int32_t asym;      // asymmetric pair found
    int32_t pad;
};

__global__ void k_row_scan(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                           const double *__restrict__ av, int validate, ScanOut *out) {
    int lmax = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int a = rp[i], b = rp[i + 1];
        lmax = max(lmax, b - a);
        if (!validate) continue;
        if (b < a) {
            atomicOr(&out->bad, 1);
            continue;
        }
        bool diag = false;
        for (int e = a; e < b; ++e) {
            const int c = ci[e];
            if (c < 0 || c >= n || (e > a && c <= ci[e - 1])) {
                atomicOr(&out->bad, 1);
                break;
            }
            if (c == i) diag = true;
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
        if (!diag) atomicOr(&out->bad, 1);
    }
    lmax = wave_max(lmax);
    if ((threadIdx.x & 63) == 0) atomicMax(&out->maxlen, lmax);
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

typedef void (*RowsKernel)(int, const int32_t *, const int32_t *, const double *, int, int, double, double,
                           const int32_t *, int, int32_t *, int, int32_t *, double *, int, int32_t *, double *,
                           int32_t *, int32_t *, int8_t *, int32_t *, int32_t *);

template <int MMAX>
static RowsKernel rows_kernel_cap(int cap) {
    switch (cap) {
        case 128: return k_afsai_rows<MMAX, 128>;
        case 256: return k_afsai_rows<MMAX, 256>;
        case 512: return k_afsai_rows<MMAX, 512>;
        case 1024: return k_afsai_rows<MMAX, 1024>;
        case 2048: return k_afsai_rows<MMAX, 2048>;
        case 4096: return k_afsai_rows<MMAX, 4096>;
        case 8192: return k_afsai_rows<MMAX, 8192>;
        default: return nullptr;
    }
}

static RowsKernel rows_kernel(int mmax_t, int cap) {
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

static int pow2ceil(int64_t v) {
    int64_t p = 1;
    while (p < v) p <<= 1;
    return (int)p;
}

static size_t rows_lds_bytes(int mmax_t, int cap) {
    return (size_t)cap * 12 + (size_t)mmax_t * (mmax_t + 1) * 8 + (size_t)mmax_t * 28 + 64 * 20 + 16;
}

static int launch_rows(RowsKernel kern, int mmax_t, int cap, const afsai_csr *A, const afsai_params *p,
                       const int32_t *list, int nlist, int32_t *counters, int ldell, int32_t *ell_col,
                       double *ell_val, int32_t *m, double *psi, int32_t *steps, int32_t *reason, int8_t *st,
                       int32_t *ovf_count, int32_t *ovf_list, const DeviceInfo &di, hipStream_t s) {
    const size_t lds = rows_lds_bytes(mmax_t, cap);
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
        hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(64), 0, s, A->n, A->row_ptr, A->col_idx, A->val, p->kmax,
                           p->s, p->eps, p->tie_rtol, list, nlist, counters, nx, ell_col, ell_val, ldell, m, psi, steps,
                           reason, st, ovf_count, ovf_list);
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
    hipLaunchKernelGGL(k_row_scan, dim3(grid1d(n, di)), dim3(256), 0, s, n, A->row_ptr, A->col_idx, A->val, validate,
                       scanb.as<ScanOut>());
    AFSAI_HIP_TRY(hipMemcpyAsync(&so, scanb.p, sizeof so, hipMemcpyDeviceToHost, s));
    AFSAI_HIP_TRY(hipStreamSynchronize(s));
    AFSAI_HIP_TRY(hipGetLastError());
    if (so.bad) AFSAI_FAIL(AFSAI_ERR_BAD_MATRIX, "afsai_setup: CSR structure invalid (columns unsorted, duplicate, out of range, or a missing diagonal)");
    if (so.asym) AFSAI_FAIL(AFSAI_ERR_BAD_MATRIX, "afsai_setup: matrix is not exactly symmetric");
    const int maxlen = so.maxlen > 0 ? so.maxlen : 1;

    // ---- kernel shape: pattern capacity and candidate table size
    int mmax_t = 8;
    for (int c : {8, 16, 24, 32, 48, 64})
        if (c >= mmax) {
            mmax_t = c;
            break;
        }
    const int64_t bound = (int64_t)mmax * maxlen + mmax;  // distinct columns a step can touch
    int cap1 = pow2ceil((bound * 3 + 1) / 2);
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

    RowsKernel k1 = rows_kernel(mmax_t, cap1);
    if (!k1) AFSAI_FAIL(AFSAI_ERR_TOO_LARGE, "afsai_setup: no kernel for pattern %d / table %d", mmax_t, cap1);
    if ((rc = launch_rows(k1, mmax_t, cap1, A, p, nullptr, n, ctr.as<int32_t>(), ldell, ell_col.as<int32_t>(),
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
        RowsKernel k2 = rows_kernel(mmax_t, cap2);
        if (!k2) AFSAI_FAIL(AFSAI_ERR_TOO_LARGE, "afsai_setup: no kernel for table %d", cap2);
        if ((rc = launch_rows(k2, mmax_t, cap2, A, p, list2.as<int32_t>(), novf, ctr.as<int32_t>(), ldell,
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
