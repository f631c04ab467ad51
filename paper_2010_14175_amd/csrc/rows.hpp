// The fused per-row kernel of the adaptive FSAI setup (Sec. 2; the paper's Kaporin-gradient,
// systems-gather and batched-Cholesky kernels of Sec. 3 merged into one).
//
// One 64-lane wavefront owns one row i for all of its growth steps, so the pattern P_i, the
// scaled row g_i, the candidate table and the dense block A[P_i,P_i] stay on chip.  Per step:
//
//  1. product pass over the rows r in P_i: every stored entry a_rc with c <= i is looked up in
//     an LDS open-addressing table.  Members of P_i were entered first, tagged with their
//     position; their entries fill A[P,P] (lower part, taken from the row of the larger index).
//     Any other column is a candidate and accumulates v_c += a_rc g_r = (A g)_c by symmetry,
//     the Kaporin gradient of eq. grapsi up to a positive factor.
//  2. selection: the largest |v_c| over the candidates, then s rounds of "largest |v|, ties
//     within the relative band tie_rtol go to the smallest column" (64-lane reductions).
//  3. gather: A[P,P] is re-indexed to the enlarged pattern; only the s new rows are read.
//  4. Cholesky A[P,P] = L L^T, g = L^-T e_m (eq. DensSys with the scaling of eq. diagScal),
//     psi = L_mm^2, in FP64.
//  5. exit test psi / psi_0 <= eps (eq. exit_crit).
//
// Two forms of steps 3-4, chosen at compile time:
//  REG  (patterns of at most 32 entries, s <= 4): lane p holds row p of the block in registers;
//       the factorisation and the back substitution exchange values with v_readlane, with no
//       LDS traffic and no barriers;
//  LDS  (any pattern up to 64 entries): the block lives in LDS, one column step at a time.
// Both apply the same operations in the same order as a column-by-column textbook Cholesky
// with separately rounded products and sums, so G is identical in either form.  The gradient
// accumulation uses LDS atomics (order not fixed); it only ranks candidates, and the tie band
// absorbs rounding noise.
#pragma once

#include "common.hpp"

#pragma clang fp contract(off)

namespace afsai {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint32_t kPBit = 0x80000000u;
constexpr int kRegSMax = 4;  // new rows per step held by the REG form

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
__device__ __forceinline__ int table_find(uint32_t *hkey, uint32_t c, uint32_t ins, bool insert, bool &tagged) {
    uint32_t slot = hash0<CAP>(c);
    for (int probe = 0; probe < CAP; ++probe) {
        uint32_t k = __hip_atomic_load(&hkey[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (k == kEmpty) {
            if (!insert) return -1;
            const uint32_t old = atomicCAS(&hkey[slot], kEmpty, ins);
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

// Offsets of the concatenation of rows list[0..cnt) (cnt <= 64); off[cnt] = total.
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
    if (lane == 0) off[cnt] = total;
    __syncthreads();
    return total;
}

// value of v in lane `src` (src uniform)
__device__ __forceinline__ double rl(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

constexpr int kUnroll = 8;

template <int MMAX, int CAP, bool REG>
__global__ __launch_bounds__(64) void k_afsai_rows(
    int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, const double *__restrict__ av,
    const double *__restrict__ diag, int kmax, int s, double eps, double tau, const int32_t *__restrict__ list,
    int nlist, int32_t *__restrict__ counters, int nxcd, int32_t *__restrict__ ell_col, double *__restrict__ ell_val,
    int ldell, int32_t *__restrict__ m_out, double *__restrict__ psi_out, int32_t *__restrict__ steps_out,
    int32_t *__restrict__ reason_out, int8_t *__restrict__ status_out, int32_t *__restrict__ ovf_count,
    int32_t *__restrict__ ovf_list) {
    static_assert(!REG || MMAX <= 32, "register form holds at most 32 rows");
    constexpr int TRI = MMAX * (MMAX + 1) / 2;
    constexpr int SPL = CAP / 64;        // table slots per lane
    constexpr bool SEL_REG = SPL <= 16;  // selection from registers
    __shared__ uint32_t hkey[CAP];
    __shared__ double hval[CAP];
    __shared__ double X[TRI];                          // A[P,P] of the current pattern (packed lower)
    __shared__ double Y[REG ? 1 : TRI];                // LDS form: block of the enlarged pattern
    __shared__ double NR[REG ? kRegSMax * MMAX : 1];   // REG form: new rows, by new position
    __shared__ int32_t Pl[MMAX];     // pattern, ascending
    __shared__ int32_t Pn[MMAX];     // enlarged pattern
    __shared__ int32_t pslot[MMAX];  // table slot of each member of Pl
    __shared__ int32_t nslot[MMAX];  // table slot of each member of Pn
    __shared__ int32_t npos[MMAX];   // new position of old member t
    __shared__ int32_t opos[MMAX];   // old position of new member p, or -1-u for the u-th new column
    __shared__ double gl[MMAX];      // scaled row on Pl
    __shared__ int32_t off[65], beg[64];
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
        const double aii = diag[i];
        int8_t status = ROW_OK;
        int m = 1, steps = 0;
        int32_t reason = STOP_KMAX;
        double psi = aii;
        if (!(aii > 0.0) || !isfinite(aii)) status = ROW_NOT_SPD;
        if (lane == 0) {
            Pl[0] = i;
            gl[0] = 1.0 / sqrt(aii);
        }
        __syncthreads();
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
            int tseg = 0;
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
                        if (u == 0) tseg = seg_of(off, m, e);
                        else
                            while (off[tseg + 1] <= e) ++tseg;
                        const int idx = beg[tseg] + (e - off[tseg]);
                        tt[u] = tseg;
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
            int ns = 0;
            if constexpr (SEL_REG) {
                uint32_t kr[SPL];
                double ar[SPL];
                double lmax = -1.0;
#pragma unroll
                for (int j = 0; j < SPL; ++j) {
                    const uint32_t kk = hkey[lane + 64 * j];
                    const bool cand = (kk != kEmpty) && !(kk & kPBit);
                    kr[j] = cand ? kk : kEmpty;
                    ar[j] = cand ? fabs(hval[lane + 64 * j]) : -1.0;
                    lmax = fmax(lmax, ar[j]);
                }
                const double M = wave_max(lmax);
                if (M > 0.0) {
                    const double thr = 0x1.0p-40 * M;
                    for (int round = 0; round < s; ++round) {
                        double l = 0.0;
#pragma unroll
                        for (int j = 0; j < SPL; ++j)
                            if (ar[j] > thr) l = fmax(l, ar[j]);
                        const double Mp = wave_max(l);
                        if (!(Mp > 0.0)) break;
                        const double band = (1.0 - tau) * Mp;
                        uint32_t lb = kEmpty;
#pragma unroll
                        for (int j = 0; j < SPL; ++j)
                            if (ar[j] > thr && ar[j] >= band && kr[j] < lb) lb = kr[j];
                        const uint32_t js = wave_min(lb);
#pragma unroll
                        for (int j = 0; j < SPL; ++j)
                            if (kr[j] == js) {
                                hkey[lane + 64 * j] = js | kPBit;
                                selslot[ns] = lane + 64 * j;
                                kr[j] = kEmpty;
                                ar[j] = -1.0;
                            }
                        if (lane == 0) sel[ns] = (int32_t)js;
                        ++ns;
                    }
                }
                __syncthreads();
            } else {
                double lmax = 0.0;
                for (int j = lane; j < CAP; j += 64) {
                    const uint32_t kk = hkey[j];
                    if (kk != kEmpty && !(kk & kPBit)) lmax = fmax(lmax, fabs(hval[j]));
                }
                const double M = wave_max(lmax);
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
            }
            if (ns == 0) {
                reason = STOP_NOCAND;
                break;
            }

            // ---- 3. enlarged pattern and positions
            const int mn = m + ns;
            if (lane < m) {
                const int c = Pl[lane];
                int add = 0;
                for (int u = 0; u < ns; ++u) add += (sel[u] < c);
                const int p = lane + add;
                npos[lane] = p;
                opos[p] = lane;
                Pn[p] = c;
                nslot[p] = pslot[lane];
                hval[pslot[lane]] = (double)p;
            } else if (lane < m + ns) {
                const int u = lane - m;
                const int c = sel[u];
                int lo = 0, hi = m;  // old members below c
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (Pl[mid] < c) lo = mid + 1; else hi = mid;
                }
                int add = 0;
                for (int v = 0; v < ns; ++v) add += (sel[v] < c);
                const int p = lo + add;
                selpos[u] = p;
                opos[p] = -1 - u;
                Pn[p] = c;
                nslot[p] = selslot[u];
                hval[selslot[u]] = (double)p;
            }
            if constexpr (REG) {
                for (int j = lane; j < ns * MMAX; j += 64) NR[j] = 0.0;
            } else {
                const int ntn = (mn * (mn + 1)) >> 1;
                for (int j = lane; j < ntn; j += 64) Y[j] = 0.0;
            }
            __syncthreads();
            if constexpr (!REG) {
                const float invm = 1.0f / (float)m;
                for (int e = lane; e < m * m; e += 64) {
                    const int a = (int)(((float)e + 0.5f) * invm);
                    const int b = e - a * m;
                    if (b <= a) Y[tri(npos[a], npos[b])] = X[tri(a, b)];
                }
            }
            // new rows: entries (sel[u], c) with c in the enlarged pattern
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
                        if constexpr (REG) {
                            NR[u * MMAX + pc] = av[idx];
                        } else {
                            const int pn = selpos[u];
                            Y[pc <= pn ? tri(pn, pc) : tri(pc, pn)] = av[idx];
                        }
                    }
                }
            }
            __syncthreads();

            // ---- 4. Cholesky A[P,P] = L L^T and g = L^-T e_m
            bool spd = true;
            double gx = 0.0, lmm = 0.0;
            if constexpr (REG) {
                // lane p holds row p of the block (columns 0..p)
                double row[MMAX];
                const int op = (lane < mn) ? opos[lane] : 0;
#pragma unroll
                for (int qq = 0; qq < MMAX; ++qq) {
                    double v = 0.0;
                    if (qq < mn && qq <= lane && lane < mn) {
                        const int oq = opos[qq];
                        if (op >= 0 && oq >= 0) v = X[tri(op, oq)];
                        else if (op < 0) v = NR[(-1 - op) * MMAX + qq];
                        else v = NR[(-1 - oq) * MMAX + lane];
                    }
                    row[qq] = v;
                }
#pragma unroll
                for (int kk = 0; kk < MMAX; ++kk) {
                    if (kk < mn && spd) {
                        const double d2 = rl(row[kk], kk);
                        if (!(d2 > 0.0) || !isfinite(d2)) {
                            spd = false;
                        } else {
                            const double d = sqrt(d2);
                            lmm = d;
                            if (lane == kk) row[kk] = d;
                            else if (lane > kk) row[kk] = row[kk] / d;
#pragma unroll
                            for (int c = kk + 1; c < MMAX; ++c) {
                                if (c < mn) {
                                    const double lck = rl(row[kk], c);
                                    if (lane >= c) row[c] = row[c] - row[kk] * lck;
                                }
                            }
                        }
                    }
                }
                if (spd) {
                    // back substitution L^T x = e_m: lane t accumulates sum_{l>t} L_lt x_l, l descending
                    double acc = 0.0;
#pragma unroll
                    for (int l = MMAX - 1; l >= 0; --l) {
                        if (l < mn) {
                            const double Lll = rl(row[l], l);
                            const double xl = (l == mn - 1) ? 1.0 / Lll : -(rl(acc, l) / Lll);
                            if (lane == l) gx = xl;
#pragma unroll
                            for (int t = 0; t < l; ++t) {
                                const double v = rl(row[t], l);
                                if (lane == t) acc = acc + v * xl;
                            }
                        }
                    }
                }
            } else {
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
                if (spd) {
                    double acc = 0.0;
                    for (int l = mn - 1; l >= 0; --l) {
                        const double Lll = Y[tri(l, l)];
                        const double accl = __shfl(acc, l, 64);
                        const double xl = (l == mn - 1) ? 1.0 / Lll : -(accl / Lll);
                        if (lane == l) gx = xl;
                        if (lane < l) acc = acc + Y[tri(l, lane)] * xl;
                    }
                    lmm = Y[tri(mn - 1, mn - 1)];
                }
            }
            if (!spd) {
                status = ROW_NOT_SPD;
                break;
            }
            if (lane < mn) {
                gl[lane] = gx;
                Pl[lane] = Pn[lane];
                pslot[lane] = nslot[lane];
            }
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
        if (status == ROW_OK && lane < m) {
            ell_col[(size_t)i * ldell + lane] = Pl[lane];
            ell_val[(size_t)i * ldell + lane] = gl[lane];
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

typedef void (*RowsKernel)(int, const int32_t *, const int32_t *, const double *, const double *, int, int,
                           double, double, const int32_t *, int, int32_t *, int, int32_t *, double *, int,
                           int32_t *, double *, int32_t *, int32_t *, int8_t *, int32_t *, int32_t *);

template <int MMAX, bool REG>
static RowsKernel rows_kernel_cap(int cap) {
    switch (cap) {
        case 128: return k_afsai_rows<MMAX, 128, REG>;
        case 256: return k_afsai_rows<MMAX, 256, REG>;
        case 512: return k_afsai_rows<MMAX, 512, REG>;
        case 1024: return k_afsai_rows<MMAX, 1024, REG>;
        case 2048: return k_afsai_rows<MMAX, 2048, REG>;
        case 4096: return k_afsai_rows<MMAX, 4096, REG>;
        case 8192: return k_afsai_rows<MMAX, 8192, REG>;
        default: return nullptr;
    }
}

}  // namespace afsai
