// The fused per-row kernel of the adaptive FSAI setup (Sec. 2; the paper's Kaporin-gradient,
// systems-gather and batched-Cholesky kernels of Sec. 3 merged into one).
//
// One 64-lane wavefront owns one row i for all of its growth steps, so the pattern P_i, the
// scaled row g_i, the Cholesky factor of A[P_i,P_i] and the candidate table stay on chip.
//
// The pattern is kept in growth order: position t < m-1 holds the t-th column that joined the
// pattern, i is last.  A[P,P] = L L^T in that order means that the rows of L for the old
// positions never change when the pattern grows: a step only appends the rows of its new
// positions (a forward substitution against the stored rows) and redoes the new columns of
// the last row.  Every entry still receives exactly the operations of a from-scratch,
// column-by-column factorisation in that order (entries below a pivot multiplied by the
// pivot's reciprocal), so G is bit-identical to such a factorisation.  Per step:
//
//  1. product pass over the rows r in P_i, entries a_rc with c < i only (the part of each row
//     left of column i, a prefix): c is looked up in an LDS open-addressing table.  Members of
//     P_i were entered first, tagged; any other column is a candidate and accumulates
//     v_c += a_rc g_r = (A g)_c by symmetry, the Kaporin gradient of eq. grapsi up to a
//     positive factor.
//  2. selection: the largest |v_c| over the candidates, then s rounds of "largest |v|, ties
//     within the relative band tie_rtol go to the smallest column" (64-lane reductions).
//  3. gather of the new rows A[u, P] (their entries with column <= i).
//  4. factor update: the new rows of L and the new columns of the last row, at most kGMax
//     rows at a time; lanes own entries of the rows being appended, column j's values are
//     broadcast with v_readlane and applied right-looking.
//  5. back substitution L^T g = e_m from the last position down (eq. DensSys with the scaling
//     of eq. diagScal), psi = L_mm^2, exit test psi / psi_0 <= eps (eq. exit_crit).
// The gradient accumulation uses LDS atomics (order not fixed); it only ranks candidates, and
// the tie band absorbs rounding noise.
#pragma once

#include "common.hpp"

#pragma clang fp contract(off)

namespace afsai {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint32_t kPBit = 0x80000000u;
constexpr int kGMax = 4;  // rows appended to the factor together

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

// value of v in lane `src` (src uniform)
__device__ __forceinline__ double rl(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

// entries of one factor update that appends g rows to mb final rows: row v of the new ones
// has columns 0..mb+v, the last row (i) has the g new columns and its diagonal
__host__ __device__ __forceinline__ int upd_entries(int mb, int g) { return g * (mb + 1) + (g * (g - 1)) / 2 + g + 1; }
// index of entry (v, c) of new row v, and of the last row's entry at column mb + d
__device__ __forceinline__ int upd_index(int mb, int v, int c) { return v * (mb + 1) + (v * (v - 1)) / 2 + c; }

constexpr int kUnroll = 8;

template <int MMAX, int CAP>
__global__ __launch_bounds__(64) void k_afsai_rows(
    int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, const double *__restrict__ av,
    const double *__restrict__ diag, const int32_t *__restrict__ dlo, int kmax, int s, double eps, double tau,
    int gmax, const int32_t *__restrict__ list, int nlist, int32_t *__restrict__ counters, int nxcd,
    int32_t *__restrict__ ell_col, double *__restrict__ ell_val, int ldell, int32_t *__restrict__ m_out,
    double *__restrict__ psi_out, int32_t *__restrict__ steps_out, int32_t *__restrict__ reason_out,
    int8_t *__restrict__ status_out, int32_t *__restrict__ ovf_count, int32_t *__restrict__ ovf_list) {
    constexpr int K = (MMAX + 1 + 63) / 64;           // update entries per lane
    constexpr int LTRI = (MMAX * (MMAX - 1)) / 2;     // rows 0..MMAX-2 of L, packed lower
    constexpr int SPL = CAP / 64;                     // table slots per lane
    constexpr bool SEL_REG = SPL <= 16;               // selection from registers
    __shared__ uint32_t hkey[CAP];
    __shared__ double hval[CAP];
    __shared__ double Lp[LTRI];           // rows of L for the off-diagonal positions
    __shared__ double dinv[MMAX];         // their reciprocal pivots
    __shared__ double li[MMAX];           // row of i in L, columns 0..m-2
    __shared__ double gq[MMAX];           // scaled row by position (i at m-1)
    __shared__ int32_t Qc[MMAX];          // column of each off-diagonal position
    __shared__ int32_t mbeg[MMAX], mlen[MMAX];  // row start and number of entries left of column i
    __shared__ int32_t off[MMAX + 1];
    __shared__ double NR[kGMax * MMAX];   // gathered new rows, by position (i at MMAX-1)
    __shared__ int32_t sel[64], selslot[64];
    __shared__ int32_t nlo[kGMax], nbeg[kGMax + 1];
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
        const int ibeg = rp[i], ilen = dlo[i];
        int8_t status = ROW_OK;
        int m = 1, steps = 0;
        int32_t reason = STOP_KMAX;
        double psi = aii;
        double di = aii;  // last row's diagonal less the squares of its final entries
        if (!(aii > 0.0) || !isfinite(aii)) status = ROW_NOT_SPD;
        if (lane == 0) gq[0] = 1.0 / sqrt(aii);
        __syncthreads();
        const double psi0 = aii;

        for (int k = 1; k <= kmax && status == ROW_OK; ++k) {
            // ---- 1. product pass: gradient on the candidates
            for (int j = lane; j < CAP; j += 64) {
                hkey[j] = kEmpty;
                hval[j] = 0.0;
            }
            if (lane == 0) s_flag = 0;
            __syncthreads();
            int len = 0;
            if (lane < m - 1) {
                // members are entered tagged, with their position as the slot's value
                bool tg;
                const uint32_t c = (uint32_t)Qc[lane];
                const int slot = table_find<CAP>(hkey, c, c | kPBit, true, tg);
                if (slot >= 0) hval[slot] = (double)lane;
                else s_flag = 1;
                len = mlen[lane];
            } else if (lane == m - 1) {
                mbeg[lane] = ibeg;
                len = ilen;
            }
            const int incl = wave_incl_scan(len);
            if (lane < m) off[lane] = incl - len;
            const int total = __shfl(incl, m - 1, 64);
            if (lane == 0) off[m] = total;
            __syncthreads();
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
                        const int idx = mbeg[tseg] + (e - off[tseg]);
                        tt[u] = tseg;
                        cc[u] = __builtin_nontemporal_load(&ci[idx]);
                        vv[u] = __builtin_nontemporal_load(&av[idx]);
                    }
                }
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    if (cc[u] >= 0) {
                        bool tg = false;
                        const int slot = table_find<CAP>(hkey, (uint32_t)cc[u], (uint32_t)cc[u], true, tg);
                        if (slot < 0)
                            s_flag = 1;
                        else if (!tg)
                            __hip_atomic_fetch_add(&hval[slot], vv[u] * gq[tt[u]], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
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

            // ---- new positions m-1 .. m+ns-2 in selection order; i moves to mn-1
            const int mn = m + ns;
            if (lane < ns) {
                hval[selslot[lane]] = (double)(m - 1 + lane);
                Qc[m - 1 + lane] = sel[lane];
            }
            __syncthreads();

            // ---- 3./4. append the new rows to the factor, at most kGMax at a time
            bool spd = true;
            int mb = m - 1;
            for (int v0 = 0; v0 < ns && spd;) {
                int G = min(ns - v0, gmax);
                while (G > 1 && upd_entries(mb, G) > 64 * K) --G;
                const int m1 = mb + G;  // position of i within this update
                // gather rows sel[v0 .. v0+G): NR[v][pos] for members, NR[v][MMAX-1] = a_{u,i}
                for (int j = lane; j < G * MMAX; j += 64) NR[j] = 0.0;
                int rlen = 0;
                if (lane < G) {
                    const int u = sel[v0 + lane];
                    const int b = rp[u];
                    rlen = rp[u + 1] - b;
                    mbeg[mb + lane] = b;
                    nlo[lane] = 0;
                }
                const int rincl = wave_incl_scan(rlen);
                if (lane < G) nbeg[lane] = rincl - rlen;
                const int rtot = __shfl(rincl, G - 1, 64);
                if (lane == 0) nbeg[G] = rtot;
                __syncthreads();
                for (int e = lane; e < rtot; e += 64) {
                    const int v = seg_of(nbeg, G, e);
                    const int idx = mbeg[mb + v] + (e - nbeg[v]);
                    const int c = ci[idx];
                    if (c < i) {
                        atomicAdd(&nlo[v], 1);
                        bool tg = false;
                        const int slot = table_find<CAP>(hkey, (uint32_t)c, 0u, false, tg);
                        if (slot >= 0 && tg) NR[v * MMAX + (int)hval[slot]] = av[idx];
                    } else if (c == i) {
                        NR[v * MMAX + (MMAX - 1)] = av[idx];
                    }
                }
                __syncthreads();
                if (lane < G) mlen[mb + lane] = nlo[lane];

                // update entries owned by this lane: (row r, column c); r == G is the row of i
                const int E = upd_entries(mb, G);
                const int ibase = upd_index(mb, G, 0);
                int er[K], ec[K];
                double run[K];
#pragma unroll
                for (int kk = 0; kk < K; ++kk) {
                    const int e = kk * 64 + lane;
                    er[kk] = -1;
                    ec[kk] = 0;
                    run[kk] = 0.0;
                    if (e < E) {
                        if (e >= ibase) {
                            const int d = e - ibase;  // 0..G-1 new columns, G the diagonal
                            er[kk] = G;
                            ec[kk] = mb + d;
                            run[kk] = (d < G) ? NR[d * MMAX + (MMAX - 1)] : di;
                        } else {
                            int v = 0, rest = e;
                            while (rest >= mb + v + 1) {
                                rest -= mb + v + 1;
                                ++v;
                            }
                            er[kk] = v;
                            ec[kk] = rest;
                            run[kk] = NR[v * MMAX + rest];
                        }
                    }
                }
                for (int j = 0; j < m1; ++j) {
                    double dj;
                    if (j >= mb) {
                        // pivot of new row j - mb: its diagonal entry is final
                        const int e = upd_index(mb, j - mb, j);
                        double xd = 0.0;
#pragma unroll
                        for (int kk = 0; kk < K; ++kk)
                            if ((e >> 6) == kk) xd = rl(run[kk], e & 63);
                        if (!(xd > 0.0) || !isfinite(xd)) {
                            spd = false;
                            break;
                        }
                        const double Ljj = sqrt(xd);
                        dj = 1.0 / Ljj;
#pragma unroll
                        for (int kk = 0; kk < K; ++kk)
                            if ((e >> 6) == kk && lane == (e & 63)) run[kk] = Ljj;
                        if (lane == 0) dinv[j] = dj;
                    } else {
                        dj = dinv[j];
                    }
                    // values of column j: U[v] = L[mb+v][j], U[G] = L[i][j]
                    double U[kGMax + 1];
#pragma unroll
                    for (int v = 0; v <= kGMax; ++v) U[v] = 0.0;
#pragma unroll
                    for (int v = 0; v < kGMax; ++v) {
                        if (v < G && j < mb + v) {
                            const int e = upd_index(mb, v, j);
                            double xv = 0.0;
#pragma unroll
                            for (int kk = 0; kk < K; ++kk)
                                if ((e >> 6) == kk) xv = rl(run[kk], e & 63);
                            U[v] = xv * dj;
#pragma unroll
                            for (int kk = 0; kk < K; ++kk)
                                if ((e >> 6) == kk && lane == (e & 63)) run[kk] = U[v];
                        }
                    }
                    if (j < mb) {
                        U[kGMax] = li[j];
                    } else {
                        const int e = ibase + (j - mb);
                        double xv = 0.0;
#pragma unroll
                        for (int kk = 0; kk < K; ++kk)
                            if ((e >> 6) == kk) xv = rl(run[kk], e & 63);
                        U[kGMax] = xv * dj;
#pragma unroll
                        for (int kk = 0; kk < K; ++kk)
                            if ((e >> 6) == kk && lane == (e & 63)) run[kk] = U[kGMax];
                    }
                    // right-looking update of the entries right of column j
#pragma unroll
                    for (int kk = 0; kk < K; ++kk) {
                        const int r = er[kk], c = ec[kk];
                        const bool idiag = (r == G) && (c == m1);
                        if (r >= 0 && c > j && !(idiag && j < mb)) {
                            double a = U[kGMax];
#pragma unroll
                            for (int v = 0; v < kGMax; ++v)
                                if (v == r && r < G) a = U[v];
                            double b;
                            if (c < mb) {
                                b = Lp[tri(c, j)];
                            } else if (idiag) {
                                b = U[kGMax];
                            } else {
                                b = 0.0;
#pragma unroll
                                for (int v = 0; v < kGMax; ++v)
                                    if (v == c - mb) b = U[v];
                            }
                            run[kk] = run[kk] - a * b;
                        }
                    }
                }
                if (!spd) break;
                // store the appended rows, the last row's new entries and its running diagonal
#pragma unroll
                for (int kk = 0; kk < K; ++kk) {
                    const int r = er[kk], c = ec[kk];
                    if (r >= 0 && r < G) Lp[tri(mb + r, c)] = run[kk];
                    else if (r == G && c < m1) li[c] = run[kk];
                }
                {
                    const int e = ibase + G;
                    double xd = 0.0;
#pragma unroll
                    for (int kk = 0; kk < K; ++kk)
                        if ((e >> 6) == kk) xd = rl(run[kk], e & 63);
                    di = xd;
                }
                __syncthreads();
                mb += G;
                v0 += G;
            }
            if (spd && (!(di > 0.0) || !isfinite(di))) spd = false;
            if (!spd) {
                status = ROW_NOT_SPD;
                break;
            }

            // ---- 5. g = L^-T e_m, positions from the last down
            const double lmm = sqrt(di);
            const double dm = 1.0 / lmm;
            double acc = 0.0, gmine = 0.0;
            for (int l = mn - 1; l >= 0; --l) {
                const double gl = (l == mn - 1) ? dm : -(rl(acc, l) * dinv[l]);
                if (lane == l) gmine = gl;
                if (lane < l) {
                    const double Lv = (l == mn - 1) ? li[lane] : Lp[tri(l, lane)];
                    acc = acc + Lv * gl;
                }
            }
            if (lane < mn) gq[lane] = gmine;
            psi = lmm * lmm;
            m = mn;
            steps = k;
            __syncthreads();
            // ---- exit test (eq. exit_crit)
            if (psi <= eps * psi0) {
                reason = STOP_EPS;
                break;
            }
        }

        // ---- outputs: the row with ascending columns
        if (status == ROW_OK) {
            int col = 0x7fffffff;
            double val = 0.0;
            if (lane < m) {
                col = (lane == m - 1) ? i : Qc[lane];
                val = gq[lane];
            }
            int rank = 0;
            for (int t = 0; t < m; ++t) rank += (__shfl(col, t, 64) < col) ? 1 : 0;
            if (lane < m) {
                ell_col[(size_t)i * ldell + rank] = col;
                ell_val[(size_t)i * ldell + rank] = val;
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

typedef void (*RowsKernel)(int, const int32_t *, const int32_t *, const double *, const double *, const int32_t *,
                           int, int, double, double, int, const int32_t *, int, int32_t *, int, int32_t *, double *, int,
                           int32_t *, double *, int32_t *, int32_t *, int8_t *, int32_t *, int32_t *);

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

// LDS bytes of one k_afsai_rows<MMAX, CAP> block
__host__ __forceinline__ size_t rows_lds_bytes(int mmax_t, int cap) {
    return (size_t)cap * 12 + (size_t)mmax_t * (mmax_t - 1) / 2 * 8 + (size_t)mmax_t * (3 * 8 + 3 * 4) +
           (size_t)(mmax_t + 1) * 4 + (size_t)kGMax * mmax_t * 8 + 64 * 8 + (2 * kGMax + 1) * 4 + 8;
}

}  // namespace afsai
