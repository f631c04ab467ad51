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
// keys of the register-list form: column in bits 0..23, a member's position in bits 24..30
constexpr uint32_t kCol24 = 0x00FFFFFFu;
constexpr int kGMax = 4;  // rows appended to the factor together
#ifndef AFSAI_PROD_BATCH
#define AFSAI_PROD_BATCH 4
#endif
constexpr int kProdBatch = AFSAI_PROD_BATCH;

enum : int8_t { ROW_OK = 0, ROW_OVERFLOW = 1, ROW_BAD = 2, ROW_NOT_SPD = 3 };
enum : int32_t { STOP_KMAX = 0, STOP_EPS = 1, STOP_NOCAND = 2 };

__device__ __forceinline__ int tri(int p, int q) { return ((p * (p + 1)) >> 1) + q; }  // q <= p

template <int CAP>
__device__ __forceinline__ uint32_t hash0(uint32_t c) {
    constexpr int B = __builtin_ctz(CAP);
    return (c * 2654435761u) >> (32 - B);
}

// Finds column c in the table; inserts `ins` (c, possibly tagged) when absent and `insert` is
// set.  Returns the slot, -1 if absent (lookup only) or -2 if the table is full; `key` is the
// stored key.  KM masks the column out of a key.
template <int CAP, uint32_t KM = ~kPBit>
__device__ __forceinline__ int table_find(uint32_t *hkey, uint32_t c, uint32_t ins, bool insert, bool &tagged,
                                          uint32_t &key) {
    uint32_t slot = hash0<CAP>(c);
    for (int probe = 0; probe < CAP; ++probe) {
        uint32_t k = __hip_atomic_load(&hkey[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (k == kEmpty) {
            if (!insert) return -1;
            const uint32_t old = atomicCAS(&hkey[slot], kEmpty, ins);
            if (old == kEmpty) {
                tagged = (ins & kPBit) != 0;
                key = ins;
                return (int)slot;
            }
            k = old;
        }
        if ((k & KM) == c) {
            tagged = (k & kPBit) != 0;
            key = k;
            return (int)slot;
        }
        slot = (slot + 1) & (CAP - 1);
    }
    return -2;
}

// value of v in lane `src` (src uniform)
__device__ __forceinline__ double rl(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float rl(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// One factor update that appends G rows (positions mb .. mb+G-1; the rows of L for the positions
// below mb are final) and moves the last row (row i) behind them.  Lane l holds column l: R[v]
// the running value of entry (mb + v, l) and, for the new columns l >= mb, R[GA] the running
// value of entry (i, l).  Columns are taken left to right; column j's values of the new rows
// (and of row i) are scaled by the pivot reciprocal, broadcast, and every entry right of column
// j receives its product term (right-looking), so each entry gets the operations of a
// column-by-column factorisation in the same order.  Column j of the new rows goes to Lp; the
// last row's entries of the old columns are final already and its diagonal `di` receives the
// squares of its new entries.  Returns false on a pivot that is not positive.
template <int G, int GA, typename T>
__device__ __forceinline__ bool upd_lanes(int mb, T (&R)[GA + 1], T &r_dinv, T &r_li, T &di,
                                          T *Lp, int lane) {
    static_assert(G <= GA, "group fits the register array");
    const int m1 = mb + G;  // position of i after the update
    const int rowbase = tri(lane, 0);
    for (int j = 0; j < m1; ++j) {
        T U[G], A;
        if (j < mb) {
            const T dj = rl(r_dinv, j);
#pragma unroll
            for (int v = 0; v < G; ++v) U[v] = rl(R[v], j) * dj;
            A = rl(r_li, j);
        } else {
            // pivot of new row w = j - mb: its diagonal entry has all its terms
            const int w = j - mb;
            T xd = T(0);
#pragma unroll
            for (int v = 0; v < G; ++v)
                if (v == w) xd = rl(R[v], j);
            if (!(xd > T(0)) || !isfinite(xd)) return false;
            const T Ljj = sqrt(xd);
            const T dj = T(1) / Ljj;
#pragma unroll
            for (int v = 0; v < G; ++v) U[v] = (v == w) ? Ljj : rl(R[v], j) * dj;  // rows v < w unused
            A = rl(R[GA], j) * dj;                                                   // L[i][j]
            if (lane == j) {
                r_dinv = dj;
                r_li = A;
            }
            di = di - A * A;
        }
        if (lane == 0) {
#pragma unroll
            for (int v = 0; v < G; ++v)
                if (j < mb + v + 1) Lp[tri(mb + v, j)] = U[v];
        }
        if (lane > j && lane < m1) {
            T b = (lane < mb) ? Lp[rowbase + j] : U[0];
#pragma unroll
            for (int v = 1; v < G; ++v)
                if (lane == mb + v) b = U[v];
#pragma unroll
            for (int v = 0; v < G; ++v) R[v] = R[v] - U[v] * b;
            R[GA] = R[GA] - A * b;
        }
    }
    return true;
}

// Slot-list entries per table slot: each member row's entries left of column i are looked up
// once, when the row joins the pattern, and their table slots are kept for the later steps.
template <int CAP>
constexpr int sl_cap() { return CAP >= 2048 ? 2 * CAP : 4 * CAP; }

// RSL: the slot lists live in registers (rows of at most 128 entries: lane l keeps the slots of
// entries l and 64 + l of every member, packed in one 32-bit register per member) instead of LDS,
// which frees LDS for more resident rows; in this form a member's position is kept in its table
// key (columns below 2^24), the gathered rows share the gradient's array (not in use from the
// selection to the next product pass) and the rows of L are sized by the launch (dynamic LDS).
// Register budget of the register-list form: patterns of at most 32 positions with at most 512
// table slots fit 20 rows per CU in LDS, and 5 waves per SIMD measured faster than 4 without
// spills; the smallest patterns target 8.  Larger patterns and tables are limited by LDS, and
// the compiler keeps all their registers.
template <int MMAX, int CAP, bool RSL, typename T>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(!RSL ? 1 : (MMAX <= 8 && CAP <= 256) ? 8 : ((MMAX <= 32 && CAP <= 512) ? (sizeof(T) == 4 ? 6 : 5) : 1), 8))) void k_afsai_rows(
    int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, const double *__restrict__ av,
    const float *__restrict__ /* FP32 gradient values: inverse-factor form only */,
    const double *__restrict__ diag, const int32_t *__restrict__ dlo, int kmax, int s, double eps, double tau,
    int gmax, const int32_t *__restrict__ list, int nlist, int32_t *__restrict__ counters, int nxcd, int claim,
    int32_t *__restrict__ ell_col, double *__restrict__ ell_val, int ldell, int32_t *__restrict__ m_out,
    double *__restrict__ psi_out, int32_t *__restrict__ steps_out, int32_t *__restrict__ reason_out,
    int8_t *__restrict__ status_out, int32_t *__restrict__ ovf_count, int32_t *__restrict__ ovf_list) {
    static_assert(MMAX <= 64, "one lane per pattern position");
    static_assert(!RSL || MMAX <= 64, "positions fit the 7-bit field of a key");
    constexpr bool NR_ALIAS = RSL && CAP >= kGMax * MMAX;  // gathered rows in the gradient array
    constexpr uint32_t KM = RSL ? kCol24 : ~kPBit;
    constexpr int QB = kProdBatch;  // members whose entries one product round loads together (RSL)
    // rows one factor update appends at most: 2 up to 32 positions (the running values of the
    // appended rows stay in registers; 4 would spill at the 5-wave budget), else kGMax
    constexpr int GCAP = MMAX <= 32 ? 2 : kGMax;
    constexpr int LTRI = (MMAX * (MMAX - 1)) / 2;  // rows 0..MMAX-2 of L, packed lower
    constexpr int SPL = CAP / 64;                  // table slots per lane
    constexpr bool SEL_REG = SPL <= 16;            // selection from registers
    constexpr int SLCAP = RSL ? 1 : sl_cap<CAP>();
    __shared__ uint32_t hkey[CAP];       // column (tagged when a member), kept for the whole row
    __shared__ T hval[CAP];         // gradient of this step
    __shared__ int8_t hpos[RSL ? 1 : CAP];                 // position of a member
    __shared__ uint16_t SL[SLCAP];                         // table slots of the member rows' entries left of i
    __shared__ T Lp_s[RSL ? 1 : LTRI];                // rows of L for the off-diagonal positions
    __shared__ T NR_s[NR_ALIAS ? 1 : kGMax * MMAX];   // gathered new rows, by position (a_{u,i} at MMAX-1)
    extern __shared__ __align__(8) unsigned char lds_dyn_b[];  // RSL: rows of L, sized by the launch
    T *const Lp = RSL ? reinterpret_cast<T *>(lds_dyn_b) : Lp_s;
    const T epsT = (T)eps, tauT = (T)tau;
    T *const NR = NR_ALIAS ? hval : NR_s;
    __shared__ int32_t s_row;

    const int lane = threadIdx.x;
    const int x = blockIdx.x % nxcd;
    const int64_t per = ((int64_t)nlist + nxcd - 1) / nxcd;
    const int q0 = (int)min<int64_t>(nlist, per * x), q1 = (int)min<int64_t>(nlist, per * (x + 1));

    // rows are claimed `claim` at a time from the XCD's counter (one atomic per claim)
    int qn = 0, qe = 0;
    for (;;) {
        if (qn >= qe) {
            if (lane == 0) s_row = q0 + atomicAdd(&counters[x], claim);
            __syncthreads();
            qn = s_row;
            __syncthreads();
            if (qn >= q1) break;
            qe = min(qn + claim, q1);
        }
        const int i = list ? list[qn] : qn;
        ++qn;

        // per-position state, lane t = position t (i at m-1): column, row start, number of
        // row entries left of column i, their offset in SL, scaled row value, reciprocal
        // pivot, L[i][t]
        int r_col = i, r_beg = 0, r_len = 0, r_so = 0;
        T r_g = T(0), r_dinv = T(0), r_li = T(0);
        int r_nb = 0, r_ne = 0;  // row extents of the columns selected in this step (lane = rank)

        // ---- G_0 = I scaled: P = {i}, g = a_ii^-1/2, psi_0 = a_ii
        const T aii = (T)diag[i];
        const int ibeg = rp[i], ilen = dlo[i];
        int8_t status = ROW_OK;
        int m = 1, steps = 0;
        int32_t reason = STOP_KMAX;
        T psi = aii;
        T di = aii;  // last row's diagonal less the squares of its final entries
        if (!(aii > T(0)) || !isfinite(aii)) status = ROW_NOT_SPD;
        const T psi0 = aii;
        int sl_used = 0;  // SL entries in use (uniform)
        // register slot lists: member 0 is row i, member t + 1 the column at position t
        uint32_t slr[RSL ? MMAX : 1];
#pragma unroll
        for (int q = 0; q < (RSL ? MMAX : 1); ++q) slr[q] = 0u;

        // table: empty; row i's entries left of the diagonal are entered as candidates
        for (int j = lane; j < CAP; j += 64) hkey[j] = kEmpty;
        __syncthreads();
        if (kmax > 0 && status == ROW_OK) {
            bool ovf = RSL ? ilen > 128 : ilen > SLCAP;
            for (int o = lane; o < ilen && !ovf; o += 64) {
                bool tg;
                uint32_t kf;
                const int slot = table_find<CAP, KM>(hkey, (uint32_t)ci[ibeg + o], (uint32_t)ci[ibeg + o], true, tg, kf);
                if (slot < 0) ovf = true;
                else if constexpr (RSL) slr[0] |= (uint32_t)slot << (o >= 64 ? 16 : 0);
                else SL[o] = (uint16_t)slot;
            }
            if (__ballot(ovf)) status = ROW_OVERFLOW;
            sl_used = ilen;
        }
        if (lane == 0) {
            r_g = T(1) / sqrt(aii);
            r_beg = ibeg;
            r_len = ilen;
            r_so = 0;
        }
        __syncthreads();

        for (int k = 1; k <= kmax && status == ROW_OK; ++k) {
            // ---- 1. product pass: v_c += a_rc g_r over the members' entries left of i (the
            //         slots of members collect values that are never read)
            for (int j = lane; j < CAP; j += 64) hval[j] = T(0);
            __syncthreads();
            if constexpr (RSL) {
#pragma unroll
                for (int q0 = 0; q0 < MMAX; q0 += QB) {
                    if (q0 < m) {
                        int sl[2 * QB];
                        T aa[2 * QB], gg[QB];
                        int lens[QB], begs[QB];
#pragma unroll
                        for (int u = 0; u < QB; ++u) {
                            const int q = q0 + u;
                            const int pos = (q == 0) ? m - 1 : q - 1;
                            lens[u] = 0;
                            begs[u] = 0;
                            gg[u] = T(0);
                            if (q < m) {
                                lens[u] = __builtin_amdgcn_readlane(r_len, pos);
                                begs[u] = __builtin_amdgcn_readlane(r_beg, pos);
                                gg[u] = rl(r_g, pos);
                            }
#pragma unroll
                            for (int hh = 0; hh < 2; ++hh) {
                                const int o = hh * 64 + lane;
                                sl[2 * u + hh] = -1;
                                aa[2 * u + hh] = T(0);
                                if (o < lens[u]) {
                                    sl[2 * u + hh] = (int)((slr[q] >> (16 * hh)) & 0xffffu);
                                    aa[2 * u + hh] = (T)__builtin_nontemporal_load(&av[begs[u] + o]);
                                }
                            }
                        }
#pragma unroll
                        for (int u = 0; u < QB; ++u)
#pragma unroll
                            for (int hh = 0; hh < 2; ++hh)
                                if (sl[2 * u + hh] >= 0)
                                    __hip_atomic_fetch_add(&hval[sl[2 * u + hh]], aa[2 * u + hh] * gg[u],
                                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                }
            } else {
                for (int t0 = 0; t0 < m; t0 += 4) {
                    int sl[8];
                    T aa[8], gg[4];
                    int lens[4], begs[4], sos[4];
    #pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int t = t0 + u;
                        lens[u] = 0;
                        begs[u] = 0;
                        sos[u] = 0;
                        gg[u] = T(0);
                        if (t < m) {
                            lens[u] = __builtin_amdgcn_readlane(r_len, t);
                            begs[u] = __builtin_amdgcn_readlane(r_beg, t);
                            sos[u] = __builtin_amdgcn_readlane(r_so, t);
                            gg[u] = rl(r_g, t);
                        }
    #pragma unroll
                        for (int hh = 0; hh < 2; ++hh) {
                            const int o = hh * 64 + lane;
                            sl[2 * u + hh] = -1;
                            aa[2 * u + hh] = T(0);
                            if (o < lens[u]) {
                                sl[2 * u + hh] = SL[sos[u] + o];
                                aa[2 * u + hh] = (T)__builtin_nontemporal_load(&av[begs[u] + o]);
                            }
                        }
                    }
    #pragma unroll
                    for (int u = 0; u < 4; ++u)
    #pragma unroll
                        for (int hh = 0; hh < 2; ++hh)
                            if (sl[2 * u + hh] >= 0)
                                __hip_atomic_fetch_add(&hval[sl[2 * u + hh]], aa[2 * u + hh] * gg[u], __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_WORKGROUP);
    #pragma unroll
                    for (int u = 0; u < 4; ++u)
                        for (int o = 128 + lane; o < lens[u]; o += 64)
                            __hip_atomic_fetch_add(&hval[SL[sos[u] + o]], (T)av[begs[u] + o] * gg[u], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            }
            __syncthreads();

            // ---- 2. selection (top-s of |v| over the candidates, tie band, smallest column);
            //         the j-th selected column takes position m-1+j, and its row extents are
            //         fetched at once into lane j
            int ns = 0;
            if constexpr (SEL_REG) {
                uint32_t kr[SPL];
                T ar[SPL];
                T lm = T(-1);
#pragma unroll
                for (int j = 0; j < SPL; ++j) {
                    const uint32_t kk = hkey[lane + 64 * j];
                    const bool cand = (kk != kEmpty) && !(kk & kPBit);
                    kr[j] = cand ? kk : kEmpty;
                    ar[j] = cand ? fabs(hval[lane + 64 * j]) : T(-1);
                    lm = fmax(lm, ar[j]);
                }
                const T M = wave_max_dpp(lm);
                if (M > T(0)) {
                    const T thr = T(0x1.0p-40) * M;
                    for (int round = 0; round < s; ++round) {
                        // the first round's largest eligible value is M itself (M > thr)
                        T Mp = M;
                        if (round > 0) {
                            T l = T(0);
#pragma unroll
                            for (int j = 0; j < SPL; ++j)
                                if (ar[j] > thr) l = fmax(l, ar[j]);
                            Mp = wave_max_dpp(l);
                        }
                        if (!(Mp > T(0))) break;
                        const T band = (T(1) - tauT) * Mp;
                        uint32_t lb = kEmpty;
#pragma unroll
                        for (int j = 0; j < SPL; ++j)
                            if (ar[j] > thr && ar[j] >= band && kr[j] < lb) lb = kr[j];
                        const uint32_t js = wave_min_dpp(lb);
                        int myslot = -1;
#pragma unroll
                        for (int j = 0; j < SPL; ++j) {
                            const bool hit = (kr[j] == js);
                            myslot = hit ? lane + 64 * j : myslot;
                            kr[j] = hit ? kEmpty : kr[j];
                            ar[j] = hit ? T(-1) : ar[j];
                        }
                        const uint64_t who = __ballot(myslot >= 0);
                        const int wslot = __builtin_amdgcn_readlane(myslot, (int)__builtin_ctzll(who));
                        if (lane == 0) {
                            if constexpr (RSL) {
                                hkey[wslot] = js | kPBit | ((uint32_t)(m - 1 + ns) << 24);
                            } else {
                                hkey[wslot] = js | kPBit;
                                hpos[wslot] = (int8_t)(m - 1 + ns);
                            }
                        }
                        if (lane == ns) {
                            r_nb = rp[js];
                            r_ne = rp[js + 1];
                        }
                        if (lane == m - 1 + ns) r_col = (int)js;
                        ++ns;
                    }
                }
            } else {
                T lm = T(0);
                for (int j = lane; j < CAP; j += 64) {
                    const uint32_t kk = hkey[j];
                    if (kk != kEmpty && !(kk & kPBit)) lm = fmax(lm, fabs(hval[j]));
                }
                const T M = wave_max_dpp(lm);
                if (M > T(0)) {
                    const T thr = T(0x1.0p-40) * M;
                    for (int round = 0; round < s; ++round) {
                        T Mp = M;
                        if (round > 0) {
                            T l = T(0);
                            for (int j = lane; j < CAP; j += 64) {
                                const uint32_t kk = hkey[j];
                                if (kk != kEmpty && !(kk & kPBit)) {
                                    const T a = fabs(hval[j]);
                                    if (a > thr) l = fmax(l, a);
                                }
                            }
                            Mp = wave_max_dpp(l);
                        }
                        if (!(Mp > T(0))) break;
                        const T band = (T(1) - tauT) * Mp;
                        uint32_t lb = kEmpty;
                        for (int j = lane; j < CAP; j += 64) {
                            const uint32_t kk = hkey[j];
                            if (kk != kEmpty && !(kk & kPBit)) {
                                const T a = fabs(hval[j]);
                                if (a > thr && a >= band && kk < lb) lb = kk;
                            }
                        }
                        const uint32_t js = wave_min_dpp(lb);
                        for (int j = lane; j < CAP; j += 64)
                            if (hkey[j] == js) {
                                if constexpr (RSL) {
                                    hkey[j] = js | kPBit | ((uint32_t)(m - 1 + ns) << 24);
                                } else {
                                    hkey[j] = js | kPBit;
                                    hpos[j] = (int8_t)(m - 1 + ns);
                                }
                            }
                        if (lane == ns) {
                            r_nb = rp[js];
                            r_ne = rp[js + 1];
                        }
                        if (lane == m - 1 + ns) r_col = (int)js;
                        ++ns;
                        __syncthreads();
                    }
                }
            }
            __syncthreads();
            if (ns == 0) {
                reason = STOP_NOCAND;
                break;
            }

            // ---- 3./4. append the new rows to the factor, at most gmax at a time
            const int mn = m + ns;
            bool spd = true, ovf = false;
            int mb = m - 1;
            for (int v0 = 0; v0 < ns && spd && !ovf;) {
                const int G = min(ns - v0, min(gmax, GCAP));
                const int m1 = mb + G;  // position of i within this update
                // gather rows v0 .. v0+G-1: NR[v][pos] for members, NR[v][MMAX-1] = a_{u,i};
                // their entries left of i are entered in the table and their slots listed
                for (int j = lane; j < G * MMAX; j += 64) NR[j] = T(0);
                __syncthreads();
                if constexpr (RSL && MMAX >= 16) {
                    // rows of at most 128 entries: every new row's entries are loaded first, so
                    // that their latencies overlap, then entered in the table (not for the
                    // smallest patterns, whose registers it would spill)
                    int gnb[kGMax], gnl[kGMax], gc[kGMax][2];
                    T ga[kGMax][2];
#pragma unroll
                    for (int v = 0; v < kGMax; ++v) {
                        gnb[v] = 0;
                        gnl[v] = 0;
                        if (v < G) {
                            gnb[v] = __builtin_amdgcn_readlane(r_nb, v0 + v);
                            gnl[v] = __builtin_amdgcn_readlane(r_ne, v0 + v) - gnb[v];
                        }
                        if (gnl[v] > 128) ovf = true;  // uniform
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const int o = h * 64 + lane;
                            gc[v][h] = 0x7fffffff;
                            ga[v][h] = T(0);
                            if (o < gnl[v] && o < 128) {
                                gc[v][h] = ci[gnb[v] + o];
                                ga[v][h] = (T)av[gnb[v] + o];
                            }
                        }
                    }
#pragma unroll
                    for (int v = 0; v < kGMax; ++v) {
                        if (v < G && !ovf) {
                            int nlo = 0;
                            uint32_t pk = 0u;
#pragma unroll
                            for (int h = 0; h < 2; ++h) {
                                if (h * 64 < gnl[v]) {
                                    const int c = gc[v][h];
                                    const T a = ga[v][h];
                                    if (c == i) NR[v * MMAX + (MMAX - 1)] = a;
                                    bool bad = false;
                                    if (c < i) {
                                        bool tg = false;
                                        uint32_t kf = 0u;
                                        const int slot =
                                            table_find<CAP, KM>(hkey, (uint32_t)c, (uint32_t)c, true, tg, kf);
                                        if (slot < 0) {
                                            bad = true;
                                        } else {
                                            pk |= (uint32_t)slot << (16 * h);
                                            if (tg) NR[v * MMAX + (int)((kf >> 24) & 0x7Fu)] = a;
                                        }
                                    }
                                    nlo += __popcll(__ballot(c < i));
                                    if (__ballot(bad)) ovf = true;
                                }
                            }
                            if (lane == mb + v) {
                                r_beg = gnb[v];
                                r_len = nlo;
                            }
                            const int qn = mb + v + 1;  // member of position mb + v
#pragma unroll
                            for (int qq = 1; qq < (RSL ? MMAX : 1); ++qq)
                                if (qq == qn) slr[qq] = pk;
                        }
                    }
                } else
                for (int v = 0; v < G; ++v) {
                    const int nb = __builtin_amdgcn_readlane(r_nb, v0 + v);
                    const int nl = __builtin_amdgcn_readlane(r_ne, v0 + v) - nb;
                    if (!RSL && sl_used + nl > SLCAP) ovf = true;  // uniform
                    if (RSL && nl > 128) ovf = true;
                    int nlo = 0;
                    uint32_t pk = 0u;  // register slot list of this row (RSL)
                    for (int h = 0; h * 64 < nl && !ovf; ++h) {
                        const int o = h * 64 + lane;
                        int c = 0x7fffffff;
                        T a = T(0);
                        if (o < nl) {
                            c = ci[nb + o];
                            a = (T)av[nb + o];
                        }
                        if (c == i) NR[v * MMAX + (MMAX - 1)] = a;
                        bool bad = false;
                        if (c < i) {
                            bool tg = false;
                            uint32_t kf = 0u;
                            const int slot = table_find<CAP, KM>(hkey, (uint32_t)c, (uint32_t)c, true, tg, kf);
                            if (slot < 0) {
                                bad = true;
                            } else {
                                if constexpr (RSL) pk |= (uint32_t)slot << (16 * h);
                                else SL[sl_used + o] = (uint16_t)slot;
                                if (tg) NR[v * MMAX + (RSL ? (int)((kf >> 24) & 0x7Fu) : (int)hpos[slot])] = a;
                            }
                        }
                        nlo += __popcll(__ballot(c < i));
                        if (__ballot(bad)) ovf = true;
                    }
                    if (lane == mb + v) {
                        r_beg = nb;
                        r_len = nlo;
                        r_so = sl_used;
                    }
                    if constexpr (RSL) {
                        const int qn = mb + v + 1;  // member of position mb + v
#pragma unroll
                        for (int qq = 1; qq < (RSL ? MMAX : 1); ++qq)
                            if (qq == qn) slr[qq] = pk;
                    }
                    sl_used += nlo;
                }
                __syncthreads();
                if (ovf) break;

                // factor update: lane l holds the running values of column l for the new rows
                // (R[v] = entry (mb + v, l)) and, for the new columns, of the last row (R[G])
                T R[GCAP + 1];
#pragma unroll
                for (int v = 0; v < GCAP; ++v) R[v] = (v < G && lane < m1) ? NR[v * MMAX + lane] : T(0);
                R[GCAP] = T(0);
#pragma unroll
                for (int w = 0; w < GCAP; ++w)
                    if (w < G && lane == mb + w) R[GCAP] = NR[w * MMAX + (MMAX - 1)];
                switch (G) {
                    case 1: spd = upd_lanes<1, GCAP, T>(mb, R, r_dinv, r_li, di, Lp, lane); break;
                    case 2: spd = upd_lanes<(GCAP < 2 ? GCAP : 2), GCAP, T>(mb, R, r_dinv, r_li, di, Lp, lane); break;
                    case 3: spd = upd_lanes<(GCAP < 3 ? GCAP : 3), GCAP, T>(mb, R, r_dinv, r_li, di, Lp, lane); break;
                    default: spd = upd_lanes<GCAP, GCAP, T>(mb, R, r_dinv, r_li, di, Lp, lane); break;
                }
                if (!spd) break;
                __syncthreads();
                mb += G;
                v0 += G;
            }
            if (ovf) {
                status = ROW_OVERFLOW;
                break;
            }
            if (spd && (!(di > T(0)) || !isfinite(di))) spd = false;
            if (!spd) {
                status = ROW_NOT_SPD;
                break;
            }

            // ---- 5. g = L^-T e_m, positions from the last down
            const T lmm = sqrt(di);
            const T dm = T(1) / lmm;
            // l = mn-1 (row i of L), then the stored rows; lane t accumulates sum_l L[l][t] g_l
            T gmine = (lane == mn - 1) ? dm : T(0);
            T acc = (lane < mn - 1) ? T(0) + r_li * dm : T(0);
            for (int l = mn - 2; l >= 0; --l) {
                const T Lv = Lp[tri(l, lane < l ? lane : 0)];
                const T gl = -(rl(acc, l) * rl(r_dinv, l));
                gmine = (lane == l) ? gl : gmine;
                const T na = acc + Lv * gl;
                acc = (lane < l) ? na : acc;
            }
            if (lane < mn) r_g = gmine;
            if (lane == mn - 1) {
                r_beg = ibeg;
                r_len = ilen;
                r_so = 0;
            }
            psi = lmm * lmm;
            m = mn;
            steps = k;
            // ---- exit test (eq. exit_crit)
            if (psi <= epsT * psi0) {
                reason = STOP_EPS;
                break;
            }
        }

        // ---- outputs: the row with ascending columns
        if (status == ROW_OK) {
            const int col = (lane < m - 1) ? r_col : (lane == m - 1 ? i : 0x7fffffff);
            int rank = 0;
            for (int t = 0; t < m; ++t) rank += (__builtin_amdgcn_readlane(col, t) < col) ? 1 : 0;
            if (lane < m) {
                ell_col[(size_t)i * ldell + rank] = col;
                ell_val[(size_t)i * ldell + rank] = r_g;
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

typedef void (*RowsKernel)(int, const int32_t *, const int32_t *, const double *, const float *, const double *,
                           const int32_t *,
                           int, int, double, double, int, const int32_t *, int, int32_t *, int, int, int32_t *, double *, int,
                           int32_t *, double *, int32_t *, int32_t *, int8_t *, int32_t *, int32_t *);

template <int MMAX, bool RSL, typename T = double>
static RowsKernel rows_kernel_cap(int cap) {
    switch (cap) {
        case 128: return k_afsai_rows<MMAX, 128, RSL, T>;
        case 256: return k_afsai_rows<MMAX, 256, RSL, T>;
        case 512: return k_afsai_rows<MMAX, 512, RSL, T>;
        case 1024: return k_afsai_rows<MMAX, 1024, RSL, T>;
        case 2048: return k_afsai_rows<MMAX, 2048, RSL, T>;
        case 4096: return k_afsai_rows<MMAX, 4096, RSL, T>;
        case 8192: return k_afsai_rows<MMAX, 8192, RSL, T>;
        default: return nullptr;
    }
}

// dynamic LDS bytes of one k_afsai_rows<MMAX, CAP, RSL, T> block (rows 0..mmax-2 of L; RSL
// only); tb = sizeof(T)
__host__ __forceinline__ size_t rows_lds_dyn_bytes(int mmax, bool rsl, int tb = 8) {
    return rsl ? (size_t)(mmax > 1 ? mmax - 1 : 1) * (size_t)mmax / 2 * tb + 8 : 0;
}
// LDS bytes of one k_afsai_rows<MMAX, CAP, RSL, T> block, static and dynamic
__host__ __forceinline__ size_t rows_lds_bytes(int mmax_t, int mmax, int cap, bool rsl, int tb = 8) {
    if (rsl) {
        const size_t nr = (size_t)cap >= (size_t)kGMax * mmax_t ? tb : (size_t)kGMax * mmax_t * tb;
        return (size_t)cap * (4 + tb) + 2 + 8 + nr + rows_lds_dyn_bytes(mmax, rsl, tb) + 16;
    }
    const size_t slcap = cap >= 2048 ? 2 * (size_t)cap : 4 * (size_t)cap;
    return (size_t)cap * 13 + slcap * 2 + (size_t)mmax_t * (mmax_t - 1) / 2 * 8 + (size_t)kGMax * mmax_t * 8 + 16;
}

}  // namespace afsai
