// Group-per-row CSR products and the PCG iteration (Sec. 3 "miniwarp" SpMV; Sec. 5.2 PCG).
//
// SpMV: a group of GS lanes (GS in {4, 8, 16, 32, 64}, chosen from the average row length like
// the paper's miniwarps, but sized for 64-lane wavefronts) owns one row; lanes stride through
// the row's entries with coalesced, non-temporal loads of the matrix and cached loads of x;
// the group reduces with cross-lane shuffles in a fixed order.  Each block owns one
// contiguous range of rows and blocks are renumbered so that every XCD streams one contiguous
// part of the matrix (its L2 then holds the x entries its rows share).
//
// Batches: the solver always runs over a batch of independent systems (one system for
// pcg_solve).  Each system keeps its own scalars and done flag; every launch maps its blocks
// to (system, block within the system) with the block count a single-system solve of that
// system would use, and dot products are summed per system over exactly those blocks, so a
// system's iterates do not depend on its batch-mates (bit for bit).
//
// PCG: all scalars (rho, alpha, beta, ||r||) live on the device.  Dot products are fused into
// the kernel that produces one of their operands, which stores one partial sum per block; a
// one-block kernel then adds the partials in block order (results do not depend on
// scheduling) and updates the scalars.  (A last-block-done reduction inside the producing
// kernel needs a device-scope release per block, which on this 8-XCD part writes back the
// L2 and cost more than the extra launch.)  A device flag ends the iteration: kernels that
// see it return at once, so the host enqueues chunks of iterations and reads the flag once
// per chunk, one chunk behind.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>
#include <vector>

#include "handle.hpp"

namespace afsai {

constexpr int kThreads = 256;
constexpr int kFusedMaxRows = 200000;  // automatic PCG form: fused products below this size
// resumable solver: iterations of the first chunk, least GPU time of a chunk and its share of
// the GPU time so far
constexpr int kFirstChunk = 4;
constexpr double kMinChunkUs = 100.0;
constexpr double kChunkShare = 0.125;

enum : int { FIN_NONE = 0, FIN_ALPHA = 1, FIN_BETA = 2, FIN_RHO0 = 3, FIN_INIT = 4, FIN_UPDATE = 5, FIN_RESID = 6 };
enum : int { DONE_NO = 0, DONE_CONVERGED = 1, DONE_NOT_SPD = 2, DONE_MAXIT = 3, DONE_ZERO_RHS = 4 };

struct PcgScalars {  // 80 bytes: copied as 10 double words
    double rho;      // r.z of the current iterate
    double alpha;
    double beta;
    double rr;       // ||r||^2
    double bb;       // ||b||^2
    double tol;      // rtol * ||b||
    double rtol;
    int32_t it;      // iterations completed
    int32_t maxit;
    int32_t done;    // DONE_*
    int32_t plain;   // 1: M = I (z = r)
    double resid;    // ||b - A x||^2 of the final check
};
static_assert(sizeof(PcgScalars) == 80, "PcgScalars is copied as 10 double words");

// Systems of a batch (device arrays; nullptr: one system covering everything)
struct Systems {
    const int32_t *row0 = nullptr;    // [nsys + 1] first row of each system
    const int32_t *slice0 = nullptr;  // [nsys + 1] first SELL slice of each system
};
// Blocks of one launch shape (device arrays; nullptr: one system, block b = its block b)
struct Map {
    const int32_t *blk_sys = nullptr;  // [nblocks] system of each (logical) block
    const int32_t *sys_b0 = nullptr;   // [nsys] first block of each system
    const int32_t *sys_nb = nullptr;   // [nsys] blocks of each system
};

struct Job {
    int k;   // system
    int lb;  // block within the system
    int nb;  // blocks of the system
    int gb;  // logical block of the launch (index of the partial sums)
};

__device__ __forceinline__ Job block_job(const Map &mp, int nxcd) {
    Job j;
    j.gb = xcd_block(blockIdx.x, gridDim.x, nxcd);
    if (mp.blk_sys) {
        j.k = mp.blk_sys[j.gb];
        j.lb = j.gb - mp.sys_b0[j.k];
        j.nb = mp.sys_nb[j.k];
    } else {
        j.k = 0;
        j.lb = j.gb;
        j.nb = gridDim.x;
    }
    return j;
}

// [lo, hi) of the `count` items starting at `base` that block lb of nb owns
__device__ __forceinline__ void block_range(int base, int count, int lb, int nb, int &lo, int &hi) {
    const int64_t per = ((int64_t)count + nb - 1) / nb;
    lo = base + (int)min<int64_t>(count, per * lb);
    hi = base + (int)min<int64_t>(count, per * (lb + 1));
}

__device__ __forceinline__ void sys_rows(const Systems &sy, int n, int k, int &r0, int &r1) {
    if (sy.row0) {
        r0 = sy.row0[k];
        r1 = sy.row0[k + 1];
    } else {
        r0 = 0;
        r1 = n;
    }
}

// ---------------------------------------------------------------------------------------
// block helpers
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double *sh /* >= kThreads/64 */) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < kThreads / 64; ++k) t += sh[k];
    __syncthreads();
    return t;  // valid in thread 0
}

// thread 0 stores this block's partial sums, slot k at partials[k * gridDim.x + gb], gb being
// the logical block (blocks of one system are consecutive and cover its rows in order)
__device__ __forceinline__ void store_partials(double *partials, int slots, const double *mine, int gb) {
    if (threadIdx.x == 0)
        for (int k = 0; k < slots; ++k) partials[(size_t)k * gridDim.x + gb] = mine[k];
}

// One block per system: sums the system's partials of the previous launch (nblocks blocks in
// all) in block order and updates its scalars.
__global__ __launch_bounds__(kThreads) void k_finalize(const double *__restrict__ partials, int nblocks, Map mp,
                                                       int fin, PcgScalars *scs) {
    const int k = blockIdx.x;
    PcgScalars *sc = scs + k;
    if ((fin == FIN_ALPHA || fin == FIN_BETA || fin == FIN_UPDATE || fin == FIN_RHO0) && sc->done) return;
    const int b0 = mp.blk_sys ? mp.sys_b0[k] : 0;
    const int nparts = mp.blk_sys ? mp.sys_nb[k] : nblocks;
    __shared__ double sh[kThreads / 64];
    const int slots = (fin == FIN_INIT) ? 2 : 1;
    double tot[2] = {0.0, 0.0};
    const int per = (nparts + kThreads - 1) / kThreads;
    const int lo = threadIdx.x * per, hi = min(nparts, lo + per);
    for (int sl = 0; sl < slots; ++sl) {
        double v = 0.0;
        for (int j = lo; j < hi; ++j) v += partials[(size_t)sl * nblocks + b0 + j];
        tot[sl] = block_sum(v, sh);
    }
    if (threadIdx.x != 0) return;
    const double v = tot[0];
    switch (fin) {
        case FIN_ALPHA:  // v = p.q
            if (!(v > 0.0) || !isfinite(v)) sc->done = DONE_NOT_SPD;
            else sc->alpha = sc->rho / v;
            break;
        case FIN_BETA:  // v = r.z
            sc->beta = v / sc->rho;
            sc->rho = v;
            break;
        case FIN_RHO0:
            sc->rho = v;
            break;
        case FIN_INIT: {  // v = b.b, tot[1] = r.r
            const double bb = v, rr = tot[1];
            sc->bb = bb;
            sc->rr = rr;
            sc->tol = sc->rtol * sqrt(bb);
            sc->it = 0;
            if (bb == 0.0) sc->done = DONE_ZERO_RHS;
            else if (sqrt(rr) <= sc->tol) sc->done = DONE_CONVERGED;
            else if (sc->maxit == 0) sc->done = DONE_MAXIT;
            if (sc->plain) sc->rho = rr;
            break;
        }
        case FIN_UPDATE:  // v = r.r after the update
            sc->rr = v;
            sc->it += 1;
            if (sqrt(v) <= sc->tol) sc->done = DONE_CONVERGED;
            else if (sc->it >= sc->maxit) sc->done = DONE_MAXIT;
            else if (sc->plain) {
                sc->beta = v / sc->rho;
                sc->rho = v;
            }
            break;
        case FIN_RESID:
            sc->resid = v;
            break;
        default:
            break;
    }
}

// ---------------------------------------------------------------------------------------
// CSR SpMV, one group of GS lanes per row; optional fused dot y.w (one system)
// ---------------------------------------------------------------------------------------
template <int GS, int U, typename VT, bool DOT>
__global__ __launch_bounds__(kThreads) void k_spmv(int n, const int32_t *__restrict__ rp,
                                                    const int32_t *__restrict__ ci,
                                                    const VT *__restrict__ val,
                                                    const double *__restrict__ x,
                                                    double *__restrict__ y,
                                                    const double *__restrict__ w,
                                                    double *__restrict__ partials,
                                                    PcgScalars *sc, int nxcd) {
    if (sc && sc->done) return;
    __shared__ double sh[kThreads / 64];
    const int lb = xcd_block(blockIdx.x, gridDim.x, nxcd);
    int r0, r1;
    block_range(0, n, lb, gridDim.x, r0, r1);
    const int lg = threadIdx.x % GS, grp = threadIdx.x / GS;
    constexpr int RPI = kThreads / GS;  // rows per block iteration
    double part = 0.0;
    for (int row = r0 + grp; row < r1; row += RPI) {
        const int a = rp[row], b = rp[row + 1];
        double acc = 0.0;
        for (int e0 = a + lg; e0 < b; e0 += GS * U) {
            int c[U];
            VT v[U];
            // all loads of a round are issued before any is used
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = e0 + u * GS;
                c[u] = -1;
                v[u] = VT(0);
                if (e < b) {
                    c[u] = __builtin_nontemporal_load(&ci[e]);
                    v[u] = __builtin_nontemporal_load(&val[e]);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (c[u] >= 0) acc = fma((double)v[u], x[c[u]], acc);
        }
#pragma unroll
        for (int off = GS / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, GS);
        if (lg == 0) {
            y[row] = acc;
            if (DOT) part = fma(acc, w[row], part);
        }
    }
    if (DOT) {
        const double bs = block_sum(part, sh);
        store_partials(partials, 1, &bs, lb);
    }
}

// rows [r0, r1) of SELL slice sl
__device__ __forceinline__ void sell_slice_rows(const int32_t *srow0, int n, int sl, int &r0, int &r1) {
    if (srow0) {
        r0 = srow0[sl];
        r1 = srow0[sl + 1];
    } else {
        r0 = sl * kSlice;
        r1 = min(n, r0 + kSlice);
    }
}

// The wavefront's index within its block, as a scalar: slice indices, their offsets and widths
// then stay in scalar registers and the per-lane loops over a slice run on scalar bounds
// (from the thread index the compiler would keep them in vector registers and guard every
// unrolled step with exec-mask branches).
__device__ __forceinline__ int wave_index() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// Windows (kWin consecutive slices, one per wavefront of a block) of logical block lb of nb
// over nw windows: the blocks are grouped like the XCDs of xcd_block(); each group takes a
// contiguous part of the windows and deals it to its blocks in rounds of one window each, so
// that the blocks running at once on an XCD share one narrow band of rows and of the gathered
// vector (A's product at 150^3: 1,982 -> 1,928 us against one contiguous range per block).
// With one window per block (nb = nw) block lb takes window lb.  The walk depends only on
// (nw, lb, nb, nxcd): a system's partial sums are the same alone and in a batch, and the same
// for its natural and its length-ordered layouts.
__device__ __forceinline__ void window_walk(int nw, int lb, int nb, int nxcd, int &w0, int &w1, int &step) {
    const int ng = nxcd < 1 ? 1 : (nb < nxcd ? nb : nxcd);
    const int per = nb / ng, extra = nb % ng;
    int off, cnt;
    if (lb < extra * (per + 1)) {
        off = (lb / (per + 1)) * (per + 1);
        cnt = per + 1;
    } else {
        off = extra * (per + 1) + ((lb - extra * (per + 1)) / per) * per;
        cnt = per;
    }
    w0 = (int)((int64_t)nw * off / nb) + (lb - off);
    w1 = (int)((int64_t)nw * (off + cnt) / nb);
    step = cnt;
}

// One lane's sum over `len` entries stored `stride` apart from base, continuing acc: one
// sequential fma chain in stored order.  Software pipeline: the columns and values of the
// next U entries are loaded before the gathers of the current U, so one round trip to memory
// serves both.
template <int U, int STRIDE, typename VT>
__device__ __forceinline__ double lane_chain(const int32_t *__restrict__ col, const VT *__restrict__ val,
                                             const double *__restrict__ x, int64_t base, int len, double acc) {
    int c[U];
    VT v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        c[u] = 0;
        v[u] = VT(0);
        if (u < len) {
            const int64_t d = base + (int64_t)u * STRIDE;
            c[u] = __builtin_nontemporal_load(&col[d]);
            v[u] = __builtin_nontemporal_load(&val[d]);
        }
    }
    for (int k0 = 0; k0 < len; k0 += U) {
        int cn[U];
        VT vn[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            cn[u] = 0;
            vn[u] = VT(0);
            if (k0 + U + u < len) {
                const int64_t d = base + (int64_t)(k0 + U + u) * STRIDE;
                cn[u] = __builtin_nontemporal_load(&col[d]);
                vn[u] = __builtin_nontemporal_load(&val[d]);
            }
        }
        double xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = (k0 + u < len) ? x[c[u]] : 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u < len) acc = fma((double)v[u], xv[u], acc);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            c[u] = cn[u];
            v[u] = vn[u];
        }
    }
    return acc;
}

// SELL-64 product: one wavefront per slice of 64 rows, one lane per row; entry k of the 64
// rows is one contiguous wave load.  Optional fused dot y.w.  For the tail of a split layout
// (perm/rowmap set) the launch is not tied to systems (mp, sy empty, scs may be null).  With
// rows ordered by length (lens set, instance ORD) a block takes whole windows of kWin slices,
// its wavefronts taking the slices in turn, and the sums reach their natural rows through LDS,
// so that y is written and the dot summed in row order.  The ordered instance keeps twice as many entries in flight
// (its gathers are scattered over the window's rows and wait longest).
template <int U, typename VT, bool DOT, bool ORD = false>
__global__ __launch_bounds__(kThreads) void k_sell_spmv(int n, int nslices, const uint32_t *__restrict__ sptr,
                                                         const int32_t *__restrict__ srow0,
                                                         const int32_t *__restrict__ perm,
                                                         const int32_t *__restrict__ rowmap,
                                                         const uint64_t *__restrict__ init,
                                                         const int32_t *__restrict__ col,
                                                         const VT *__restrict__ val,
                                                         const double *__restrict__ x, double *__restrict__ y,
                                                         const double *__restrict__ w,
                                                         double *__restrict__ partials, PcgScalars *scs, Map mp,
                                                         Systems sy, int nxcd, const int32_t *__restrict__ lens,
                                                         const int32_t *__restrict__ wsl,
                                                         const int32_t *__restrict__ wofs,
                                                         const uint32_t *__restrict__ tsptr,
                                                         const int32_t *__restrict__ tcol,
                                                         const VT *__restrict__ tval,
                                                         const int32_t *__restrict__ toff) {
    const Job jb = block_job(mp, nxcd);
    if (scs && scs[jb.k].done) return;
    __shared__ double sh[kThreads / 64];
    const int sb = sy.slice0 ? sy.slice0[jb.k] : 0;
    const int sn = sy.slice0 ? sy.slice0[jb.k + 1] - sb : nslices;
    static_assert(kWin == kThreads / 64, "a window holds one slice per wavefront of a block");
    // (the ordered instance keeps the thread-derived index: measured faster there)
    const int wv = ORD ? (int)(threadIdx.x >> 6) : wave_index(), lane = threadIdx.x & 63;
    double part = 0.0;
    if constexpr (ORD) {
        static_assert(kWin * kSlice % kThreads == 0, "the wavefronts of a block take a window's slices in turn");
        constexpr int UO = U >= 8 ? 16 : U;
        __shared__ double sy_win[kWin * kSlice];
        const int wa = wofs[sb], wb = wofs[sb + sn];
        int w0, w1, wstep;
        window_walk(wb - wa, jb.lb, jb.nb, nxcd, w0, w1, wstep);
        for (int wi = wa + w0; wi < wa + w1; wi += wstep) {
            const int ws = wsl[wi], we = wsl[wi + 1];
            int wr0, u0;
            sell_slice_rows(srow0, n, ws, wr0, u0);
            for (int sl = ws + wv; sl < we; sl += kThreads / 64) {
                const int64_t li = (int64_t)sl * kSlice + lane;
                const int r = perm[li];
                const int len = lens[li];
                const int64_t base = (int64_t)sptr[sl] * kSlice + lane;
                const double acc = lane_chain<UO, kSlice>(col, val, x, base, len, 0.0);
                if (r >= 0) sy_win[r - wr0] = acc;
            }
            __syncthreads();
            for (int sl = ws + wv; sl < we; sl += kThreads / 64) {
                int r0, r1;
                sell_slice_rows(srow0, n, sl, r0, r1);
                const int rn = r0 + lane;
                if (rn < r1) {
                    const double an = sy_win[rn - wr0];
                    y[rn] = an;
                    if (DOT) part = fma(an, w[rn], part);
                }
            }
            __syncthreads();
        }
        if (DOT) {
            const double bs = block_sum(part, sh);
            store_partials(partials, 1, &bs, jb.gb);
        }
        return;
    }
    int w0, w1, wstep;
    window_walk((sn + kWin - 1) / kWin, jb.lb, jb.nb, nxcd, w0, w1, wstep);
    for (int wi = w0; wi < w1; wi += wstep) {
        const int sl = sb + wi * kWin + wv;
        if (sl >= sb + sn) break;
        int r0, r1;
        sell_slice_rows(srow0, n, sl, r0, r1);
        int r = r0 + lane;
        if (perm) r = perm[sl * kSlice + lane];
        const bool valid = r >= 0 && r < (perm ? n : r1);
        const int ro = (valid && rowmap) ? rowmap[r] : r;
        const uint32_t c0 = sptr[sl];
        const int width = (int)(sptr[sl + 1] - c0);
        const int64_t base = (int64_t)c0 * kSlice + lane;
        // rows split between the two layouts start with their leading entries: run here from the
        // tail layout (tcol set; the slice's split rows are consecutive tail rows), or continue
        // the sum a separate tail product left in y
        double acc = 0.0;
        if (init && valid && ((init[sl] >> lane) & 1)) {
            if (tcol) {
                const int t = toff[sl] + __popcll(init[sl] & ((1ull << lane) - 1ull));
                const uint32_t tc0 = tsptr[t >> 6];
                const int tw = (int)(tsptr[(t >> 6) + 1] - tc0);
                const int64_t tb = (int64_t)tc0 * kSlice + (t & 63);
                for (int k = 0; k < tw; ++k) {
                    const int64_t d = tb + (int64_t)k * kSlice;
                    acc = fma((double)tval[d], x[tcol[d]], acc);
                }
            } else {
                acc = y[ro];
            }
        }
        acc = lane_chain<U, kSlice>(col, val, x, base, width, acc);
        if (valid) {
            y[ro] = acc;
            if (DOT) part = fma(acc, w[ro], part);
        }
    }
    if (DOT) {
        const double bs = block_sum(part, sh);
        store_partials(partials, 1, &bs, jb.gb);
    }
}

// One lane's sum over `nr` runs of three consecutive columns (the layout with one column
// index per run): the values of run j are entries 3j..3j+2 of the lane, stored kSlice apart
// from vbase, its first column at rbase + j * kSlice.  The same sequential fma chain over the
// entries in stored order as lane_chain, with UR runs (3 UR entries) in flight.
template <int UR, typename VT>
__device__ __forceinline__ double run_chain(const int32_t *__restrict__ col3, const VT *__restrict__ val,
                                            const double *__restrict__ x, int64_t rbase, int64_t vbase, int nr,
                                            double acc) {
    int c[UR];
    VT v[UR][3];
#pragma unroll
    for (int u = 0; u < UR; ++u) {
        c[u] = 0;
#pragma unroll
        for (int e = 0; e < 3; ++e) v[u][e] = VT(0);
        if (u < nr) {
            c[u] = __builtin_nontemporal_load(&col3[rbase + (int64_t)u * kSlice]);
#pragma unroll
            for (int e = 0; e < 3; ++e) v[u][e] = __builtin_nontemporal_load(&val[vbase + (int64_t)(3 * u + e) * kSlice]);
        }
    }
    for (int j0 = 0; j0 < nr; j0 += UR) {
        int cn[UR];
        VT vn[UR][3];
#pragma unroll
        for (int u = 0; u < UR; ++u) {
            cn[u] = 0;
#pragma unroll
            for (int e = 0; e < 3; ++e) vn[u][e] = VT(0);
            if (j0 + UR + u < nr) {
                const int j = j0 + UR + u;
                cn[u] = __builtin_nontemporal_load(&col3[rbase + (int64_t)j * kSlice]);
#pragma unroll
                for (int e = 0; e < 3; ++e)
                    vn[u][e] = __builtin_nontemporal_load(&val[vbase + (int64_t)(3 * j + e) * kSlice]);
            }
        }
        double xv[UR][3];
#pragma unroll
        for (int u = 0; u < UR; ++u)
#pragma unroll
            for (int e = 0; e < 3; ++e) xv[u][e] = (j0 + u < nr) ? x[c[u] + e] : 0.0;
#pragma unroll
        for (int u = 0; u < UR; ++u)
            if (j0 + u < nr) {
#pragma unroll
                for (int e = 0; e < 3; ++e) acc = fma((double)v[u][e], xv[u][e], acc);
            }
#pragma unroll
        for (int u = 0; u < UR; ++u) {
            c[u] = cn[u];
#pragma unroll
            for (int e = 0; e < 3; ++e) v[u][e] = vn[u][e];
        }
    }
    return acc;
}

// SELL-64 product over the layout with one column index per run of three (plain layouts
// only: natural row order, no split): the walk, row sums, stores and fused dot of k_sell_spmv,
// so products and dots are identical to it bit for bit.
template <int UR, typename VT, bool DOT>
__global__ __launch_bounds__(kThreads) void k_sell_spmv_runs(int n, const uint32_t *__restrict__ sptr,
                                                             const int32_t *__restrict__ srow0,
                                                             const int32_t *__restrict__ col3,
                                                             const VT *__restrict__ val,
                                                             const double *__restrict__ x, double *__restrict__ y,
                                                             const double *__restrict__ w,
                                                             double *__restrict__ partials, PcgScalars *scs, Map mp,
                                                             Systems sy, int nslices, int nxcd) {
    const Job jb = block_job(mp, nxcd);
    if (scs && scs[jb.k].done) return;
    __shared__ double sh[kThreads / 64];
    const int sb = sy.slice0 ? sy.slice0[jb.k] : 0;
    const int sn = sy.slice0 ? sy.slice0[jb.k + 1] - sb : nslices;
    const int wv = wave_index(), lane = threadIdx.x & 63;
    double part = 0.0;
    int w0, w1, wstep;
    window_walk((sn + kWin - 1) / kWin, jb.lb, jb.nb, nxcd, w0, w1, wstep);
    for (int wi = w0; wi < w1; wi += wstep) {
        const int sl = sb + wi * kWin + wv;
        if (sl >= sb + sn) break;
        int r0, r1;
        sell_slice_rows(srow0, n, sl, r0, r1);
        const int r = r0 + lane;
        const uint32_t c0 = sptr[sl];
        const int nr = (int)(sptr[sl + 1] - c0) / 3;
        const double acc = run_chain<UR, VT>(col3, val, x, (int64_t)(c0 / 3u) * kSlice + lane,
                                             (int64_t)c0 * kSlice + lane, nr, 0.0);
        if (r < r1) {
            y[r] = acc;
            if (DOT) part = fma(acc, w[r], part);
        }
    }
    if (DOT) {
        const double bs = block_sum(part, sh);
        store_partials(partials, 1, &bs, jb.gb);
    }
}

// Fused PCG products (SELL-64, one lane per row, layouts without a tail).  The vector being
// multiplied is formed on the fly from two others with the same fma the separate update
// kernel would use, so the result is identical to update-then-multiply; the owner lane of
// each row also stores the updated entry.
//   FUSE_AP:  p_new = z + beta p_old (p_new = z on the first iteration); q = A p_new;
//             partial sums of p_new.q
//   FUSE_GR:  r_new = r_old - alpha q; x += alpha p_new; t = G r_new; partial sums of r_new.r_new
enum : int { FUSE_AP = 1, FUSE_GR = 2 };

template <int U, typename VT, int MODE>
__global__ __launch_bounds__(kThreads) void k_sell_fused(int n, int nslices, const uint32_t *__restrict__ sptr,
                                                          const int32_t *__restrict__ srow0,
                                                          const int32_t *__restrict__ col,
                                                          const VT *__restrict__ val,
                                                          const double *__restrict__ va,   // z | r_old
                                                          const double *__restrict__ vb,   // p_old | q
                                                          double *__restrict__ own_out,    // p_new | r_new
                                                          double *__restrict__ x,          // - | x
                                                          const double *__restrict__ pn,   // - | p_new
                                                          double *__restrict__ y,          // q | t
                                                          double *__restrict__ partials,
                                                          const PcgScalars *scs, int first, Map mp, Systems sy,
                                                          int nxcd) {
    const Job jb = block_job(mp, nxcd);
    const PcgScalars *sc = scs + jb.k;
    if (sc->done) return;
    __shared__ double sh[kThreads / 64];
    const double alpha = sc->alpha;
    const double coef = (MODE == FUSE_AP) ? sc->beta : -alpha;
    const int sb = sy.slice0 ? sy.slice0[jb.k] : 0;
    const int sn = sy.slice0 ? sy.slice0[jb.k + 1] - sb : nslices;
    const int wv = wave_index(), lane = threadIdx.x & 63;
    int w0, w1, wstep;
    window_walk((sn + kWin - 1) / kWin, jb.lb, jb.nb, nxcd, w0, w1, wstep);
    double part = 0.0;
    for (int wi = w0; wi < w1; wi += wstep) {
        const int sl = sb + wi * kWin + wv;
        if (sl >= sb + sn) break;
        int r0, r1;
        sell_slice_rows(srow0, n, sl, r0, r1);
        const int r = r0 + lane;
        const uint32_t c0 = sptr[sl];
        const int width = (int)(sptr[sl + 1] - c0);
        const int64_t base = (int64_t)c0 * kSlice + lane;
        double acc = 0.0;
        // software pipeline as in lane_chain: the next U columns and values are loaded before
        // the current gathers
        int c[U];
        VT v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            c[u] = 0;
            v[u] = VT(0);
            if (u < width) {
                const int64_t d = base + (int64_t)u * kSlice;
                c[u] = __builtin_nontemporal_load(&col[d]);
                v[u] = __builtin_nontemporal_load(&val[d]);
            }
        }
        for (int k0 = 0; k0 < width; k0 += U) {
            int cn[U];
            VT vn[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                cn[u] = 0;
                vn[u] = VT(0);
                if (k0 + U + u < width) {
                    const int64_t d = base + (int64_t)(k0 + U + u) * kSlice;
                    cn[u] = __builtin_nontemporal_load(&col[d]);
                    vn[u] = __builtin_nontemporal_load(&val[d]);
                }
            }
            double xa[U], xb[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool in = k0 + u < width;
                xa[u] = in ? va[c[u]] : 0.0;
                xb[u] = (in && !(MODE == FUSE_AP && first)) ? vb[c[u]] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (k0 + u < width) {
                    const double xv = (MODE == FUSE_AP && first) ? xa[u] : fma(coef, xb[u], xa[u]);
                    acc = fma((double)v[u], xv, acc);
                }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                c[u] = cn[u];
                v[u] = vn[u];
            }
        }
        if (r < r1) {
            const double own = (MODE == FUSE_AP && first) ? va[r] : fma(coef, vb[r], va[r]);
            own_out[r] = own;
            y[r] = acc;
            if (MODE == FUSE_AP) {
                part = fma(own, acc, part);
            } else {
                x[r] = fma(alpha, pn[r], x[r]);
                part = fma(own, own, part);
            }
        }
    }
    const double bs = block_sum(part, sh);
    store_partials(partials, 1, &bs, jb.gb);
}

// r = b - q ; partials of b.b and r.r ; finalisation checks ||b|| = 0 and ||r0|| <= tol
__global__ __launch_bounds__(kThreads) void k_init_residual(int n, const double *__restrict__ b,
                                                             const double *__restrict__ q,
                                                             double *__restrict__ r,
                                                             double *__restrict__ partials, Map mp, Systems sy,
                                                             int nxcd) {
    __shared__ double sh[kThreads / 64];
    const Job jb = block_job(mp, nxcd);
    int a0, a1, i0, i1;
    sys_rows(sy, n, jb.k, a0, a1);
    block_range(a0, a1 - a0, jb.lb, jb.nb, i0, i1);
    double pb = 0.0, pr = 0.0;
    for (int i = i0 + threadIdx.x; i < i1; i += kThreads) {
        const double bi = b[i], ri = bi - q[i];
        r[i] = ri;
        pb = fma(bi, bi, pb);
        pr = fma(ri, ri, pr);
    }
    double mine[2];
    mine[0] = block_sum(pb, sh);
    mine[1] = block_sum(pr, sh);
    store_partials(partials, 2, mine, jb.gb);
}

// x += alpha p ; r -= alpha q ; ||r||^2 ; convergence test; (plain CG) beta = rr'/rr
__global__ __launch_bounds__(kThreads) void k_update_xr(int n, double *__restrict__ x,
                                                         double *__restrict__ r,
                                                         const double *__restrict__ p,
                                                         const double *__restrict__ q,
                                                         double *__restrict__ partials,
                                                         PcgScalars *scs, Map mp, Systems sy, int nxcd) {
    const Job jb = block_job(mp, nxcd);
    const PcgScalars *sc = scs + jb.k;
    if (sc->done) return;
    __shared__ double sh[kThreads / 64];
    const double alpha = sc->alpha;
    int a0, a1, i0, i1;
    sys_rows(sy, n, jb.k, a0, a1);
    block_range(a0, a1 - a0, jb.lb, jb.nb, i0, i1);
    double pr = 0.0;
    for (int i = i0 + threadIdx.x; i < i1; i += kThreads) {
        x[i] = fma(alpha, p[i], x[i]);
        const double ri = fma(-alpha, q[i], r[i]);
        r[i] = ri;
        pr = fma(ri, ri, pr);
    }
    const double bs = block_sum(pr, sh);
    store_partials(partials, 1, &bs, jb.gb);
}

// p = z + beta p   (first = 1: p = z)
__global__ __launch_bounds__(kThreads) void k_update_p(int n, double *__restrict__ p,
                                                        const double *__restrict__ z,
                                                        const PcgScalars *scs, int first, Map mp, Systems sy,
                                                        int nxcd) {
    const Job jb = block_job(mp, nxcd);
    const PcgScalars *sc = scs + jb.k;
    if (sc->done) return;
    const double beta = first ? 0.0 : sc->beta;
    int a0, a1, i0, i1;
    sys_rows(sy, n, jb.k, a0, a1);
    block_range(a0, a1 - a0, jb.lb, jb.nb, i0, i1);
    if (first)
        for (int i = i0 + threadIdx.x; i < i1; i += kThreads) p[i] = z[i];
    else
        for (int i = i0 + threadIdx.x; i < i1; i += kThreads) p[i] = fma(beta, p[i], z[i]);
}

// x = 0 for the systems whose right-hand side is zero
__global__ __launch_bounds__(kThreads) void k_zero_rhs(int n, double *__restrict__ x, const PcgScalars *scs, Map mp,
                                                       Systems sy, int nxcd) {
    const Job jb = block_job(mp, nxcd);
    if (scs[jb.k].done != DONE_ZERO_RHS) return;
    int a0, a1, i0, i1;
    sys_rows(sy, n, jb.k, a0, a1);
    block_range(a0, a1 - a0, jb.lb, jb.nb, i0, i1);
    for (int i = i0 + threadIdx.x; i < i1; i += kThreads) x[i] = 0.0;
}

// Copies the scalars of every system into pinned host memory (mapped), where the host reads
// them once the chunk's event has completed; a kernel is cheaper here than a copy engine
// transfer of a few hundred bytes.
__global__ void k_publish(const PcgScalars *__restrict__ sc, int nwords, PcgScalars *__restrict__ host) {
    const double *src = reinterpret_cast<const double *>(sc);
    double *dst = reinterpret_cast<double *>(host);
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nwords; k += gridDim.x * blockDim.x) dst[k] = src[k];
}

__global__ void k_set_scalars(PcgScalars *scs, int nsys, double rtol, int maxit, int plain) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nsys; k += gridDim.x * blockDim.x) {
        PcgScalars s{};
        s.rtol = rtol;
        s.maxit = maxit;
        s.plain = plain;
        scs[k] = s;
    }
}

// true residual partials: ||b - Ax||^2 with q = A x
__global__ __launch_bounds__(kThreads) void k_resid_norm(int n, const double *__restrict__ b,
                                                          const double *__restrict__ q,
                                                          double *__restrict__ partials, Map mp, Systems sy,
                                                          int nxcd) {
    __shared__ double sh[kThreads / 64];
    const Job jb = block_job(mp, nxcd);
    int a0, a1, i0, i1;
    sys_rows(sy, n, jb.k, a0, a1);
    block_range(a0, a1 - a0, jb.lb, jb.nb, i0, i1);
    double pr = 0.0;
    for (int i = i0 + threadIdx.x; i < i1; i += kThreads) {
        const double d = b[i] - q[i];
        pr = fma(d, d, pr);
    }
    const double bs = block_sum(pr, sh);
    store_partials(partials, 1, &bs, jb.gb);
}

// ---------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------
// Lanes per row (the paper's miniwarp, Sec. 3) and independent loads per lane per round, from
// the average row length: about four entries per lane per round and at most 8 loads in flight
// per lane.
static void spmv_shape(double avg_nnz, int *gs, int *un) {
    int g = 4;
    while (g < 64 && g * 4 < avg_nnz) g <<= 1;
    int u = 1;
    while (u < 8 && g * u < avg_nnz) u <<= 1;
    if (option(AFSAI_OPT_SPMV_GROUP) > 0) g = (int)option(AFSAI_OPT_SPMV_GROUP);
    if (option(AFSAI_OPT_SPMV_UNROLL) > 0) u = (int)option(AFSAI_OPT_SPMV_UNROLL);
    *gs = g;
    *un = u;
}

static int blocks_for_rows(int n, int gs, const DeviceInfo &di) {
    const int64_t rows_per_iter = kThreads / gs;
    int64_t want = (n + rows_per_iter - 1) / rows_per_iter;
    int64_t cap = (int64_t)di.num_cus * 8;
    int64_t b = want < cap ? want : cap;
    return (int)(b < 1 ? 1 : b);
}

static int blocks_for_vec(int n, const DeviceInfo &di) {
    int64_t want = ((int64_t)n + kThreads * 4 - 1) / (kThreads * 4);
    int64_t cap = (int64_t)di.num_cus * 8;
    int64_t b = want < cap ? want : cap;
    return (int)(b < 1 ? 1 : b);
}

static int blocks_for_slices(int nslices, const DeviceInfo &di) {
    int64_t nb = ((int64_t)nslices + kThreads / 64 - 1) / (kThreads / 64);
    const int64_t cap = (int64_t)di.num_cus * 16;
    if (nb > cap) nb = cap;
    if (nb < 1) nb = 1;
    return (int)nb;
}

struct Csr {
    int n = 0;
    int64_t nnz = 0;
    const int32_t *rp = nullptr, *ci = nullptr;
    const void *val = nullptr;
    bool f32 = false;
};

template <int GS, int U, typename VT>
static void launch_spmv_t(const Csr &A, const double *x, double *y, const double *w, double *partials,
                          PcgScalars *sc, int nb, int nxcd, hipStream_t s) {
    if (w)
        hipLaunchKernelGGL((k_spmv<GS, U, VT, true>), dim3(nb), dim3(kThreads), 0, s, A.n, A.rp, A.ci,
                           (const VT *)A.val, x, y, w, partials, sc, nxcd);
    else
        hipLaunchKernelGGL((k_spmv<GS, U, VT, false>), dim3(nb), dim3(kThreads), 0, s, A.n, A.rp, A.ci,
                           (const VT *)A.val, x, y, w, partials, sc, nxcd);
}

template <int GS, typename VT>
static void launch_spmv_u(const Csr &A, int un, const double *x, double *y, const double *w, double *partials,
                          PcgScalars *sc, int nb, int nxcd, hipStream_t s) {
    switch (un) {
        case 1: launch_spmv_t<GS, 1, VT>(A, x, y, w, partials, sc, nb, nxcd, s); break;
        case 2: launch_spmv_t<GS, 2, VT>(A, x, y, w, partials, sc, nb, nxcd, s); break;
        case 4: launch_spmv_t<GS, 4, VT>(A, x, y, w, partials, sc, nb, nxcd, s); break;
        default: launch_spmv_t<GS, 8, VT>(A, x, y, w, partials, sc, nb, nxcd, s); break;
    }
}

template <typename VT>
static void launch_spmv_v(const Csr &A, int gs, int un, const double *x, double *y, const double *w,
                          double *partials, PcgScalars *sc, int nb, int nxcd, hipStream_t s) {
    switch (gs) {
        case 4: launch_spmv_u<4, VT>(A, un, x, y, w, partials, sc, nb, nxcd, s); break;
        case 8: launch_spmv_u<8, VT>(A, un, x, y, w, partials, sc, nb, nxcd, s); break;
        case 16: launch_spmv_u<16, VT>(A, un, x, y, w, partials, sc, nb, nxcd, s); break;
        case 32: launch_spmv_u<32, VT>(A, un, x, y, w, partials, sc, nb, nxcd, s); break;
        default: launch_spmv_u<64, VT>(A, un, x, y, w, partials, sc, nb, nxcd, s); break;
    }
}

// y = A x, CSR (one system; optionally fused dot y.w finalised into sc)
static void spmv(const char *name, const Csr &A, const double *x, double *y, const double *w,
                 double *partials, PcgScalars *sc, int fin, const DeviceInfo &di, hipStream_t s) {
    const double avg = A.n ? (double)A.nnz / A.n : 0.0;
    int gs, un;
    spmv_shape(avg, &gs, &un);
    const int nb = blocks_for_rows(A.n, gs, di);
    {
        ProfScope ps(name, s);
        if (A.f32)
            launch_spmv_v<float>(A, gs, un, x, y, w, partials, sc, nb, di.num_xcds, s);
        else
            launch_spmv_v<double>(A, gs, un, x, y, w, partials, sc, nb, di.num_xcds, s);
    }
    if (w) hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, s, partials, nb, Map(), fin, sc);
}

// Block maps of a batch for the three launch shapes (SELL products, vector kernels), held on
// the device for one solve; empty for a single system.
struct Shape {
    Map mp;
    int nblocks = 0;
};
struct BatchMaps {
    int nsys = 1;
    Systems sy;
    Shape sell, vec;
    DevBuf buf;
};

static int make_batch_maps(int n, int nsys, const int32_t *row0, const DeviceInfo &di, hipStream_t s,
                           BatchMaps *bm) {
    bm->nsys = nsys;
    std::vector<int32_t> slice0(nsys + 1);
    Segments seg;
    seg.nsys = nsys;
    seg.row0 = row0;
    segment_slices(seg, n, slice0.data());
    if (nsys == 1) {
        bm->sell.nblocks = blocks_for_slices(slice0[1], di);
        bm->vec.nblocks = blocks_for_vec(n, di);
        return AFSAI_OK;
    }
    std::vector<int32_t> nb_sell(nsys), nb_vec(nsys);
    int64_t tot_sell = 0, tot_vec = 0;
    for (int k = 0; k < nsys; ++k) {
        nb_sell[k] = blocks_for_slices(slice0[k + 1] - slice0[k], di);
        nb_vec[k] = blocks_for_vec(row0[k + 1] - row0[k], di);
        tot_sell += nb_sell[k];
        tot_vec += nb_vec[k];
    }
    if (tot_sell >= (1 << 30) || tot_vec >= (1 << 30)) AFSAI_FAIL(AFSAI_ERR_TOO_LARGE, "batch: too many blocks");
    // layout: row0 | slice0 | sell: blk_sys, b0, nb | vec: blk_sys, b0, nb
    std::vector<int32_t> h;
    h.reserve((size_t)2 * (nsys + 1) + tot_sell + tot_vec + 4 * (size_t)nsys);
    h.insert(h.end(), row0, row0 + nsys + 1);
    h.insert(h.end(), slice0.begin(), slice0.end());
    size_t off_sell = h.size();
    for (int k = 0; k < nsys; ++k) h.insert(h.end(), nb_sell[k], k);
    size_t off_sell_b0 = h.size();
    int32_t acc = 0;
    for (int k = 0; k < nsys; ++k) {
        h.push_back(acc);
        acc += nb_sell[k];
    }
    size_t off_sell_nb = h.size();
    h.insert(h.end(), nb_sell.begin(), nb_sell.end());
    size_t off_vec = h.size();
    for (int k = 0; k < nsys; ++k) h.insert(h.end(), nb_vec[k], k);
    size_t off_vec_b0 = h.size();
    acc = 0;
    for (int k = 0; k < nsys; ++k) {
        h.push_back(acc);
        acc += nb_vec[k];
    }
    size_t off_vec_nb = h.size();
    h.insert(h.end(), nb_vec.begin(), nb_vec.end());
    int rc;
    if ((rc = dalloc(bm->buf, sizeof(int32_t) * h.size(), s))) return rc;
    AFSAI_HIP_TRY(hipMemcpyAsync(bm->buf.p, h.data(), sizeof(int32_t) * h.size(), hipMemcpyHostToDevice, s));
    AFSAI_HIP_TRY(hipStreamSynchronize(s));
    const int32_t *d = bm->buf.as<int32_t>();
    bm->sy.row0 = d;
    bm->sy.slice0 = d + nsys + 1;
    bm->sell.mp = Map{d + off_sell, d + off_sell_b0, d + off_sell_nb};
    bm->sell.nblocks = (int)tot_sell;
    bm->vec.mp = Map{d + off_vec, d + off_vec_b0, d + off_vec_nb};
    bm->vec.nblocks = (int)tot_vec;
    return AFSAI_OK;
}

// fused: a split layout's tail runs inside the slices' product (else the caller launched it)
template <int U, typename VT>
static void launch_sell_t(const Sell &S, const double *x, double *y, const double *w, double *partials,
                          PcgScalars *scs, const Map &mp, const Systems &sy, int nb, int nxcd, hipStream_t s,
                          bool fused) {
    const Sell *T = fused ? S.tail : nullptr;
    const uint32_t *tsp = T ? T->sptr : nullptr;
    const int32_t *tcl = T ? T->col : nullptr;
    const VT *tvl = T ? (const VT *)T->val : nullptr;
    const int32_t *tof = T ? S.toff : nullptr;
    if (S.col3) {
        // runs of three: about as many entries in flight as U
        constexpr int UR = U >= 8 ? 3 : 1;
        if (w)
            hipLaunchKernelGGL((k_sell_spmv_runs<UR, VT, true>), dim3(nb), dim3(kThreads), 0, s, S.n, S.sptr,
                               S.srow0, S.col3, (const VT *)S.val, x, y, w, partials, scs, mp, sy, S.nslices, nxcd);
        else
            hipLaunchKernelGGL((k_sell_spmv_runs<UR, VT, false>), dim3(nb), dim3(kThreads), 0, s, S.n, S.sptr,
                               S.srow0, S.col3, (const VT *)S.val, x, y, w, partials, scs, mp, sy, S.nslices, nxcd);
        return;
    }
    if (S.lens) {
        if (w)
            hipLaunchKernelGGL((k_sell_spmv<U, VT, true, true>), dim3(nb), dim3(kThreads), 0, s, S.n, S.nslices,
                               S.sptr, S.srow0, S.perm, S.rowmap, S.init, S.col, (const VT *)S.val, x, y, w, partials,
                               scs, mp, sy, nxcd, S.lens, S.wsl, S.wofs, tsp, tcl, tvl, tof);
        else
            hipLaunchKernelGGL((k_sell_spmv<U, VT, false, true>), dim3(nb), dim3(kThreads), 0, s, S.n, S.nslices,
                               S.sptr, S.srow0, S.perm, S.rowmap, S.init, S.col, (const VT *)S.val, x, y, w, partials,
                               scs, mp, sy, nxcd, S.lens, S.wsl, S.wofs, tsp, tcl, tvl, tof);
        return;
    }
    if (w)
        hipLaunchKernelGGL((k_sell_spmv<U, VT, true>), dim3(nb), dim3(kThreads), 0, s, S.n, S.nslices, S.sptr,
                           S.srow0, S.perm, S.rowmap, S.init, S.col, (const VT *)S.val, x, y, w, partials, scs, mp,
                           sy, nxcd, S.lens, S.wsl, S.wofs, tsp, tcl, tvl, tof);
    else
        hipLaunchKernelGGL((k_sell_spmv<U, VT, false>), dim3(nb), dim3(kThreads), 0, s, S.n, S.nslices, S.sptr,
                           S.srow0, S.perm, S.rowmap, S.init, S.col, (const VT *)S.val, x, y, w, partials, scs, mp,
                           sy, nxcd, S.lens, S.wsl, S.wofs, tsp, tcl, tvl, tof);
}

template <typename VT>
static void launch_sell_v(const Sell &S, int un, const double *x, double *y, const double *w, double *partials,
                          PcgScalars *scs, const Map &mp, const Systems &sy, int nb, int nxcd, hipStream_t s,
                          bool fused = false) {
    switch (un) {
        case 1: launch_sell_t<1, VT>(S, x, y, w, partials, scs, mp, sy, nb, nxcd, s, fused); break;
        case 2: launch_sell_t<2, VT>(S, x, y, w, partials, scs, mp, sy, nb, nxcd, s, fused); break;
        case 4: launch_sell_t<4, VT>(S, x, y, w, partials, scs, mp, sy, nb, nxcd, s, fused); break;
        default: launch_sell_t<8, VT>(S, x, y, w, partials, scs, mp, sy, nb, nxcd, s, fused); break;
    }
}

// Entries in flight per lane of a SELL product: 8 (16 in the length-ordered instance), or 4
// for matrices of at most 8 stored entries per row on average, whose lanes finish within one
// or two rounds anyway and gain more from the resident wavefronts the smaller register budget
// allows (a batch of short 7-point systems: its PCG 27.9 -> 25.0 ms).  The sums do not depend
// on it.
static int sell_unroll(const Sell &S) {
    if (option(AFSAI_OPT_SPMV_UNROLL) > 0) return (int)option(AFSAI_OPT_SPMV_UNROLL);
    return (S.n > 0 && S.entries <= 8 * (int64_t)S.n) ? 4 : 8;
}

// y = S x for a SELL-64 matrix laid out for the batch (optionally fused dot y.w finalised into
// the systems' scalars); a split layout's tail is multiplied first
static void sell_spmv(const char *name, const Sell &S, const BatchMaps &bm, const double *x, double *y,
                      const double *w, double *partials, PcgScalars *scs, int fin, const DeviceInfo &di,
                      hipStream_t s) {
    const int un = sell_unroll(S);
    // a split layout's tail runs in a launch of its own first; inside the slices' product when
    // asked for (measured slower: the lanes of long rows serialise their tails while the rest of
    // the wavefront waits)
    const bool fused = S.tail && S.toff && option(AFSAI_OPT_SELL_TAIL) == 1;
    if (S.tail && !fused) {
        const Sell &T = *S.tail;
        const int nbt = blocks_for_slices(T.nslices, di);
        // the tail's rows belong to any system: with one system it stops with it
        PcgScalars *tsc = (bm.nsys == 1) ? scs : nullptr;
        ProfScope ps("sell_tail", s);
        if (T.f32)
            launch_sell_v<float>(T, sell_unroll(T), x, y, nullptr, nullptr, tsc, Map(), Systems(), nbt, di.num_xcds, s);
        else
            launch_sell_v<double>(T, sell_unroll(T), x, y, nullptr, nullptr, tsc, Map(), Systems(), nbt, di.num_xcds,
                                  s);
    }
    const int nb = bm.sell.nblocks;
    {
        ProfScope ps(name, s);
        if (S.f32)
            launch_sell_v<float>(S, un, x, y, w, partials, scs, bm.sell.mp, bm.sy, nb, di.num_xcds, s, fused);
        else
            launch_sell_v<double>(S, un, x, y, w, partials, scs, bm.sell.mp, bm.sy, nb, di.num_xcds, s, fused);
    }
    if (w)
        hipLaunchKernelGGL(k_finalize, dim3(bm.nsys), dim3(kThreads), 0, s, partials, nb, bm.sell.mp, fin, scs);
}

template <int U, typename VT, int MODE>
static void launch_fused_t(const Sell &S, const double *va, const double *vb, double *own, double *x,
                           const double *pn, double *y, double *partials, PcgScalars *scs, int first,
                           const BatchMaps &bm, int nxcd, hipStream_t s) {
    hipLaunchKernelGGL((k_sell_fused<U, VT, MODE>), dim3(bm.sell.nblocks), dim3(kThreads), 0, s, S.n, S.nslices,
                       S.sptr, S.srow0, S.col, (const VT *)S.val, va, vb, own, x, pn, y, partials, scs, first,
                       bm.sell.mp, bm.sy, nxcd);
}

template <typename VT, int MODE>
static void launch_fused_v(const Sell &S, int un, const double *va, const double *vb, double *own, double *x,
                           const double *pn, double *y, double *partials, PcgScalars *scs, int first,
                           const BatchMaps &bm, int nxcd, hipStream_t s) {
    switch (un) {
        case 1: launch_fused_t<1, VT, MODE>(S, va, vb, own, x, pn, y, partials, scs, first, bm, nxcd, s); break;
        case 2: launch_fused_t<2, VT, MODE>(S, va, vb, own, x, pn, y, partials, scs, first, bm, nxcd, s); break;
        case 4: launch_fused_t<4, VT, MODE>(S, va, vb, own, x, pn, y, partials, scs, first, bm, nxcd, s); break;
        default: launch_fused_t<8, VT, MODE>(S, va, vb, own, x, pn, y, partials, scs, first, bm, nxcd, s); break;
    }
}

// fused product followed by the finalisation of its dot
template <int MODE>
static void sell_fused(const char *name, const Sell &S, const BatchMaps &bm, const double *va, const double *vb,
                       double *own, double *x, const double *pn, double *y, double *partials, PcgScalars *scs,
                       int first, int fin, const DeviceInfo &di, hipStream_t s) {
    const int un = sell_unroll(S);
    {
        ProfScope ps(name, s);
        if (S.f32)
            launch_fused_v<float, MODE>(S, un, va, vb, own, x, pn, y, partials, scs, first, bm, di.num_xcds, s);
        else
            launch_fused_v<double, MODE>(S, un, va, vb, own, x, pn, y, partials, scs, first, bm, di.num_xcds, s);
    }
    hipLaunchKernelGGL(k_finalize, dim3(bm.nsys), dim3(kThreads), 0, s, partials, bm.sell.nblocks, bm.sell.mp, fin,
                       scs);
}

// Y = A X for K vectors stored row by row (entry (i, j) at i * K + j): one wavefront per
// SELL-64 slice, one lane per row; every matrix entry is read once for the K vectors and the
// K values of a gathered row are contiguous.  Each output is the same sequential chain over
// the row's entries as in the single-vector product.
template <int K, typename VT, bool DOT = false>
__global__ __launch_bounds__(kThreads) void k_sell_spmm(int n, int nslices, const uint32_t *__restrict__ sptr,
                                                         const int32_t *__restrict__ perm,
                                                         const int32_t *__restrict__ lens,
                                                         const int32_t *__restrict__ col,
                                                         const VT *__restrict__ val, const double *__restrict__ x,
                                                         double *__restrict__ y, int nxcd,
                                                         const double *__restrict__ w = nullptr,
                                                         double *__restrict__ partials = nullptr) {
    constexpr int U = K <= 2 ? 8 : 4;  // entries in flight per lane (fewer for wide blocks: registers)
    __shared__ double sh[kThreads / 64];
    double part[K];
#pragma unroll
    for (int j = 0; j < K; ++j) part[j] = 0.0;
    const int lb = xcd_block(blockIdx.x, gridDim.x, nxcd);
    const int wv = wave_index(), lane = threadIdx.x & 63;
    int w0, w1, wstep;
    window_walk((nslices + kWin - 1) / kWin, lb, gridDim.x, nxcd, w0, w1, wstep);
    for (int wi = w0; wi < w1; wi += wstep) {
        const int sl = wi * kWin + wv;
        if (sl >= nslices) break;
        const uint32_t c0 = sptr[sl];
        int r = sl * kSlice + lane;
        bool valid = r < n;
        int len = (int)(sptr[sl + 1] - c0);
        if (lens) {
            r = perm[(int64_t)sl * kSlice + lane];
            len = lens[(int64_t)sl * kSlice + lane];
            valid = r >= 0;
        }
        const int64_t base = (int64_t)c0 * kSlice + lane;
        double acc[K];
#pragma unroll
        for (int j = 0; j < K; ++j) acc[j] = 0.0;
        // software pipeline as in lane_chain: the next U columns and values are loaded before
        // the current gathers
        int c[U];
        VT v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            c[u] = 0;
            v[u] = VT(0);
            if (u < len) {
                const int64_t d = base + (int64_t)u * kSlice;
                c[u] = __builtin_nontemporal_load(&col[d]);
                v[u] = __builtin_nontemporal_load(&val[d]);
            }
        }
        for (int k0 = 0; k0 < len; k0 += U) {
            int cn[U];
            VT vn[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                cn[u] = 0;
                vn[u] = VT(0);
                if (k0 + U + u < len) {
                    const int64_t d = base + (int64_t)(k0 + U + u) * kSlice;
                    cn[u] = __builtin_nontemporal_load(&col[d]);
                    vn[u] = __builtin_nontemporal_load(&val[d]);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (k0 + u < len) {
                    const double *xc = x + (int64_t)c[u] * K;
#pragma unroll
                    for (int j = 0; j < K; ++j) acc[j] = fma((double)v[u], xc[j], acc[j]);
                }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                c[u] = cn[u];
                v[u] = vn[u];
            }
        }
        if (valid) {
#pragma unroll
            for (int j = 0; j < K; ++j) {
                y[(int64_t)r * K + j] = acc[j];
                if (DOT) part[j] = fma(acc[j], w[(int64_t)r * K + j], part[j]);
            }
        }
    }
    if (DOT) {
        // per column j: this block's partial sum at partials[j * gridDim.x + lb]
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const double bs = block_sum(part[j], sh);
            if (threadIdx.x == 0) partials[(size_t)j * gridDim.x + lb] = bs;
        }
    }
}

// Block product over the layout with one column index per run of three (plain layouts: no
// length ordering): a lane reads a run's index and its three values and the 3K consecutive
// entries of X's rows c..c+2; per column the sum is the same chain over the entries in stored
// order as k_sell_spmm's, so Y and the partial sums are identical to it bit for bit.
template <int K, bool DOT = false>
__global__ __launch_bounds__(kThreads) void k_sell_spmm_runs(int n, int nslices, const uint32_t *__restrict__ sptr,
                                                              const int32_t *__restrict__ col3,
                                                              const double *__restrict__ val,
                                                              const double *__restrict__ x, double *__restrict__ y,
                                                              int nxcd, const double *__restrict__ w = nullptr,
                                                              double *__restrict__ partials = nullptr) {
    constexpr int UR = K <= 2 ? 3 : 1;  // runs in flight per lane (9 or 3 entries)
    __shared__ double sh[kThreads / 64];
    double part[K];
#pragma unroll
    for (int j = 0; j < K; ++j) part[j] = 0.0;
    const int lb = xcd_block(blockIdx.x, gridDim.x, nxcd);
    const int wv = wave_index(), lane = threadIdx.x & 63;
    int w0, w1, wstep;
    window_walk((nslices + kWin - 1) / kWin, lb, gridDim.x, nxcd, w0, w1, wstep);
    for (int wi = w0; wi < w1; wi += wstep) {
        const int sl = wi * kWin + wv;
        if (sl >= nslices) break;
        const uint32_t c0 = sptr[sl];
        const int r = sl * kSlice + lane;
        const int nr = (int)(sptr[sl + 1] - c0) / 3;
        const int64_t rbase = (int64_t)(c0 / 3u) * kSlice + lane, vbase = (int64_t)c0 * kSlice + lane;
        double acc[K];
#pragma unroll
        for (int j = 0; j < K; ++j) acc[j] = 0.0;
        int c[UR];
        double v[UR][3];
#pragma unroll
        for (int u = 0; u < UR; ++u) {
            c[u] = 0;
#pragma unroll
            for (int e = 0; e < 3; ++e) v[u][e] = 0.0;
            if (u < nr) {
                c[u] = __builtin_nontemporal_load(&col3[rbase + (int64_t)u * kSlice]);
#pragma unroll
                for (int e = 0; e < 3; ++e) v[u][e] = __builtin_nontemporal_load(&val[vbase + (int64_t)(3 * u + e) * kSlice]);
            }
        }
        for (int j0 = 0; j0 < nr; j0 += UR) {
            int cn[UR];
            double vn[UR][3];
#pragma unroll
            for (int u = 0; u < UR; ++u) {
                cn[u] = 0;
#pragma unroll
                for (int e = 0; e < 3; ++e) vn[u][e] = 0.0;
                if (j0 + UR + u < nr) {
                    const int jr = j0 + UR + u;
                    cn[u] = __builtin_nontemporal_load(&col3[rbase + (int64_t)jr * kSlice]);
#pragma unroll
                    for (int e = 0; e < 3; ++e)
                        vn[u][e] = __builtin_nontemporal_load(&val[vbase + (int64_t)(3 * jr + e) * kSlice]);
                }
            }
#pragma unroll
            for (int u = 0; u < UR; ++u)
                if (j0 + u < nr) {
                    const double *xc = x + (int64_t)c[u] * K;
#pragma unroll
                    for (int e = 0; e < 3; ++e)
#pragma unroll
                        for (int j = 0; j < K; ++j) acc[j] = fma(v[u][e], xc[e * K + j], acc[j]);
                }
#pragma unroll
            for (int u = 0; u < UR; ++u) {
                c[u] = cn[u];
#pragma unroll
                for (int e = 0; e < 3; ++e) v[u][e] = vn[u][e];
            }
        }
        if (r < n) {
#pragma unroll
            for (int j = 0; j < K; ++j) {
                y[(int64_t)r * K + j] = acc[j];
                if (DOT) part[j] = fma(acc[j], w[(int64_t)r * K + j], part[j]);
            }
        }
    }
    if (DOT) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const double bs = block_sum(part[j], sh);
            if (threadIdx.x == 0) partials[(size_t)j * gridDim.x + lb] = bs;
        }
    }
}

// ---------------------------------------------------------------------------------------
// PCG over a block of K right-hand sides (x0 = 0): K independent recurrences with their own
// scalars and stopping tests; the vectors are n x K row-major blocks and every product reads
// its matrix once for the K columns.
// ---------------------------------------------------------------------------------------
struct MultiScal {
    double bb, rho, alpha, beta, rr, tr;
    int32_t done, iters, status, pad;
};
enum : int { MF_BB = 0, MF_RHO0 = 1, MF_PQ = 2, MF_RR = 3, MF_RZ = 4, MF_TRUE = 5 };

// One block per column: the column's partial sums (nb per column) added in block order, then
// the scalar step of the textbook recurrence for that column.
__global__ __launch_bounds__(kThreads) void k_fin_multi(const double *__restrict__ partials, int nb, int mode,
                                                         double rtol, int maxit, MultiScal *sc) {
    __shared__ double sh[kThreads / 64];
    const int j = blockIdx.x;
    const int per = (nb + kThreads - 1) / kThreads;
    const int lo = threadIdx.x * per, hi = min(nb, lo + per);
    double v = 0.0;
    for (int b = lo; b < hi; ++b) v += partials[(size_t)j * nb + b];
    const double t = block_sum(v, sh);
    if (threadIdx.x != 0) return;
    MultiScal &m = sc[j];
    switch (mode) {
        case MF_BB:
            m.bb = t;
            m.rr = t;
            m.iters = 0;
            m.done = 0;
            m.status = AFSAI_ERR_NOT_CONVERGED;
            if (t == 0.0 || sqrt(t) <= rtol * sqrt(t)) {
                m.done = 1;  // b = 0 (x = 0) or converged at x0
                m.status = AFSAI_OK;
            } else if (maxit <= 0) {
                m.done = 1;
            }
            break;
        case MF_RHO0: m.rho = t; break;
        case MF_PQ:
            if (!m.done) {
                if (!(t > 0.0)) {
                    m.done = 1;
                    m.status = AFSAI_ERR_NOT_SPD;
                } else {
                    m.alpha = m.rho / t;
                }
            }
            break;
        case MF_RR:
            if (!m.done) {
                m.rr = t;
                m.iters += 1;
                if (sqrt(t) <= rtol * sqrt(m.bb)) {
                    m.done = 1;
                    m.status = AFSAI_OK;
                } else if (m.iters >= maxit) {
                    m.done = 1;
                }
            }
            break;
        case MF_RZ:
            if (!m.done) {
                m.beta = t / m.rho;
                m.rho = t;
            }
            break;
        default: m.tr = t; break;
    }
}

// The vector kernels take one thread per entry of the n x K block: block b covers the
// entries of rows [i0, i1) (contiguous, in block order) and, since kThreads is a multiple of
// K, thread t always meets column t % K, so every thread sums one column in a fixed order.
template <int K>
__device__ __forceinline__ void multi_range(int n, int64_t &e0, int64_t &e1) {
    int i0, i1;
    block_range(0, n, blockIdx.x, gridDim.x, i0, i1);
    e0 = (int64_t)i0 * K;
    e1 = (int64_t)i1 * K;
}

// this block's per-column sums of part (thread t holding column t % K) at
// partials[j * gridDim.x + block]: lanes of one column added by shuffles, then the
// wavefronts in order
template <int K>
__device__ __forceinline__ void multi_store(double part, double *sh /* kThreads / 64 * K */, double *partials) {
    static_assert(kThreads % K == 0 && 64 % K == 0, "a thread keeps one column");
#pragma unroll
    for (int off = 32; off >= K; off >>= 1) part += __shfl_xor(part, off, 64);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane < K) sh[w * K + lane] = part;
    __syncthreads();
    if (threadIdx.x < K) {
        double t = 0.0;
        for (int k = 0; k < kThreads / 64; ++k) t += sh[k * K + threadIdx.x];
        partials[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
    }
}

// x = 0, r = b; partial sums of b.b per column
template <int K>
__global__ __launch_bounds__(kThreads) void k_multi_init(int n, const double *__restrict__ b, double *__restrict__ x,
                                                          double *__restrict__ r, double *__restrict__ partials) {
    __shared__ double sh[kThreads / 64 * K];
    int64_t e0, e1;
    multi_range<K>(n, e0, e1);
    double part = 0.0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kThreads) {
        const double be = b[e];
        x[e] = 0.0;
        r[e] = be;
        part = fma(be, be, part);
    }
    multi_store<K>(part, sh, partials);
}

// partial sums of a.b per column (and copy = a when given)
template <int K>
__global__ __launch_bounds__(kThreads) void k_multi_dot(int n, const double *__restrict__ a, const double *__restrict__ b,
                                                         double *__restrict__ copy, double *__restrict__ partials) {
    __shared__ double sh[kThreads / 64 * K];
    int64_t e0, e1;
    multi_range<K>(n, e0, e1);
    double part = 0.0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kThreads) {
        const double ae = a[e];
        if (copy) copy[e] = ae;
        part = fma(ae, b[e], part);
    }
    multi_store<K>(part, sh, partials);
}

// columns still running: x += alpha p, r -= alpha q; partial sums of r.r per column
template <int K>
__global__ __launch_bounds__(kThreads) void k_multi_xr(int n, double *__restrict__ x, double *__restrict__ r,
                                                        const double *__restrict__ p, const double *__restrict__ q,
                                                        const MultiScal *__restrict__ sc, double *__restrict__ partials) {
    __shared__ double sh[kThreads / 64 * K];
    int64_t e0, e1;
    multi_range<K>(n, e0, e1);
    const int j = threadIdx.x % K;
    const bool run = !sc[j].done;
    const double alpha = sc[j].alpha;
    double part = 0.0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kThreads) {
        double re = r[e];
        if (run) {
            x[e] = fma(alpha, p[e], x[e]);
            re = fma(-alpha, q[e], re);
            r[e] = re;
        }
        part = fma(re, re, part);
    }
    multi_store<K>(part, sh, partials);
}

// columns still running: p = z + beta p
template <int K>
__global__ __launch_bounds__(kThreads) void k_multi_p(int n, const double *__restrict__ z, double *__restrict__ p,
                                                       const MultiScal *__restrict__ sc) {
    int64_t e0, e1;
    multi_range<K>(n, e0, e1);
    const int j = threadIdx.x % K;
    if (sc[j].done) return;
    const double beta = sc[j].beta;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kThreads) p[e] = fma(beta, p[e], z[e]);
}

// partial sums of (b - q).(b - q) per column
template <int K>
__global__ __launch_bounds__(kThreads) void k_multi_resid(int n, const double *__restrict__ b,
                                                           const double *__restrict__ q, double *__restrict__ partials) {
    __shared__ double sh[kThreads / 64 * K];
    int64_t e0, e1;
    multi_range<K>(n, e0, e1);
    double part = 0.0;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kThreads) {
        const double d = b[e] - q[e];
        part = fma(d, d, part);
    }
    multi_store<K>(part, sh, partials);
}

template <int K, bool DOT>
static void spmm_launch(const Sell &S, const double *x, double *y, const double *w, double *partials, int nb,
                        const DeviceInfo &di, hipStream_t s) {
    if (S.col3 && !S.f32 && !S.lens)
        hipLaunchKernelGGL((k_sell_spmm_runs<K, DOT>), dim3(nb), dim3(kThreads), 0, s, S.n, S.nslices, S.sptr, S.col3,
                           (const double *)S.val, x, y, di.num_xcds, w, partials);
    else if (S.f32)
        hipLaunchKernelGGL((k_sell_spmm<K, float, DOT>), dim3(nb), dim3(kThreads), 0, s, S.n, S.nslices, S.sptr, S.perm,
                           S.lens, S.col, (const float *)S.val, x, y, di.num_xcds, w, partials);
    else
        hipLaunchKernelGGL((k_sell_spmm<K, double, DOT>), dim3(nb), dim3(kThreads), 0, s, S.n, S.nslices, S.sptr, S.perm,
                           S.lens, S.col, (const double *)S.val, x, y, di.num_xcds, w, partials);
}

static int check_csr_arg(const afsai_csr *A, const char *who) {
    if (!A) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "%s: A is NULL", who);
    if (A->n <= 0 || A->nnz < A->n) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "%s: n = %d, nnz = %d", who, A->n, A->nnz);
    if (!A->row_ptr || !A->col_idx || !A->val) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "%s: null CSR array", who);
    return AFSAI_OK;
}

static Csr csr_of(const afsai_csr *A) {
    Csr c;
    c.n = A->n;
    c.nnz = A->nnz;
    c.rp = A->row_ptr;
    c.ci = A->col_idx;
    c.val = A->val;
    return c;
}

// work vectors of the solver: r, r', z, p, p', q, t
constexpr int kWorkVectors = 7;

// A solve in progress: PCG (Sec. 5.2) over a batch of nsys independent systems (row0: host,
// nsys + 1 entries; one system when nsys == 1).  begin() enqueues the start and two chunks of
// iterations; advance() reads the state after the oldest chunk in flight (waiting for it when
// `block`, else returning at once if it is not there yet) and enqueues the next chunk, sized from
// the slowest system's convergence rate so that few iterations are queued past convergence
// (those return at once on the device flags); finish() computes the true residuals and the
// results.  All work goes to one stream; any number of runs may be in progress on different
// streams (the serving loop advances many of them from one host thread).
// A stream per thread and device on which iterations are captured into graphs (never run).
static hipStream_t capture_stream(int device) {
    struct Streams {
        hipStream_t s[64] = {};
        ~Streams() {
            for (hipStream_t &x : s)
                if (x) (void)hipStreamDestroy(x);
        }
    };
    thread_local Streams ts;
    if (device < 0 || device >= 64) return nullptr;
    if (!ts.s[device] && hipStreamCreateWithFlags(&ts.s[device], hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        ts.s[device] = nullptr;
    }
    return ts.s[device];
}

class PcgRun {
  public:
    // prepared: A's SELL layout converted beforehand (one system; not owned), else converted
    // by begin() for this solve
    PcgRun(const afsai_csr &A, afsai_precond P, int nsys, const int32_t *row0, const double *b, double *x,
           double rtol, int32_t maxit, hipStream_t s, const Sell *prepared = nullptr)
        : A_(A), P_(P), nsys_(nsys), b_(b), x_(x), rtol_(rtol), maxit_(maxit), s_(s), prepared_(prepared) {
        if (nsys > 1 && row0) row0_.assign(row0, row0 + nsys + 1);
        else row0_ = {0, A.n};
    }
    ~PcgRun() {
        if (started_) (void)hipStreamSynchronize(s_);
        for (int k = 0; k < 2; ++k) {
            if (gexec_[k]) (void)hipGraphExecDestroy(gexec_[k]);
            if (graph_[k]) (void)hipGraphDestroy(graph_[k]);
        }
        if (!prepared_) sell_free(&As_);
        for (hipEvent_t e : {t0_, t1_, ev_[0], ev_[1], ev_[2], ev_[3]})
            if (e) (void)hipEventDestroy(e);
        pinned_free(hsc_);
    }
    PcgRun(const PcgRun &) = delete;
    PcgRun &operator=(const PcgRun &) = delete;

    int begin() {
        const int n = A_.n;
        int rc;
        if ((rc = device_info(&di_))) return rc;
        AFSAI_HIP_TRY(hipEventCreate(&t0_));
        AFSAI_HIP_TRY(hipEventCreate(&t1_));
        for (hipEvent_t &e : ev_) AFSAI_HIP_TRY(hipEventCreate(&e));
        // the host copies of the scalars (cached pinned blocks: no hipHostMalloc per solve)
        hsc_ = (PcgScalars *)pinned_alloc(2 * sizeof(PcgScalars) * (size_t)nsys_);
        if (!hsc_) return set_error_code(AFSAI_ERR_NO_MEMORY, "pcg: out of pinned host memory");
        hs_[0] = hsc_;
        hs_[1] = hsc_ + nsys_;
        AFSAI_HIP_TRY(hipHostGetDevicePointer((void **)&dhs_[0], hsc_, 0));
        dhs_[1] = dhs_[0] + nsys_;
        AFSAI_HIP_TRY(hipEventRecord(t0_, s_));
        started_ = true;
        if ((rc = make_batch_maps(n, nsys_, row0_.data(), di_, s_, &bm_))) return rc;
        Segments seg;
        seg.nsys = nsys_;
        seg.row0 = row0_.data();

        const size_t np = (size_t)2 * std::max(bm_.sell.nblocks, std::max(bm_.vec.nblocks, di_.num_cus * 16)) + 64;
        const size_t nsc_elems = (sizeof(PcgScalars) * (size_t)nsys_ + sizeof(double) - 1) / sizeof(double);
        const size_t need = (size_t)kWorkVectors * n + np + nsc_elems + 16;
        double *ws = nullptr;
        if (P_ && P_->work_elems >= need) {
            ws = P_->work;
        } else {
            if ((rc = dalloc(own_, need * sizeof(double), s_))) return rc;
            ws = own_.as<double>();
        }
        r_ = ws;
        r2_ = ws + n;
        z_ = ws + 2 * (size_t)n;
        p_ = ws + 3 * (size_t)n;
        p2_ = ws + 4 * (size_t)n;
        q_ = ws + 5 * (size_t)n;
        t_ = ws + 6 * (size_t)n;
        partials_ = ws + kWorkVectors * (size_t)n;
        sc_ = (PcgScalars *)(partials_ + np);

        // A in the SELL-64 layout for the iteration (one conversion per solve); CSR only for one
        // system when asked for
        use_sell_ = option(AFSAI_OPT_PCG_CSR_A) == 0 || nsys_ > 1 || prepared_;
        if (prepared_) {
            As_ = *prepared_;
        } else if (use_sell_) {
            ProfScope ps("sell_A", s_);
            if ((rc = sell_from_csr(n, A_.nnz, A_.row_ptr, A_.col_idx, A_.val, false, false, &As_, di_, s_, seg)))
                return rc;
        }
        const dim3 gv(bm_.vec.nblocks), gs(bm_.nsys);
        const int plain = P_ ? 0 : 1;
        hipLaunchKernelGGL(k_set_scalars, dim3((nsys_ + 255) / 256), dim3(256), 0, s_, sc_, nsys_, rtol_, maxit_,
                           plain);
        // r0 = b - A x0
        spmv_A("spmv_A", x_, q_, nullptr, FIN_NONE, false);
        hipLaunchKernelGGL(k_init_residual, gv, dim3(kThreads), 0, s_, n, b_, q_, r_, partials_, bm_.vec.mp, bm_.sy,
                           di_.num_xcds);
        hipLaunchKernelGGL(k_finalize, gs, dim3(kThreads), 0, s_, partials_, bm_.vec.nblocks, bm_.vec.mp,
                           (int)FIN_INIT, sc_);
        // z0 = M^-1 r0, rho0 = r0.z0, p0 = z0
        zz_ = z_;
        if (P_) {
            sell_spmv("spmv_G", P_->sg, bm_, r_, t_, nullptr, nullptr, sc_, FIN_NONE, di_, s_);
            sell_spmv("spmv_GT_dot", P_->sgt, bm_, t_, z_, r_, partials_, sc_, FIN_RHO0, di_, s_);
        } else {
            zz_ = r_;
        }
        // fused products where launches dominate (small systems), separate updates where the
        // fused products' second gather costs more than the update kernels; the fused kernels
        // need layouts without a tail
        const int64_t form = option(AFSAI_OPT_PCG_FORM);
        int nmax = 0;
        for (int k = 0; k < nsys_; ++k) nmax = std::max(nmax, row0_[k + 1] - row0_[k]);
        const bool want_fused = form == 2 || (form == 0 && nmax < kFusedMaxRows);
        fused_ = P_ && use_sell_ && want_fused && !As_.tail && !P_->sg.tail && !As_.perm && !P_->sg.perm;
        // A's product with one column index per run of three consecutive columns where every
        // row is made of such runs (3 x 3 blocks): 9.3 instead of 12 bytes per FP64 entry, the
        // same sums (the fused kernels keep the plain layout)
        if (use_sell_ && !prepared_ && !fused_ && option(AFSAI_OPT_SELL_RUNS) != 1) {
            ProfScope ps("sell_A_runs", s_);
            if ((rc = sell_group_runs(&As_, di_, s_))) return rc;
        }
        // iterations replayed from captured graphs only when asked for (never while the kernel
        // timer is on: its events would be captured); on MI355X with ROCm 7 enqueuing the
        // kernels measured faster than replaying graphs at every size tried
        use_graph_ = !profiling_on() && option(AFSAI_OPT_PCG_GRAPH) == 2;
        if (!fused_)
            hipLaunchKernelGGL(k_update_p, gv, dim3(kThreads), 0, s_, n, p_, zz_, sc_, 1, bm_.vec.mp, bm_.sy,
                               di_.num_xcds);
        mark0_ = prof_mark();
        prev_it_.assign(nsys_, 0);
        prev_rr_.assign(nsys_, 0.0);
        rate_.assign(nsys_, 0.0);
        tol_.assign(nsys_, 0.0);
        have_prev_.assign(nsys_, 0);
        // the state after the start (a chunk of no iterations) and a first chunk in flight
        // before any state is read
        if ((rc = enqueue_chunk(0))) return rc;
        if ((rc = enqueue_chunk(kFirstChunk))) return rc;
        return AFSAI_OK;
    }

    // Returns AFSAI_OK and sets *finished; with block == false returns at once (finished
    // false) when the oldest chunk in flight has not completed.
    int advance(bool block, bool *finished) {
        *finished = false;
        if (done_) {
            *finished = true;
            return AFSAI_OK;
        }
        const int slot = (c_ - 2) & 1;  // state after the oldest chunk in flight
        hipEvent_t ev = ev_[(c_ - 2) & 3];
        if (!block) {
            const hipError_t q = hipEventQuery(ev);
            if (q == hipErrorNotReady) return AFSAI_OK;
            if (q != hipSuccess) AFSAI_HIP_TRY(q);
        } else {
            AFSAI_HIP_TRY(hipEventSynchronize(ev));
        }
        // GPU time of that chunk (from the end of the chunk before it)
        if (c_ >= 3 && its_[(c_ - 2) & 3] > 0) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev_[(c_ - 3) & 3], ev) == hipSuccess && ms > 0.f) {
                gpu_us_ += 1e3 * ms;
                it_us_ = 1e3 * ms / its_[(c_ - 2) & 3];
            } else {
                (void)hipGetLastError();
            }
        }
        const PcgScalars *st = hs_[slot];
        bool all_done = true;
        for (int k = 0; k < nsys_; ++k) {
            if (st[k].done != DONE_NO) continue;
            all_done = false;
            tol_[k] = st[k].tol;
            if (have_prev_[k] && st[k].it > prev_it_[k] && st[k].rr > 0.0 && prev_rr_[k] > 0.0) {
                const double rt = std::log(st[k].rr / prev_rr_[k]) / (st[k].it - prev_it_[k]);
                if (rt < 0.0) rate_[k] = rt;
            }
            if (st[k].rr > 0.0) {
                prev_rr_[k] = st[k].rr;
                prev_it_[k] = st[k].it;
                have_prev_[k] = 1;
            }
        }
        if (all_done || enqueued_ >= maxit_) {
            done_ = true;
            *finished = true;
            return AFSAI_OK;
        }
        // Chunk size: enough GPU work to cover the host's turnaround (two chunks are in flight)
        // and a fixed share of the time so far, so that the iterations enqueued past
        // convergence stay a small part of the solve; capped by the iterations the slowest
        // active system still needs at its observed rate.
        int todo = kFirstChunk;
        if (it_us_ > 0.0) {
            const double window_us = std::max(kMinChunkUs, gpu_us_ * kChunkShare);
            todo = (int)std::min(64.0, std::max(1.0, std::ceil(window_us / it_us_)));
        }
        int need_max = -1;
        for (int k = 0; k < nsys_; ++k) {
            if (st[k].done != DONE_NO) continue;
            if (!(rate_[k] < 0.0 && have_prev_[k])) {
                need_max = -1;
                break;
            }
            const double need_it = std::ceil(std::log(tol_[k] * tol_[k] / prev_rr_[k]) / rate_[k]);
            need_max = std::max(need_max, (int)need_it - (enqueued_ - prev_it_[k]) + 1);
        }
        if (need_max >= 0) todo = std::min(todo, std::max(1, need_max));
        return enqueue_chunk(todo);
    }

    int finish(afsai_pcg_info *info) {
        const int n = A_.n;
        AFSAI_HIP_TRY(hipStreamSynchronize(s_));
        std::vector<PcgScalars> fin_s(nsys_);
        const size_t scbytes = sizeof(PcgScalars) * (size_t)nsys_;
        AFSAI_HIP_TRY(hipMemcpyAsync(fin_s.data(), sc_, scbytes, hipMemcpyDeviceToHost, s_));
        AFSAI_HIP_TRY(hipStreamSynchronize(s_));
        int it_max = 0;
        for (int k = 0; k < nsys_; ++k) it_max = std::max(it_max, (int)fin_s[k].it);
        {
            const int keep_to = it_max >= 1 && it_max <= (int)marks_.size() ? marks_[it_max - 1] : mark0_;
            prof_drop(keep_to, prof_mark());
        }
        const dim3 gv(bm_.vec.nblocks), gs(bm_.nsys);
        hipLaunchKernelGGL(k_zero_rhs, gv, dim3(kThreads), 0, s_, n, x_, sc_, bm_.vec.mp, bm_.sy, di_.num_xcds);
        // true residuals ||b - A x||
        spmv_A("spmv_A", x_, q_, nullptr, FIN_NONE, false);
        hipLaunchKernelGGL(k_resid_norm, gv, dim3(kThreads), 0, s_, n, b_, q_, partials_, bm_.vec.mp, bm_.sy,
                           di_.num_xcds);
        hipLaunchKernelGGL(k_finalize, gs, dim3(kThreads), 0, s_, partials_, bm_.vec.nblocks, bm_.vec.mp,
                           (int)FIN_RESID, sc_);
        AFSAI_HIP_TRY(hipMemcpyAsync(hs_[0], sc_, scbytes, hipMemcpyDeviceToHost, s_));
        AFSAI_HIP_TRY(hipEventRecord(t1_, s_));
        AFSAI_HIP_TRY(hipStreamSynchronize(s_));
        AFSAI_HIP_TRY(hipGetLastError());
        float ms = 0.f;
        AFSAI_HIP_TRY(hipEventElapsedTime(&ms, t0_, t1_));
        prof_flush();
        int status = AFSAI_OK;
        for (int k = 0; k < nsys_ && status == AFSAI_OK; ++k) {
            const PcgScalars &f = fin_s[k];
            if (f.done == DONE_NOT_SPD) {
                if (nsys_ == 1)
                    set_error("pcg_solve: p.Ap <= 0 at iteration %d (matrix or preconditioner not SPD)", f.it + 1);
                else
                    set_error("pcg_solve_batched: system %d: p.Ap <= 0 at iteration %d (not SPD)", k, f.it + 1);
                status = AFSAI_ERR_NOT_SPD;
            } else if (f.done == DONE_MAXIT || f.done == DONE_NO) {
                if (nsys_ == 1) set_error("pcg_solve: not converged in %d iterations", f.it);
                else set_error("pcg_solve_batched: system %d not converged in %d iterations", k, f.it);
                status = AFSAI_ERR_NOT_CONVERGED;
            }
        }
        if (info) {
            for (int k = 0; k < nsys_; ++k) {
                const PcgScalars &f = fin_s[k];
                const double nb = sqrt(f.bb);
                info[k].iters = f.it;
                info[k].converged = (f.done == DONE_CONVERGED || f.done == DONE_ZERO_RHS) ? 1 : 0;
                info[k].relres = nb > 0 ? sqrt(f.rr) / nb : 0.0;
                info[k].true_relres = (nb > 0 && f.done != DONE_ZERO_RHS) ? sqrt(hs_[0][k].resid) / nb : 0.0;
                info[k].ms = ms;
            }
        }
        return status;
    }

  private:
    // products inside the iteration stop with their system (gate); the first and the final
    // A x run for every system
    void spmv_A(const char *name, const double *xin, double *yout, const double *w, int fin, bool gate) {
        PcgScalars *g = gate ? sc_ : nullptr;
        if (use_sell_) sell_spmv(name, As_, bm_, xin, yout, w, w ? partials_ : nullptr, g, fin, di_, s_);
        else spmv(name, csr_of(&A_), xin, yout, w, w ? partials_ : nullptr, g, fin, di_, s_);
    }

    // One iteration: from the captured graph of its buffer parity (captured at its first use;
    // the first fused iteration, which forms p = z, always runs directly), else enqueued.
    // Capture runs on a private stream of this thread (the caller's stream may be the null
    // stream, which cannot capture); nothing executes there, the graph is launched on s_.
    int launch_iteration() {
        const int par = fused_ ? (iter_no_ & 1) : 0;
        if (!use_graph_ || (fused_ && iter_no_ == 0)) {
            enqueue_iteration();
            return AFSAI_OK;
        }
        if (!gexec_[par]) {
            hipStream_t cs = capture_stream(di_.device);
            hipGraph_t g = nullptr;
            hipError_t e = cs ? hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) : hipErrorUnknown;
            if (e == hipSuccess) {
                const int it0 = iter_no_;
                const size_t nmarks = marks_.size();
                hipStream_t keep = s_;
                s_ = cs;
                enqueue_iteration();
                s_ = keep;
                iter_no_ = it0;
                marks_.resize(nmarks);
                e = hipStreamEndCapture(cs, &g);
            }
            if (e == hipSuccess && g) e = hipGraphInstantiate(&gexec_[par], g, nullptr, nullptr, 0);
            if (e != hipSuccess || !gexec_[par]) {
                // capture not available: enqueue directly from here on
                (void)hipGetLastError();
                if (g) (void)hipGraphDestroy(g);
                gexec_[par] = nullptr;
                use_graph_ = false;
                enqueue_iteration();
                return AFSAI_OK;
            }
            graph_[par] = g;
        }
        AFSAI_HIP_TRY(hipGraphLaunch(gexec_[par], s_));
        marks_.push_back(prof_mark());
        ++iter_no_;
        return AFSAI_OK;
    }

    void enqueue_iteration() {
        const int n = A_.n;
        const dim3 gv(bm_.vec.nblocks), gs(bm_.nsys);
        if (fused_) {
            // p and r are double-buffered: the products read neighbours' old entries while
            // owners store the new ones
            const bool odd = (iter_no_ & 1) == 0;  // iteration 1, 3, ...: p -> p2, r -> r2
            double *p_old = odd ? p_ : p2_, *p_new = odd ? p2_ : p_;
            double *r_old = odd ? r_ : r2_, *r_new = odd ? r2_ : r_;
            sell_fused<FUSE_AP>("spmv_A_dot", As_, bm_, z_, p_old, p_new, nullptr, nullptr, q_, partials_, sc_,
                                iter_no_ == 0 ? 1 : 0, FIN_ALPHA, di_, s_);
            sell_fused<FUSE_GR>("spmv_G_upd", P_->sg, bm_, r_old, q_, r_new, x_, p_new, t_, partials_, sc_, 0,
                                FIN_UPDATE, di_, s_);
            marks_.push_back(prof_mark());
            sell_spmv("spmv_GT_dot", P_->sgt, bm_, t_, z_, r_new, partials_, sc_, FIN_BETA, di_, s_);
            ++iter_no_;
            return;
        }
        spmv_A("spmv_A_dot", p_, q_, p_, FIN_ALPHA, true);
        {
            ProfScope ps("update_xr", s_);
            hipLaunchKernelGGL(k_update_xr, gv, dim3(kThreads), 0, s_, n, x_, r_, p_, q_, partials_, sc_, bm_.vec.mp,
                               bm_.sy, di_.num_xcds);
        }
        hipLaunchKernelGGL(k_finalize, gs, dim3(kThreads), 0, s_, partials_, bm_.vec.nblocks, bm_.vec.mp,
                           (int)FIN_UPDATE, sc_);
        marks_.push_back(prof_mark());
        if (P_) {
            sell_spmv("spmv_G", P_->sg, bm_, r_, t_, nullptr, nullptr, sc_, FIN_NONE, di_, s_);
            sell_spmv("spmv_GT_dot", P_->sgt, bm_, t_, z_, r_, partials_, sc_, FIN_BETA, di_, s_);
        }
        {
            ProfScope ps("update_p", s_);
            hipLaunchKernelGGL(k_update_p, gv, dim3(kThreads), 0, s_, n, p_, zz_, sc_, 0, bm_.vec.mp, bm_.sy,
                               di_.num_xcds);
        }
        ++iter_no_;
    }

    // todo iterations (at most what maxit leaves), then a copy of the scalars into the host
    // slot of this chunk and its event
    int enqueue_chunk(int todo) {
        if (todo > maxit_ - enqueued_) todo = maxit_ - enqueued_;
        for (int k = 0; k < todo; ++k) {
            int rc;
            if ((rc = launch_iteration())) return rc;
        }
        enqueued_ += todo;
        const int slot = c_ & 1;
        const int nw = nsys_ * (int)(sizeof(PcgScalars) / sizeof(double));
        hipLaunchKernelGGL(k_publish, dim3((nw + kThreads - 1) / kThreads), dim3(kThreads), 0, s_, sc_, nw,
                           dhs_[slot]);
        its_[c_ & 3] = todo;
        AFSAI_HIP_TRY(hipEventRecord(ev_[c_ & 3], s_));
        ++c_;
        return AFSAI_OK;
    }

    const afsai_csr A_;
    afsai_precond P_;
    int nsys_;
    std::vector<int32_t> row0_;
    const double *b_;
    double *x_;
    double rtol_;
    int32_t maxit_;
    hipStream_t s_;
    DeviceInfo di_;
    BatchMaps bm_;
    DevBuf own_;
    const Sell *prepared_ = nullptr;
    Sell As_;
    bool use_sell_ = true, fused_ = false, started_ = false, done_ = false, use_graph_ = false;
    hipGraph_t graph_[2] = {nullptr, nullptr};
    hipGraphExec_t gexec_[2] = {nullptr, nullptr};
    double *r_ = nullptr, *r2_ = nullptr, *z_ = nullptr, *p_ = nullptr, *p2_ = nullptr, *q_ = nullptr, *t_ = nullptr;
    const double *zz_ = nullptr;
    double *partials_ = nullptr;
    PcgScalars *sc_ = nullptr;
    PcgScalars *hsc_ = nullptr;
    PcgScalars *hs_[2] = {nullptr, nullptr};
    PcgScalars *dhs_[2] = {nullptr, nullptr};  // device addresses of hs_
    hipEvent_t t0_ = nullptr, t1_ = nullptr, ev_[4] = {nullptr, nullptr, nullptr, nullptr};
    int its_[4] = {0, 0, 0, 0};
    double gpu_us_ = 0.0, it_us_ = 0.0;
    int iter_no_ = 0, enqueued_ = 0, c_ = 0, mark0_ = 0;
    std::vector<int> marks_, prev_it_;
    std::vector<double> prev_rr_, rate_, tol_;
    std::vector<char> have_prev_;
};

struct PcgTask {
    PcgRun run;
    PcgTask(const afsai_csr &A, afsai_precond P, const double *b, double *x, double rtol, int32_t maxit,
            hipStream_t s)
        : run(A, P, 1, nullptr, b, x, rtol, maxit, s) {}
};

int pcg_task_begin(const afsai_csr &A, afsai_precond P, const double *b, double *x, double rtol, int32_t maxit,
                   hipStream_t stream, PcgTask **out) {
    *out = nullptr;
    PcgTask *t = new PcgTask(A, P, b, x, rtol, maxit, stream);
    const int rc = t->run.begin();
    if (rc) {
        delete t;
        return rc;
    }
    *out = t;
    return AFSAI_OK;
}
int pcg_task_advance(PcgTask *t, bool block, bool *finished) { return t->run.advance(block, finished); }
int pcg_task_finish(PcgTask *t, afsai_pcg_info *info) { return t->run.finish(info); }
void pcg_task_free(PcgTask *t) { delete t; }

static int pcg_batch(const afsai_csr *A, afsai_precond P, int nsys, const int32_t *row0, const double *b, double *x,
                     double rtol, int32_t maxit, hipStream_t s, afsai_pcg_info *info, const Sell *prepared = nullptr) {
    PcgRun run(*A, P, nsys, row0, b, x, rtol, maxit, s, prepared);
    int rc = run.begin();
    if (rc) return rc;
    bool fin = false;
    while (!fin)
        if ((rc = run.advance(true, &fin))) return rc;
    return run.finish(info);
}

}  // namespace afsai

using namespace afsai;

extern "C" {

int afsai_spmv(const afsai_csr *A, const double *x, double *y, void *stream) {
    int rc = check_csr_arg(A, "afsai_spmv");
    if (rc) return rc;
    if (!x || !y) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_spmv: null vector");
    DeviceInfo di;
    if ((rc = device_info(&di))) return rc;
    hipStream_t s = (hipStream_t)stream;
    spmv("spmv_A", csr_of(A), x, y, nullptr, nullptr, nullptr, FIN_NONE, di, s);
    AFSAI_HIP_TRY(hipGetLastError());
    return AFSAI_OK;
}

}  // extern "C"

namespace afsai {

template <int K>
static int pcg_multi(const afsai_csr *A, afsai_precond P, const double *B, double *X, double rtol, int32_t maxit,
                     hipStream_t s, const DeviceInfo &di, afsai_pcg_info *info) {
    const int n = A->n;
    int rc;
    Sell SA;
    {
        ProfScope ps("sell_A", s);
        if ((rc = sell_from_csr(n, A->nnz, A->row_ptr, A->col_idx, A->val, false, false, &SA, di, s))) return rc;
    }
    struct Free {
        Sell *S;
        ~Free() { sell_free(S); }
    } free_sa{&SA};
    if (SA.tail) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "pcg_solve_multi: split SELL layouts are not supported");
    if (option(AFSAI_OPT_SELL_RUNS) != 1) {
        ProfScope ps("sell_A_runs", s);
        if ((rc = sell_group_runs(&SA, di, s))) return rc;
    }
    const int nbA = blocks_for_slices(SA.nslices, di), nbv = blocks_for_vec(n, di);
    const int nbG = P ? blocks_for_slices(P->sg.nslices, di) : 0;
    const int nbGT = P ? blocks_for_slices(P->sgt.nslices, di) : 0;
    const int nbmax = std::max(std::max(nbA, nbv), std::max(nbG, nbGT));
    const size_t blk = (size_t)n * K;
    DevBuf work, parts, scb;
    if ((rc = dalloc(work, sizeof(double) * blk * 5, s))) return rc;
    if ((rc = dalloc(parts, sizeof(double) * (size_t)K * nbmax, s))) return rc;
    if ((rc = dalloc(scb, sizeof(MultiScal) * K, s))) return rc;
    double *R = work.as<double>(), *Z = R + blk, *Pv = Z + blk, *Q = Pv + blk, *T = Q + blk;
    double *pa = parts.as<double>();
    MultiScal *sc = scb.as<MultiScal>();
    auto fin = [&](int nb, int mode) {
        hipLaunchKernelGGL(k_fin_multi, dim3(K), dim3(kThreads), 0, s, pa, nb, mode, rtol, (int)maxit, sc);
    };
    // Z = M R with partial sums of R.Z; returns the blocks of that launch
    auto precond = [&]() {
        if (P) {
            spmm_launch<K, false>(P->sg, R, T, nullptr, nullptr, nbG, di, s);
            spmm_launch<K, true>(P->sgt, T, Z, R, pa, nbGT, di, s);
            return nbGT;
        }
        hipLaunchKernelGGL((k_multi_dot<K>), dim3(nbv), dim3(kThreads), 0, s, n, R, R, Z, pa);
        return nbv;
    };
    std::vector<MultiScal> h(K);
    auto read = [&]() -> int {
        AFSAI_HIP_TRY(hipGetLastError());
        AFSAI_HIP_TRY(hipMemcpyAsync(h.data(), sc, sizeof(MultiScal) * K, hipMemcpyDeviceToHost, s));
        AFSAI_HIP_TRY(hipStreamSynchronize(s));
        return AFSAI_OK;
    };
    auto all_done = [&]() {
        for (int j = 0; j < K; ++j)
            if (!h[j].done) return false;
        return true;
    };
    hipLaunchKernelGGL((k_multi_init<K>), dim3(nbv), dim3(kThreads), 0, s, n, B, X, R, pa);
    fin(nbv, MF_BB);
    fin(precond(), MF_RHO0);
    AFSAI_HIP_TRY(hipMemcpyAsync(Pv, Z, sizeof(double) * blk, hipMemcpyDeviceToDevice, s));
    if ((rc = read())) return rc;
    for (int it = 0; it < maxit && !all_done(); ++it) {
        spmm_launch<K, true>(SA, Pv, Q, Pv, pa, nbA, di, s);
        fin(nbA, MF_PQ);
        hipLaunchKernelGGL((k_multi_xr<K>), dim3(nbv), dim3(kThreads), 0, s, n, X, R, Pv, Q, sc, pa);
        fin(nbv, MF_RR);
        if ((rc = read())) return rc;
        if (all_done()) break;
        fin(precond(), MF_RZ);
        hipLaunchKernelGGL((k_multi_p<K>), dim3(nbv), dim3(kThreads), 0, s, n, Z, Pv, sc);
    }
    // true residuals ||b - A x|| per column
    spmm_launch<K, false>(SA, X, Q, nullptr, nullptr, nbA, di, s);
    hipLaunchKernelGGL((k_multi_resid<K>), dim3(nbv), dim3(kThreads), 0, s, n, B, Q, pa);
    fin(nbv, MF_TRUE);
    if ((rc = read())) return rc;
    int worst = AFSAI_OK;
    for (int j = 0; j < K; ++j) {
        const MultiScal &m = h[j];
        if (info) {
            info[j].iters = m.iters;
            info[j].converged = m.status == AFSAI_OK ? 1 : 0;
            info[j].relres = m.bb > 0.0 ? std::sqrt(m.rr / m.bb) : 0.0;
            info[j].true_relres = m.bb > 0.0 ? std::sqrt(m.tr / m.bb) : 0.0;
        }
        if (m.status == AFSAI_ERR_NOT_SPD) worst = AFSAI_ERR_NOT_SPD;
        else if (m.status != AFSAI_OK && worst == AFSAI_OK) worst = m.status;
    }
    if (worst == AFSAI_ERR_NOT_SPD) set_error("pcg_solve_multi: p.Ap <= 0 in a column (A not SPD)");
    else if (worst != AFSAI_OK) set_error("pcg_solve_multi: a column did not converge");
    return worst;
}

}  // namespace afsai

extern "C" {

int pcg_solve_multi(const afsai_csr *A, afsai_precond P, int32_t k, const double *B, double *X, double rtol,
                    int32_t maxit, void *stream, afsai_pcg_info *info) {
    if (k != 1 && k != 2 && k != 4 && k != 8)
        AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "pcg_solve_multi: k = %d (1, 2, 4 or 8)", k);
    int rc = check_csr_arg(A, "pcg_solve_multi");
    if (rc) return rc;
    if (!B || !X || B == X) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "pcg_solve_multi: null or aliased blocks");
    if (!(rtol > 0.0) || maxit < 0) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "pcg_solve_multi: rtol = %g, maxit = %d", rtol, maxit);
    if (P && (P->n != A->n || !P->seg_row0.empty() || P->sg.tail || P->sgt.tail))
        AFSAI_FAIL(AFSAI_ERR_INVALID_ARG,
                   "pcg_solve_multi: the preconditioner must be a single system of A's size without split layouts");
    DeviceInfo di;
    if ((rc = device_info(&di))) return rc;
    hipStream_t s = (hipStream_t)stream;
    const auto t0 = std::chrono::steady_clock::now();
    switch (k) {
        case 1: rc = pcg_multi<1>(A, P, B, X, rtol, maxit, s, di, info); break;
        case 2: rc = pcg_multi<2>(A, P, B, X, rtol, maxit, s, di, info); break;
        case 4: rc = pcg_multi<4>(A, P, B, X, rtol, maxit, s, di, info); break;
        default: rc = pcg_multi<8>(A, P, B, X, rtol, maxit, s, di, info); break;
    }
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info)
        for (int j = 0; j < k; ++j) info[j].ms = ms;
    return rc;
}

}  // extern "C"

namespace afsai {

// Y = A X with A's SELL layout S (no split layout), k in {1, 2, 4, 8}; synchronous on s
static int spmm_sell(const Sell &S, int32_t k, const double *X, double *Y, const DeviceInfo &di, hipStream_t s) {
    {
        ProfScope ps("spmm_A", s);
        const int nb = blocks_for_slices(S.nslices, di);
        switch (k) {
            case 1: spmm_launch<1, false>(S, X, Y, nullptr, nullptr, nb, di, s); break;
            case 2: spmm_launch<2, false>(S, X, Y, nullptr, nullptr, nb, di, s); break;
            case 4: spmm_launch<4, false>(S, X, Y, nullptr, nullptr, nb, di, s); break;
            default: spmm_launch<8, false>(S, X, Y, nullptr, nullptr, nb, di, s); break;
        }
    }
    const hipError_t le = hipGetLastError();
    const hipError_t se = hipStreamSynchronize(s);
    if (le != hipSuccess || se != hipSuccess) AFSAI_FAIL(AFSAI_ERR_HIP, "afsai_spmm: %s", hipGetErrorString(le != hipSuccess ? le : se));
    return AFSAI_OK;
}

static int spmm_args(int32_t k, const double *X, double *Y, const char *who) {
    if (k != 1 && k != 2 && k != 4 && k != 8) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "%s: k = %d (1, 2, 4 or 8)", who, k);
    if (!X || !Y) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "%s: null block", who);
    if (X == Y) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "%s: X and Y alias", who);
    return AFSAI_OK;
}

}  // namespace afsai

extern "C" {

int afsai_spmm(const afsai_csr *A, int32_t k, const double *X, double *Y, void *stream) {
    int rc = spmm_args(k, X, Y, "afsai_spmm");
    if (rc) return rc;
    if ((rc = check_csr_arg(A, "afsai_spmm"))) return rc;
    DeviceInfo di;
    if ((rc = device_info(&di))) return rc;
    hipStream_t s = (hipStream_t)stream;
    Sell S;
    {
        ProfScope ps("sell_A", s);
        if ((rc = sell_from_csr(A->n, A->nnz, A->row_ptr, A->col_idx, A->val, false, false, &S, di, s))) return rc;
    }
    if (S.tail || S.srow0) {
        sell_free(&S);
        AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_spmm: split SELL layouts (AFSAI_OPT_SELL_UNEVEN = 1) are not supported");
    }
    rc = spmm_sell(S, k, X, Y, di, s);
    sell_free(&S);
    return rc;
}

int afsai_matrix_prepare(const afsai_csr *A, void *stream, afsai_matrix *out) {
    clear_error();
    if (out) *out = nullptr;
    if (!out) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_matrix_prepare: null handle pointer");
    int rc = check_csr_arg(A, "afsai_matrix_prepare");
    if (rc) return rc;
    DeviceInfo di;
    if ((rc = device_info(&di))) return rc;
    hipStream_t s = (hipStream_t)stream;
    afsai_matrix M = new afsai_matrix_s();
    M->device = di.device;
    M->A = *A;
    {
        ProfScope ps("sell_A", s);
        rc = sell_from_csr(A->n, A->nnz, A->row_ptr, A->col_idx, A->val, false, false, &M->S, di, s);
        // run indices for pcg_solve_prepared's products, the per-entry columns kept for the
        // block products
        if (rc == AFSAI_OK && option(AFSAI_OPT_SELL_RUNS) != 1) rc = sell_group_runs(&M->S, di, s, true);
    }
    if (rc == AFSAI_OK && hipStreamSynchronize(s) != hipSuccess) rc = set_error_code(AFSAI_ERR_HIP, "afsai_matrix_prepare: synchronisation failed");
    if (rc != AFSAI_OK) {
        sell_free(&M->S);
        delete M;
        return rc;
    }
    *out = M;
    return AFSAI_OK;
}

void afsai_matrix_destroy(afsai_matrix M) {
    if (!M) return;
    (void)hipDeviceSynchronize();
    sell_free(&M->S);
    delete M;
}

int afsai_spmm_prepared(afsai_matrix M, int32_t k, const double *X, double *Y, void *stream) {
    if (!M) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_spmm_prepared: null matrix");
    int rc = spmm_args(k, X, Y, "afsai_spmm_prepared");
    if (rc) return rc;
    if (M->S.tail || M->S.srow0)
        AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_spmm_prepared: split SELL layouts (AFSAI_OPT_SELL_UNEVEN = 1) are not supported");
    DeviceInfo di;
    if ((rc = device_info(&di))) return rc;
    if (di.device != M->device)
        AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_spmm_prepared: matrix prepared on device %d, current device %d",
                   M->device, di.device);
    return spmm_sell(M->S, k, X, Y, di, (hipStream_t)stream);
}

int pcg_solve_prepared(afsai_matrix M, afsai_precond P, const double *b, double *x, double rtol, int32_t maxit,
                       void *stream, afsai_pcg_info *info) {
    clear_error();
    if (!M) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "pcg_solve_prepared: null matrix");
    if (!b || !x) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "pcg_solve_prepared: null b or x");
    if (!(rtol > 0.0) || maxit < 0)
        AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "pcg_solve_prepared: rtol = %g, maxit = %d", rtol, maxit);
    if (P && P->n != M->A.n)
        AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "pcg_solve_prepared: preconditioner has n = %d, A has n = %d", P->n, M->A.n);
    if (P && P->seg_row0.size() > 2)
        AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "pcg_solve_prepared: the preconditioner is for a batch");
    if (M->S.tail || M->S.srow0)
        AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "pcg_solve_prepared: split SELL layouts are not supported for A");
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc) return rc;
    if (di.device != M->device || (P && P->device != M->device))
        AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "pcg_solve_prepared: matrix prepared on device %d, current device %d",
                   M->device, di.device);
    return pcg_batch(&M->A, P, 1, nullptr, b, x, rtol, maxit, (hipStream_t)stream, info, &M->S);
}

int afsai_apply(afsai_precond P, const double *r, double *z, void *stream) {
    if (!P || !r || !z) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_apply: null argument");
    if (r == z) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_apply: r and z alias");
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    double *t = P->work;  // first n entries
    // products only (no dots): the whole matrix as one system
    BatchMaps bm;
    if ((rc = make_batch_maps(P->sg.nslices * kSlice, 1, nullptr, di, s, &bm))) return rc;
    bm.sell.nblocks = blocks_for_slices(P->sg.nslices, di);
    sell_spmv("spmv_G", P->sg, bm, r, t, nullptr, nullptr, nullptr, FIN_NONE, di, s);
    bm.sell.nblocks = blocks_for_slices(P->sgt.nslices, di);
    sell_spmv("spmv_GT", P->sgt, bm, t, z, nullptr, nullptr, nullptr, FIN_NONE, di, s);
    AFSAI_HIP_TRY(hipGetLastError());
    return AFSAI_OK;
}

}  // extern "C"

namespace afsai {

// Scratch of afsai_apply_noalloc: the intermediate t = G r of one application, for up to
// kNoAllocMaxRows rows (128 MiB of doubles, held by every GPU the library runs on until the
// process ends).  Host code never passes `scratch` itself to a kernel: each device's address
// of the array is taken once with hipGetSymbolAddress (with that device current) and kept.
constexpr int64_t kNoAllocMaxRows = (int64_t)1 << 24;
static __device__ __align__(256) double scratch[kNoAllocMaxRows];

// address of `scratch` on the current device, looked up on the first call there
static int scratch_ptr(double **out) {
    constexpr int kMaxDev = 64;
    static std::mutex mu;
    static double *ptr[kMaxDev] = {};
    int dev = -1;
    AFSAI_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDev) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_apply_noalloc: device %d", dev);
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        AFSAI_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) AFSAI_FAIL(AFSAI_ERR_HIP, "afsai_apply_noalloc: no device address for the scratch array");
        ptr[dev] = (double *)p;
    }
    *out = ptr[dev];
    return AFSAI_OK;
}

}  // namespace afsai

extern "C" {

int afsai_apply_noalloc(afsai_precond P, const double *r, double *z, void *stream) {
    if (!P || !r || !z) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_apply_noalloc: null argument");
    if (r == z) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_apply_noalloc: r and z alias");
    if ((int64_t)P->n > kNoAllocMaxRows)
        AFSAI_FAIL(AFSAI_ERR_TOO_LARGE, "afsai_apply_noalloc: n = %d exceeds the scratch limit of %lld rows", P->n,
                   (long long)kNoAllocMaxRows);
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc) return rc;
    double *t = nullptr;
    if ((rc = scratch_ptr(&t))) return rc;
    hipStream_t s = (hipStream_t)stream;
    // the products of afsai_apply, the whole matrix as one system (no device block maps)
    BatchMaps bm;
    bm.sell.nblocks = blocks_for_slices(P->sg.nslices, di);
    sell_spmv("spmv_G", P->sg, bm, r, t, nullptr, nullptr, nullptr, FIN_NONE, di, s);
    bm.sell.nblocks = blocks_for_slices(P->sgt.nslices, di);
    sell_spmv("spmv_GT", P->sgt, bm, t, z, nullptr, nullptr, nullptr, FIN_NONE, di, s);
    AFSAI_HIP_TRY(hipGetLastError());
    return AFSAI_OK;
}

int pcg_solve(const afsai_csr *A, afsai_precond P, const double *b, double *x, double rtol, int32_t maxit,
              void *stream, afsai_pcg_info *info) {
    clear_error();
    int rc = check_csr_arg(A, "pcg_solve");
    if (rc) return rc;
    if (!b || !x) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "pcg_solve: null b or x");
    if (!(rtol > 0.0) || maxit < 0) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "pcg_solve: rtol = %g, maxit = %d", rtol, maxit);
    if (P && P->n != A->n) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "pcg_solve: preconditioner has n = %d, A has n = %d", P->n, A->n);
    if (P && P->seg_row0.size() > 2)
        AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "pcg_solve: the preconditioner is for a batch; use pcg_solve_batched");
    return pcg_batch(A, P, 1, nullptr, b, x, rtol, maxit, (hipStream_t)stream, info);
}

int pcg_solve_batched(const afsai_csr *A, afsai_precond P, int32_t nsys, const int32_t *offsets, const double *b,
                      double *x, double rtol, int32_t maxit, void *stream, afsai_pcg_info *info) {
    clear_error();
    int rc = check_csr_arg(A, "pcg_solve_batched");
    if (rc) return rc;
    if (!b || !x || !offsets || nsys < 1) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "pcg_solve_batched: null argument or nsys < 1");
    if (!(rtol > 0.0) || maxit < 0)
        AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "pcg_solve_batched: rtol = %g, maxit = %d", rtol, maxit);
    if (offsets[0] != 0 || offsets[nsys] != A->n)
        AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "pcg_solve_batched: offsets must run from 0 to n = %d", A->n);
    for (int k = 0; k < nsys; ++k)
        if (offsets[k + 1] <= offsets[k])
            AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "pcg_solve_batched: system %d is empty or offsets decrease", k);
    if (P) {
        if (P->n != A->n) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "pcg_solve_batched: preconditioner has n = %d, A has n = %d", P->n, A->n);
        const bool same = (nsys == 1 && P->seg_row0.size() <= 2) ||
                          (P->seg_row0.size() == (size_t)nsys + 1 &&
                           std::equal(P->seg_row0.begin(), P->seg_row0.end(), offsets));
        if (!same) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "pcg_solve_batched: the preconditioner was set up for other systems");
    }
    return pcg_batch(A, P, nsys, offsets, b, x, rtol, maxit, (hipStream_t)stream, info);
}

}  // extern "C"
