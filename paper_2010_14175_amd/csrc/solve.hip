// Group-per-row CSR products and the PCG iteration (Sec. 3 "miniwarp" SpMV; Sec. 5.2 PCG).
//
// SpMV: a group of GS lanes (GS in {4, 8, 16, 32, 64}, chosen from the average row length like
// the paper's miniwarps, but sized for 64-lane wavefronts) owns one row; lanes stride through
// the row's entries with coalesced, non-temporal loads of the matrix and cached loads of x;
// the group reduces with cross-lane shuffles in a fixed order.  Each block owns one
// contiguous range of rows and blocks are renumbered so that every XCD streams one contiguous
// part of the matrix (its L2 then holds the x entries its rows share).
//
// PCG: all scalars (rho, alpha, beta, ||r||) live on the device.  Dot products are fused into
// the kernel that produces one of their operands, which stores one partial sum per block; a
// one-block kernel then adds the partials in block order (results do not depend on
// scheduling) and updates the scalars.  (A last-block-done reduction inside the producing
// kernel needs a device-scope release per block, which on this 8-XCD part writes back the
// L2 and cost more than the extra launch.)  A device flag ends the iteration: kernels that
// see it return at once, so the host enqueues chunks of iterations and reads the flag once
// per chunk, one chunk behind.
#include <cmath>
#include <vector>

#include "handle.hpp"

namespace afsai {

constexpr int kThreads = 256;
constexpr int kFusedMaxRows = 200000;  // automatic PCG form: fused products below this size

enum : int { FIN_NONE = 0, FIN_ALPHA = 1, FIN_BETA = 2, FIN_RHO0 = 3, FIN_INIT = 4, FIN_UPDATE = 5, FIN_RESID = 6 };
enum : int { DONE_NO = 0, DONE_CONVERGED = 1, DONE_NOT_SPD = 2, DONE_MAXIT = 3, DONE_ZERO_RHS = 4 };

struct PcgScalars {
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

// thread 0 stores this block's partial sums, slot k at partials[k * gridDim.x + idx], idx being
// the index of the block's range of rows (so the sums are added in row order)
__device__ __forceinline__ void store_partials(double *partials, int slots, const double *mine, int idx) {
    if (threadIdx.x == 0)
        for (int k = 0; k < slots; ++k) partials[(size_t)k * gridDim.x + idx] = mine[k];
}

// One block: sums the partials of the previous kernel in block order and updates the scalars.
__global__ __launch_bounds__(kThreads) void k_finalize(const double *__restrict__ partials, int nparts, int fin,
                                                       PcgScalars *sc) {
    if ((fin == FIN_ALPHA || fin == FIN_BETA || fin == FIN_UPDATE || fin == FIN_RHO0) && sc->done) return;
    __shared__ double sh[kThreads / 64];
    const int slots = (fin == FIN_INIT) ? 2 : 1;
    double tot[2] = {0.0, 0.0};
    const int per = (nparts + kThreads - 1) / kThreads;
    const int lo = threadIdx.x * per, hi = min(nparts, lo + per);
    for (int k = 0; k < slots; ++k) {
        double v = 0.0;
        for (int j = lo; j < hi; ++j) v += partials[(size_t)k * nparts + j];
        tot[k] = block_sum(v, sh);
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
// CSR SpMV, one group of GS lanes per row; optional fused dot y.w with a PCG finalisation
// ---------------------------------------------------------------------------------------
template <int GS, int U, typename VT, bool DOT>
__global__ __launch_bounds__(kThreads) void k_spmv(int n, const int32_t *__restrict__ rp,
                                                    const int32_t *__restrict__ ci,
                                                    const VT *__restrict__ val,
                                                    const double *__restrict__ x,
                                                    double *__restrict__ y,
                                                    const double *__restrict__ w,
                                                    double *__restrict__ partials,
                                                    PcgScalars *sc, int fin, int nxcd) {
    if (sc && sc->done) return;
    __shared__ double sh[kThreads / 64];
    const int lb = xcd_block(blockIdx.x, gridDim.x, nxcd);
    const int64_t per = ((int64_t)n + gridDim.x - 1) / gridDim.x;
    const int r0 = (int)min<int64_t>(n, per * lb), r1 = (int)min<int64_t>(n, per * (lb + 1));
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

// SELL-64 product: one wavefront per slice of 64 rows, one lane per row; entry k of the 64
// rows is one contiguous wave load.  Optional fused dot y.w with a PCG finalisation.
template <int U, typename VT, bool DOT>
__global__ __launch_bounds__(kThreads) void k_sell_spmv(int n, int nslices, const uint32_t *__restrict__ sptr,
                                                         const int32_t *__restrict__ perm,
                                                         const int32_t *__restrict__ rowmap,
                                                         const uint64_t *__restrict__ init,
                                                         const int32_t *__restrict__ col,
                                                         const VT *__restrict__ val,
                                                         const double *__restrict__ x, double *__restrict__ y,
                                                         const double *__restrict__ w,
                                                         double *__restrict__ partials, PcgScalars *sc, int fin,
                                                         int nxcd) {
    if (sc && sc->done) return;
    __shared__ double sh[kThreads / 64];
    const int lb = xcd_block(blockIdx.x, gridDim.x, nxcd);
    const int64_t per = ((int64_t)nslices + gridDim.x - 1) / gridDim.x;
    const int s0 = (int)min<int64_t>(nslices, per * lb), s1 = (int)min<int64_t>(nslices, per * (lb + 1));
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double part = 0.0;
    for (int sl = s0 + wv; sl < s1; sl += kThreads / 64) {
        int r = sl * kSlice + lane;
        if (perm) r = perm[r];
        const bool valid = r >= 0 && r < n;
        const int ro = (valid && rowmap) ? rowmap[r] : r;
        const uint32_t c0 = sptr[sl];
        const int width = (int)(sptr[sl + 1] - c0);
        const int64_t base = (int64_t)c0 * kSlice + lane;
        // rows split between the two layouts continue the sum their tail started
        double acc = (init && valid && ((init[sl] >> lane) & 1)) ? y[ro] : 0.0;
        for (int k0 = 0; k0 < width; k0 += U) {
            int c[U];
            VT v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                c[u] = -1;
                v[u] = VT(0);
                if (k0 + u < width) {
                    const int64_t d = base + (int64_t)(k0 + u) * kSlice;
                    c[u] = __builtin_nontemporal_load(&col[d]);
                    v[u] = __builtin_nontemporal_load(&val[d]);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (c[u] >= 0) acc = fma((double)v[u], x[c[u]], acc);
        }
        if (valid) {
            y[ro] = acc;
            if (DOT) part = fma(acc, w[ro], part);
        }
    }
    if (DOT) {
        const double bs = block_sum(part, sh);
        store_partials(partials, 1, &bs, lb);
    }
}

// Fused PCG products (SELL-64, one lane per row).  The vector being multiplied is formed on
// the fly from two others with the same fma the separate update kernel would use, so the
// result is identical to update-then-multiply; the owner lane of each row also stores the
// updated entry.
//   FUSE_AP:  p_new = z + beta p_old (p_new = z on the first iteration); q = A p_new;
//             partial sums of p_new.q
//   FUSE_GR:  r_new = r_old - alpha q; x += alpha p_new; t = G r_new; partial sums of r_new.r_new
enum : int { FUSE_AP = 1, FUSE_GR = 2 };

template <int U, typename VT, int MODE>
__global__ __launch_bounds__(kThreads) void k_sell_fused(int n, int nslices, const uint32_t *__restrict__ sptr,
                                                          const int32_t *__restrict__ perm,
                                                          const int32_t *__restrict__ col,
                                                          const VT *__restrict__ val,
                                                          const double *__restrict__ va,   // z | r_old
                                                          const double *__restrict__ vb,   // p_old | q
                                                          double *__restrict__ own_out,    // p_new | r_new
                                                          double *__restrict__ x,          // - | x
                                                          const double *__restrict__ pn,   // - | p_new
                                                          double *__restrict__ y,          // q | t
                                                          double *__restrict__ partials,
                                                          const PcgScalars *sc, int first, int nxcd) {
    if (sc->done) return;
    __shared__ double sh[kThreads / 64];
    const double alpha = sc->alpha;
    const double coef = (MODE == FUSE_AP) ? sc->beta : -alpha;
    const int lb = xcd_block(blockIdx.x, gridDim.x, nxcd);
    const int64_t per = ((int64_t)nslices + gridDim.x - 1) / gridDim.x;
    const int s0 = (int)min<int64_t>(nslices, per * lb), s1 = (int)min<int64_t>(nslices, per * (lb + 1));
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double part = 0.0;
    for (int sl = s0 + wv; sl < s1; sl += kThreads / 64) {
        int r = sl * kSlice + lane;
        if (perm) r = perm[r];
        const uint32_t c0 = sptr[sl];
        const int width = (int)(sptr[sl + 1] - c0);
        const int64_t base = (int64_t)c0 * kSlice + lane;
        double acc = 0.0;
        for (int k0 = 0; k0 < width; k0 += U) {
            int c[U];
            VT v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                c[u] = -1;
                v[u] = VT(0);
                if (k0 + u < width) {
                    const int64_t d = base + (int64_t)(k0 + u) * kSlice;
                    c[u] = __builtin_nontemporal_load(&col[d]);
                    v[u] = __builtin_nontemporal_load(&val[d]);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (c[u] >= 0) {
                    const double xv = (MODE == FUSE_AP && first) ? va[c[u]] : fma(coef, vb[c[u]], va[c[u]]);
                    acc = fma((double)v[u], xv, acc);
                }
        }
        if (r >= 0 && r < n) {
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
    store_partials(partials, 1, &bs, lb);
}

// r = b - q ; partials of b.b and r.r ; finalisation checks ||b|| = 0 and ||r0|| <= tol
__global__ __launch_bounds__(kThreads) void k_init_residual(int n, const double *__restrict__ b,
                                                             const double *__restrict__ q,
                                                             double *__restrict__ r,
                                                             double *__restrict__ partials) {
    __shared__ double sh[kThreads / 64];
    const int64_t per = ((int64_t)n + gridDim.x - 1) / gridDim.x;
    const int i0 = (int)min<int64_t>(n, per * blockIdx.x), i1 = (int)min<int64_t>(n, per * (blockIdx.x + 1));
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
    store_partials(partials, 2, mine, blockIdx.x);
}

// x += alpha p ; r -= alpha q ; ||r||^2 ; convergence test; (plain CG) beta = rr'/rr
__global__ __launch_bounds__(kThreads) void k_update_xr(int n, double *__restrict__ x,
                                                         double *__restrict__ r,
                                                         const double *__restrict__ p,
                                                         const double *__restrict__ q,
                                                         double *__restrict__ partials,
                                                         PcgScalars *sc, int nxcd) {
    if (sc->done) return;
    __shared__ double sh[kThreads / 64];
    const double alpha = sc->alpha;
    const int lb = xcd_block(blockIdx.x, gridDim.x, nxcd);
    const int64_t per = ((int64_t)n + gridDim.x - 1) / gridDim.x;
    const int i0 = (int)min<int64_t>(n, per * lb), i1 = (int)min<int64_t>(n, per * (lb + 1));
    double pr = 0.0;
    for (int i = i0 + threadIdx.x; i < i1; i += kThreads) {
        x[i] = fma(alpha, p[i], x[i]);
        const double ri = fma(-alpha, q[i], r[i]);
        r[i] = ri;
        pr = fma(ri, ri, pr);
    }
    const double bs = block_sum(pr, sh);
    store_partials(partials, 1, &bs, lb);
}

// p = z + beta p   (first = 1: p = z)
__global__ __launch_bounds__(kThreads) void k_update_p(int n, double *__restrict__ p,
                                                        const double *__restrict__ z,
                                                        const PcgScalars *sc, int first, int nxcd) {
    if (sc->done) return;
    const double beta = first ? 0.0 : sc->beta;
    const int lb = xcd_block(blockIdx.x, gridDim.x, nxcd);
    const int64_t per = ((int64_t)n + gridDim.x - 1) / gridDim.x;
    const int i0 = (int)min<int64_t>(n, per * lb), i1 = (int)min<int64_t>(n, per * (lb + 1));
    if (first)
        for (int i = i0 + threadIdx.x; i < i1; i += kThreads) p[i] = z[i];
    else
        for (int i = i0 + threadIdx.x; i < i1; i += kThreads) p[i] = fma(beta, p[i], z[i]);
}

__global__ void k_zero(int n, double *__restrict__ v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) v[i] = 0.0;
}

__global__ void k_set_scalars(PcgScalars *sc, double rtol, int maxit, int plain) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        PcgScalars s{};
        s.rtol = rtol;
        s.maxit = maxit;
        s.plain = plain;
        *sc = s;
    }
}

// true residual partials: ||b - Ax||^2 with q = A x
__global__ __launch_bounds__(kThreads) void k_resid_norm(int n, const double *__restrict__ b,
                                                          const double *__restrict__ q,
                                                          double *__restrict__ partials) {
    __shared__ double sh[kThreads / 64];
    const int64_t per = ((int64_t)n + gridDim.x - 1) / gridDim.x;
    const int i0 = (int)min<int64_t>(n, per * blockIdx.x), i1 = (int)min<int64_t>(n, per * (blockIdx.x + 1));
    double pr = 0.0;
    for (int i = i0 + threadIdx.x; i < i1; i += kThreads) {
        const double d = b[i] - q[i];
        pr = fma(d, d, pr);
    }
    const double bs = block_sum(pr, sh);
    store_partials(partials, 1, &bs, blockIdx.x);
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

struct Csr {
    int n = 0;
    int64_t nnz = 0;
    const int32_t *rp = nullptr, *ci = nullptr;
    const void *val = nullptr;
    bool f32 = false;
};

template <int GS, int U, typename VT>
static void launch_spmv_t(const Csr &A, const double *x, double *y, const double *w, double *partials,
                          PcgScalars *sc, int fin, int nb, int nxcd, hipStream_t s) {
    if (w)
        hipLaunchKernelGGL((k_spmv<GS, U, VT, true>), dim3(nb), dim3(kThreads), 0, s, A.n, A.rp, A.ci,
                           (const VT *)A.val, x, y, w, partials, sc, fin, nxcd);
    else
        hipLaunchKernelGGL((k_spmv<GS, U, VT, false>), dim3(nb), dim3(kThreads), 0, s, A.n, A.rp, A.ci,
                           (const VT *)A.val, x, y, w, partials, sc, fin, nxcd);
}

template <int GS, typename VT>
static void launch_spmv_u(const Csr &A, int un, const double *x, double *y, const double *w, double *partials,
                          PcgScalars *sc, int fin, int nb, int nxcd, hipStream_t s) {
    switch (un) {
        case 1: launch_spmv_t<GS, 1, VT>(A, x, y, w, partials, sc, fin, nb, nxcd, s); break;
        case 2: launch_spmv_t<GS, 2, VT>(A, x, y, w, partials, sc, fin, nb, nxcd, s); break;
        case 4: launch_spmv_t<GS, 4, VT>(A, x, y, w, partials, sc, fin, nb, nxcd, s); break;
        default: launch_spmv_t<GS, 8, VT>(A, x, y, w, partials, sc, fin, nb, nxcd, s); break;
    }
}

template <typename VT>
static void launch_spmv_v(const Csr &A, int gs, int un, const double *x, double *y, const double *w,
                          double *partials, PcgScalars *sc, int fin, int nb, int nxcd, hipStream_t s) {
    switch (gs) {
        case 4: launch_spmv_u<4, VT>(A, un, x, y, w, partials, sc, fin, nb, nxcd, s); break;
        case 8: launch_spmv_u<8, VT>(A, un, x, y, w, partials, sc, fin, nb, nxcd, s); break;
        case 16: launch_spmv_u<16, VT>(A, un, x, y, w, partials, sc, fin, nb, nxcd, s); break;
        case 32: launch_spmv_u<32, VT>(A, un, x, y, w, partials, sc, fin, nb, nxcd, s); break;
        default: launch_spmv_u<64, VT>(A, un, x, y, w, partials, sc, fin, nb, nxcd, s); break;
    }
}

// y = A x (optionally fused dot y.w finalised into sc)
static void spmv(const char *name, const Csr &A, const double *x, double *y, const double *w,
                 double *partials, PcgScalars *sc, int fin, const DeviceInfo &di, hipStream_t s) {
    const double avg = A.n ? (double)A.nnz / A.n : 0.0;
    int gs, un;
    spmv_shape(avg, &gs, &un);
    const int nb = blocks_for_rows(A.n, gs, di);
    {
        ProfScope ps(name, s);
        if (A.f32)
            launch_spmv_v<float>(A, gs, un, x, y, w, partials, sc, fin, nb, di.num_xcds, s);
        else
            launch_spmv_v<double>(A, gs, un, x, y, w, partials, sc, fin, nb, di.num_xcds, s);
    }
    if (w) hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, s, partials, nb, fin, sc);
}

template <int U, typename VT>
static void launch_sell_t(const Sell &S, const double *x, double *y, const double *w, double *partials,
                          PcgScalars *sc, int fin, int nb, int nxcd, hipStream_t s) {
    if (w)
        hipLaunchKernelGGL((k_sell_spmv<U, VT, true>), dim3(nb), dim3(kThreads), 0, s, S.n, S.nslices, S.sptr,
                           S.perm, S.rowmap, S.init, S.col, (const VT *)S.val, x, y, w, partials, sc, fin, nxcd);
    else
        hipLaunchKernelGGL((k_sell_spmv<U, VT, false>), dim3(nb), dim3(kThreads), 0, s, S.n, S.nslices, S.sptr,
                           S.perm, S.rowmap, S.init, S.col, (const VT *)S.val, x, y, w, partials, sc, fin, nxcd);
}

template <typename VT>
static void launch_sell_v(const Sell &S, int un, const double *x, double *y, const double *w, double *partials,
                          PcgScalars *sc, int fin, int nb, int nxcd, hipStream_t s) {
    switch (un) {
        case 1: launch_sell_t<1, VT>(S, x, y, w, partials, sc, fin, nb, nxcd, s); break;
        case 2: launch_sell_t<2, VT>(S, x, y, w, partials, sc, fin, nb, nxcd, s); break;
        case 4: launch_sell_t<4, VT>(S, x, y, w, partials, sc, fin, nb, nxcd, s); break;
        default: launch_sell_t<8, VT>(S, x, y, w, partials, sc, fin, nb, nxcd, s); break;
    }
}

static int sell_blocks(const Sell &S, const DeviceInfo &di) {
    int64_t nb = ((int64_t)S.nslices + kThreads / 64 - 1) / (kThreads / 64);
    const int64_t cap = (int64_t)di.num_cus * 16;
    if (nb > cap) nb = cap;
    if (nb < 1) nb = 1;
    return (int)nb;
}

// y = S x for a SELL-64 matrix (optionally fused dot y.w finalised into sc); a split layout's
// tail is multiplied first
static void sell_spmv(const char *name, const Sell &S, const double *x, double *y, const double *w,
                      double *partials, PcgScalars *sc, int fin, const DeviceInfo &di, hipStream_t s) {
    int un = option(AFSAI_OPT_SPMV_UNROLL) > 0 ? (int)option(AFSAI_OPT_SPMV_UNROLL) : 8;
    if (S.tail) {
        const Sell &T = *S.tail;
        const int nbt = sell_blocks(T, di);
        ProfScope ps("sell_tail", s);
        if (T.f32)
            launch_sell_v<float>(T, un, x, y, nullptr, nullptr, sc, FIN_NONE, nbt, di.num_xcds, s);
        else
            launch_sell_v<double>(T, un, x, y, nullptr, nullptr, sc, FIN_NONE, nbt, di.num_xcds, s);
    }
    const int64_t nb = sell_blocks(S, di);
    {
        ProfScope ps(name, s);
        if (S.f32)
            launch_sell_v<float>(S, un, x, y, w, partials, sc, fin, (int)nb, di.num_xcds, s);
        else
            launch_sell_v<double>(S, un, x, y, w, partials, sc, fin, (int)nb, di.num_xcds, s);
    }
    if (w) hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, s, partials, (int)nb, fin, sc);
}

template <int U, typename VT, int MODE>
static void launch_fused_t(const Sell &S, const double *va, const double *vb, double *own, double *x,
                           const double *pn, double *y, double *partials, PcgScalars *sc, int first, int nb, int nxcd,
                           hipStream_t s) {
    hipLaunchKernelGGL((k_sell_fused<U, VT, MODE>), dim3(nb), dim3(kThreads), 0, s, S.n, S.nslices, S.sptr, S.perm,
                       S.col, (const VT *)S.val, va, vb, own, x, pn, y, partials, sc, first, nxcd);
}

template <typename VT, int MODE>
static void launch_fused_v(const Sell &S, int un, const double *va, const double *vb, double *own, double *x,
                           const double *pn, double *y, double *partials, PcgScalars *sc, int first, int nb, int nxcd,
                           hipStream_t s) {
    switch (un) {
        case 1: launch_fused_t<1, VT, MODE>(S, va, vb, own, x, pn, y, partials, sc, first, nb, nxcd, s); break;
        case 2: launch_fused_t<2, VT, MODE>(S, va, vb, own, x, pn, y, partials, sc, first, nb, nxcd, s); break;
        case 4: launch_fused_t<4, VT, MODE>(S, va, vb, own, x, pn, y, partials, sc, first, nb, nxcd, s); break;
        default: launch_fused_t<8, VT, MODE>(S, va, vb, own, x, pn, y, partials, sc, first, nb, nxcd, s); break;
    }
}

// fused product followed by the finalisation of its dot
template <int MODE>
static void sell_fused(const char *name, const Sell &S, const double *va, const double *vb, double *own, double *x,
                       const double *pn, double *y, double *partials, PcgScalars *sc, int first, int fin,
                       const DeviceInfo &di, hipStream_t s) {
    const int un = option(AFSAI_OPT_SPMV_UNROLL) > 0 ? (int)option(AFSAI_OPT_SPMV_UNROLL) : 8;
    int64_t nb = ((int64_t)S.nslices + kThreads / 64 - 1) / (kThreads / 64);
    const int64_t cap = (int64_t)di.num_cus * 16;
    if (nb > cap) nb = cap;
    if (nb < 1) nb = 1;
    {
        ProfScope ps(name, s);
        if (S.f32)
            launch_fused_v<float, MODE>(S, un, va, vb, own, x, pn, y, partials, sc, first, (int)nb, di.num_xcds, s);
        else
            launch_fused_v<double, MODE>(S, un, va, vb, own, x, pn, y, partials, sc, first, (int)nb, di.num_xcds, s);
    }
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, s, partials, (int)nb, fin, sc);
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

// partial-sum scratch: 2 slots x max blocks
static size_t partial_elems(const DeviceInfo &di) { return (size_t)2 * di.num_cus * 16 + 64; }

// work vectors of the solver: r, r', z, p, p', q, t
constexpr int kWorkVectors = 7;

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

int afsai_apply(afsai_precond P, const double *r, double *z, void *stream) {
    if (!P || !r || !z) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_apply: null argument");
    if (r == z) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_apply: r and z alias");
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    double *t = P->work;  // first n entries
    sell_spmv("spmv_G", P->sg, r, t, nullptr, nullptr, nullptr, FIN_NONE, di, s);
    sell_spmv("spmv_GT", P->sgt, t, z, nullptr, nullptr, nullptr, FIN_NONE, di, s);
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
    DeviceInfo di;
    if ((rc = device_info(&di))) return rc;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t t0, t1;
    AFSAI_HIP_TRY(hipEventCreate(&t0));
    AFSAI_HIP_TRY(hipEventCreate(&t1));
    AFSAI_HIP_TRY(hipEventRecord(t0, s));

    const int n = A->n;
    const size_t np = partial_elems(di);
    // workspace: r, r', z, p, p', q, t (n each), partials, scalars
    const size_t need = (size_t)kWorkVectors * n + np + 16;
    DevBuf own;
    double *ws = nullptr;
    if (P && P->work_elems >= need) {
        ws = P->work;
    } else {
        if ((rc = dalloc(own, need * sizeof(double), s))) return rc;
        ws = own.as<double>();
    }
    double *r = ws, *r2 = ws + n, *z = ws + 2 * (size_t)n, *p = ws + 3 * (size_t)n, *p2 = ws + 4 * (size_t)n;
    double *q = ws + 5 * (size_t)n, *t = ws + 6 * (size_t)n;
    double *partials = ws + kWorkVectors * (size_t)n;
    PcgScalars *sc = (PcgScalars *)(partials + np);
    // pinned host copies of the scalars, one pair per thread for the life of the process
    static thread_local PcgScalars *hsc = nullptr;
    if (!hsc) AFSAI_HIP_TRY(hipHostMalloc(&hsc, 2 * sizeof(PcgScalars), hipHostMallocDefault));

    // A in the SELL-64 layout for the iteration (one conversion per solve)
    Sell As;
    const bool use_sell = option(AFSAI_OPT_PCG_CSR_A) == 0;
    if (use_sell) {
        ProfScope ps("sell_A", s);
        if ((rc = sell_from_csr(n, A->nnz, A->row_ptr, A->col_idx, A->val, false, false, &As, di, s))) return rc;
    }
    struct SellGuard {
        Sell *S;
        hipStream_t s;
        ~SellGuard() {
            (void)hipStreamSynchronize(s);
            sell_free(S);
        }
    } sell_guard{&As, s};
    const Csr Am = csr_of(A);
    auto spmv_A = [&](const char *name, const double *xin, double *yout, const double *w, int fin, PcgScalars *scp) {
        if (use_sell) sell_spmv(name, As, xin, yout, w, w ? partials : nullptr, scp, fin, di, s);
        else spmv(name, Am, xin, yout, w, w ? partials : nullptr, scp, fin, di, s);
    };

    const int nbv = blocks_for_vec(n, di);
    const int plain = P ? 0 : 1;
    hipLaunchKernelGGL(k_set_scalars, dim3(1), dim3(64), 0, s, sc, rtol, maxit, plain);
    // r0 = b - A x0
    spmv_A("spmv_A", x, q, nullptr, FIN_NONE, nullptr);
    hipLaunchKernelGGL(k_init_residual, dim3(nbv), dim3(kThreads), 0, s, n, b, q, r, partials);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, s, partials, nbv, (int)FIN_INIT, sc);
    // z0 = M^-1 r0, rho0 = r0.z0, p0 = z0
    const double *zz = z;
    if (P) {
        sell_spmv("spmv_G", P->sg, r, t, nullptr, nullptr, sc, FIN_NONE, di, s);
        sell_spmv("spmv_GT_dot", P->sgt, t, z, r, partials, sc, FIN_RHO0, di, s);
    } else {
        zz = r;
    }
    // fused iteration (preconditioned, A in SELL-64): p and r are double-buffered because the
    // products read neighbours' old entries while owners store the new ones
    // fused products where launches dominate (small systems), separate updates where the
    // fused products' second gather costs more than the update kernels
    const int64_t form = option(AFSAI_OPT_PCG_FORM);
    const bool want_fused = form == 2 || (form == 0 && n < kFusedMaxRows);
    const bool fused = P && use_sell && want_fused && !As.tail && !P->sg.tail;
    if (!fused) hipLaunchKernelGGL(k_update_p, dim3(nbv), dim3(kThreads), 0, s, n, p, zz, sc, 1, di.num_xcds);
    int iter_no = 0;  // iterations enqueued so far

    // timer marks: after the update of each iteration (launches past the last iteration that
    // ran are dropped from the kernel timer at the end)
    std::vector<int> marks;
    const int mark0 = prof_mark();
    auto enqueue_iteration = [&]() {
        if (fused) {
            const bool odd = (iter_no & 1) == 0;  // iteration 1, 3, ...: p -> p2, r -> r2
            double *p_old = odd ? p : p2, *p_new = odd ? p2 : p;
            double *r_old = odd ? r : r2, *r_new = odd ? r2 : r;
            sell_fused<FUSE_AP>("spmv_A_dot", As, z, p_old, p_new, nullptr, nullptr, q, partials, sc,
                                iter_no == 0 ? 1 : 0, FIN_ALPHA, di, s);
            sell_fused<FUSE_GR>("spmv_G_upd", P->sg, r_old, q, r_new, x, p_new, t, partials, sc, 0, FIN_UPDATE,
                                di, s);
            marks.push_back(prof_mark());
            sell_spmv("spmv_GT_dot", P->sgt, t, z, r_new, partials, sc, FIN_BETA, di, s);
            ++iter_no;
            return;
        }
        spmv_A("spmv_A_dot", p, q, p, FIN_ALPHA, sc);
        {
            ProfScope ps("update_xr", s);
            hipLaunchKernelGGL(k_update_xr, dim3(nbv), dim3(kThreads), 0, s, n, x, r, p, q, partials, sc, di.num_xcds);
        }
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, s, partials, nbv, (int)FIN_UPDATE, sc);
        marks.push_back(prof_mark());
        if (P) {
            sell_spmv("spmv_G", P->sg, r, t, nullptr, nullptr, sc, FIN_NONE, di, s);
            sell_spmv("spmv_GT_dot", P->sgt, t, z, r, partials, sc, FIN_BETA, di, s);
        }
        {
            ProfScope ps("update_p", s);
            hipLaunchKernelGGL(k_update_p, dim3(nbv), dim3(kThreads), 0, s, n, p, zz, sc, 0, di.num_xcds);
        }
        ++iter_no;
    };

    // Chunks of iterations; the state after chunk c is read while chunk c+1 is already queued.
    // Chunk sizes follow the observed residual reduction rate so that few iterations are
    // queued past convergence (those return at once on the device flag).
    hipEvent_t ev[2];
    AFSAI_HIP_TRY(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    AFSAI_HIP_TRY(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
    AFSAI_HIP_TRY(hipMemcpyAsync(&hsc[1], sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, s));
    AFSAI_HIP_TRY(hipEventRecord(ev[1], s));
    int enqueued = 0, c = 0, chunk = 4;
    bool finished = false, have_prev = false;
    int prev_it = 0;
    double prev_rr = 0.0, rate = 0.0;  // log of the per-iteration reduction of ||r||^2
    while (!finished) {
        int todo = chunk;
        if (rate < 0.0 && have_prev) {
            const double tol2 = hsc[(c + 1) & 1].tol * hsc[(c + 1) & 1].tol;
            const double need_it = std::ceil(std::log(tol2 / prev_rr) / rate);
            int rem = (int)need_it - (enqueued - prev_it) + 1;
            todo = rem < 1 ? 1 : (rem > 64 ? 64 : rem);
        }
        if (todo > maxit - enqueued) todo = maxit - enqueued;
        for (int k = 0; k < todo; ++k) enqueue_iteration();
        enqueued += todo;
        AFSAI_HIP_TRY(hipMemcpyAsync(&hsc[c & 1], sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, s));
        AFSAI_HIP_TRY(hipEventRecord(ev[c & 1], s));
        // state after the previous chunk
        AFSAI_HIP_TRY(hipEventSynchronize(ev[(c + 1) & 1]));
        const PcgScalars &st = hsc[(c + 1) & 1];
        if (st.done != DONE_NO) finished = true;
        else {
            if (have_prev && st.it > prev_it && st.rr > 0.0 && prev_rr > 0.0) {
                const double rt = std::log(st.rr / prev_rr) / (st.it - prev_it);
                if (rt < 0.0) rate = rt;
            }
            if (st.rr > 0.0) {
                prev_rr = st.rr;
                prev_it = st.it;
                have_prev = true;
            }
        }
        if (todo == 0) {
            AFSAI_HIP_TRY(hipEventSynchronize(ev[c & 1]));
            finished = true;
        }
        ++c;
        if (chunk < 64) chunk *= 2;
    }
    AFSAI_HIP_TRY(hipStreamSynchronize(s));
    PcgScalars fin_s;
    AFSAI_HIP_TRY(hipMemcpy(&fin_s, sc, sizeof(PcgScalars), hipMemcpyDeviceToHost));
    {
        const int keep_to = fin_s.it >= 1 && fin_s.it <= (int)marks.size() ? marks[fin_s.it - 1] : mark0;
        prof_drop(keep_to, prof_mark());
    }

    int status = AFSAI_OK;
    if (fin_s.done == DONE_ZERO_RHS) {
        hipLaunchKernelGGL(k_zero, dim3(nbv), dim3(kThreads), 0, s, n, x);
    }
    double true_rr = 0.0;
    if (fin_s.done != DONE_ZERO_RHS) {
        // true residual ||b - A x||
        spmv_A("spmv_A", x, q, nullptr, FIN_NONE, nullptr);
        hipLaunchKernelGGL(k_resid_norm, dim3(nbv), dim3(kThreads), 0, s, n, b, q, partials);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, s, partials, nbv, (int)FIN_RESID, sc);
        AFSAI_HIP_TRY(hipMemcpyAsync(&hsc[0], sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, s));
        AFSAI_HIP_TRY(hipStreamSynchronize(s));
        true_rr = hsc[0].resid;
    }
    AFSAI_HIP_TRY(hipEventRecord(t1, s));
    AFSAI_HIP_TRY(hipStreamSynchronize(s));
    AFSAI_HIP_TRY(hipGetLastError());
    float ms = 0.f;
    AFSAI_HIP_TRY(hipEventElapsedTime(&ms, t0, t1));
    prof_flush();
    if (fin_s.done == DONE_NOT_SPD) {
        set_error("pcg_solve: p.Ap <= 0 at iteration %d (matrix or preconditioner not SPD)", fin_s.it + 1);
        status = AFSAI_ERR_NOT_SPD;
    } else if (fin_s.done == DONE_MAXIT || (fin_s.done == DONE_NO && maxit == 0)) {
        set_error("pcg_solve: not converged in %d iterations", fin_s.it);
        status = AFSAI_ERR_NOT_CONVERGED;
    }
    if (info) {
        const double nb = sqrt(fin_s.bb);
        info->iters = fin_s.it;
        info->converged = (fin_s.done == DONE_CONVERGED || fin_s.done == DONE_ZERO_RHS) ? 1 : 0;
        info->relres = nb > 0 ? sqrt(fin_s.rr) / nb : 0.0;
        info->true_relres = nb > 0 ? sqrt(true_rr) / nb : 0.0;
        info->ms = ms;
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    return status;
}

}  // extern "C"
