// The per-row adaptive FSAI setup (Sec. 2) in inverse-factor form: each row keeps W = L_o^-1,
// the inverse of the Cholesky factor of A[P_o,P_o] over its off-diagonal positions, instead of
// L itself.  Row i of G is the last row of L^-1 for the pattern with i last:
//
//     L = [ L_o   0  ]      L^-1 = [ W                 0     ]      l_i = W a_i,
//         [ l_i^T d_i]             [ -l_i^T W / d_i    1/d_i ]      d_i^2 = a_ii - |l_i|^2,
//
// so g = ( -(W^T l_i)/d_i , 1/d_i ), psi = d_i^2 (the Schur complement of eq. diagScal2's
// denominator; eq. DensSys with the scaling of eq. diagScal).  A new position u with row
// a_u = A[P_o,u] extends W by the row ( -(W^T l_u)/d_u , 1/d_u ) with l_u = W a_u and
// d_u^2 = a_uu - |l_u|^2 (bordering).  Both products are dense triangular matrix-vector
// products over all lanes at once, with W in LDS (row-major packed: the entries one lane
// reads for a fixed row or a fixed column fall in distinct banks) and the vector entries read
// as LDS broadcasts; no step waits on the previous one, unlike a forward substitution.  l_i
// grows by one entry per new row (a dot product of the new W row with a_i), and psi by one
// subtraction, so row i needs no product of its own.
//
// Rows per wavefront: GS lanes own one row (lane t = pattern position t), 64 / GS rows share a
// wavefront, each group with its own LDS table, factor and vectors; reductions stay inside a
// group (DPP quad and mirror moves, a swizzle across 16 lanes, readlane across 32).  Control
// flow is uniform inside a group; groups of a wavefront run their growth steps together.
//
// Per growth step of a row:
//  1. product over the member rows r of P (their entries left of column i, looked up in the
//     row's LDS hash table once, when r joined; the slots are kept in registers): every
//     non-member column c accumulates v_c += a_rc g_r = (A g)_c, the Kaporin gradient of eq.
//     grapsi up to a positive factor (LDS FP64 atomics);
//  2. selection over the compact list of table entries: s rounds of "largest |v|, ties within
//     the relative band tau go to the smallest column" (candidates with |v| <= 2^-40 max|v|
//     are not eligible; none eligible stops the row);
//  3. gather of the new rows (their entries up to column i): entries at member columns give
//     a_u, the entry at column i gives a_iu, entries left of i are entered in the table;
//  4. the new rows of W (blocks of NB: both products for the block at once, then the small
//     coupling inside the block row by row), l_i's new entries and psi;
//  5. g = -(W^T l_i)/d_i, the exit test psi/psi_0 <= eps (eq. exit_crit).
#pragma once

#include <type_traits>

#include "common.hpp"
#include "rows.hpp"

#pragma clang fp contract(off)

namespace afsai {
namespace wform {

constexpr uint32_t kEmptyKey = 0xFFFFFFFFu;
constexpr uint32_t kMember = 0x80000000u;  // key bit 31: column is a member; bits 24..30: its position
constexpr uint32_t kColBits = 0x00FFFFFFu;
// member rows whose entries one product round loads together (16 loads per lane)
__host__ __device__ constexpr int qb_of(int gs) { return 4; }
constexpr int kPU = 8;  // unrolling of the two products with W

__host__ __device__ constexpr int tri_w(int t) { return (t * (t + 1)) / 2; }
__host__ __device__ constexpr int al16(int b) { return (b + 15) & ~15; }

// slots per lane per member row (two 16-bit slots per register): GS * SPW entries left of
// column i per member row at most
__host__ __device__ constexpr int spw_of(int gs) { return gs == 64 ? 2 : (gs == 8 ? 2 : 4); }

// LDS layout of one row group (bytes): table keys; gradients, whose array also holds, from
// the end of the selection to the next product pass, the selected columns with their row
// extents (at its end) and the gathered rows and W-product vectors (from its start, unless
// they do not fit beside the former); the member records of the product pass (groups of
// fewer than 64 lanes; 64 lanes broadcast them from registers); and W, sized at launch by the
// largest pattern: rows 0..mm-2, row t with t + 1 entries.
template <int GS, int MMAX, int CAP, int NB>
struct Layout {
    static constexpr int SPW = spw_of(GS);
    static constexpr int LROW = GS * SPW;
    static constexpr int ALV = (2 * NB + 1) * MMAX + NB;          // NR, LV (with LI), NAI in doubles
    static constexpr bool ALIAS = ALV * 8 + 12 * MMAX <= CAP * 8;  // beside the selected columns
    static constexpr int O_HKEY = 0;
    static constexpr int O_HVAL = al16(CAP * 4);
    static constexpr int O_SEL = O_HVAL + CAP * 8 - 12 * MMAX;    // sel, row start, row end [MMAX]
    static constexpr int O_MS = O_HVAL + CAP * 8;                 // Memb[MMAX] (GS < 64)
    static constexpr int O_AL = O_MS + (GS < 64 ? MMAX * 16 : 0);
    static constexpr int FIXED = al16(O_AL + (ALIAS ? 0 : ALV * 8));
    static __host__ __device__ constexpr int w_entries(int mm) { return mm > 1 ? (mm - 1) * mm / 2 : 0; }
    // (8 doubles after W: the unrolled products read up to 7 entries past a row's diagonal)
    static __host__ __device__ constexpr int bytes(int mm) { return FIXED + al16((w_entries(mm) + 8) * 8); }
};

struct Memb {
    int32_t beg, len;  // row start, entries left of column i
    double g;          // value of g at the member's position
};

// ---- moves and group reductions -------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ int dmov(int v) {
    return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dmov(double v) {
    const int lo = dmov<CTRL>(__double2loint(v)), hi = dmov<CTRL>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ uint32_t dmov(uint32_t v) { return (uint32_t)dmov<CTRL>((int)v); }
// lane ^ 16 inside each half of the wavefront (ds_swizzle bit mode: and 0x1F, xor 0x10)
__device__ __forceinline__ int xor16(int v) { return __builtin_amdgcn_ds_swizzle(v, 0x401F); }
__device__ __forceinline__ uint32_t xor16(uint32_t v) { return (uint32_t)xor16((int)v); }
__device__ __forceinline__ double xor16(double v) {
    const int lo = xor16(__double2loint(v)), hi = xor16(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ int rlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ uint32_t rlane(uint32_t v, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)v, l); }
__device__ __forceinline__ double rlane(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

struct OpSum {
    __device__ static double f(double a, double b) { return a + b; }
};
struct OpMax {
    __device__ static double f(double a, double b) { return fmax(a, b); }
};
struct OpMinU {
    __device__ static uint32_t f(uint32_t a, uint32_t b) { return a < b ? a : b; }
};

// All-reduce over each group of GS lanes; every lane of the group gets the result.  The
// pairing is symmetric at every stage, so all lanes hold the same bits (sums too).
template <int GS, class Op, class T>
__device__ __forceinline__ T gred(T v) {
    v = Op::f(v, dmov<0xB1>(v));   // quad_perm [1,0,3,2]: lane ^ 1
    v = Op::f(v, dmov<0x4E>(v));   // quad_perm [2,3,0,1]: lane ^ 2
    v = Op::f(v, dmov<0x141>(v));  // row_half_mirror: quads of one 8-lane half
    if constexpr (GS >= 16) v = Op::f(v, dmov<0x140>(v));  // row_mirror: the two halves of a row
    if constexpr (GS >= 32) v = Op::f(v, xor16(v));         // rows 0/1 and 2/3
    if constexpr (GS == 64) v = Op::f(rlane(v, 0), rlane(v, 32));
    return v;
}

// 1/sqrt(x) for x > 0: the hardware estimate refined by two Newton steps
// (y <- y + y (1 - x y^2) / 2), well within the parity tolerance of G
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-x * y, y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}

// Orders LDS accesses across the lanes of the block's one wavefront: a wavefront's LDS
// instructions execute in issue order, so only the compiler must keep memory accesses on their
// side of this point (no wait for global loads still in flight).
__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_wave_barrier();
    __asm__ __volatile__("" ::: "memory");
}

// Finds column c (< 2^24) in the table, inserting it when absent; returns the slot or -1 when
// the table is full; `fresh` tells whether this call inserted it, `key` is the stored key.
// Slots form buckets of four keys read with one 16-byte load; a column lives in the first
// bucket from its hash on that has room (buckets in order), so most lookups take one read.
// Within one call of the lanes of a group the columns are distinct, so a failed claim of an
// empty slot means another column took it: the bucket is read again.
template <int CAP>
__device__ __forceinline__ int tfind(uint32_t *hkey, uint32_t c, bool &fresh, uint32_t &key) {
    constexpr int NBK = CAP / 4;
    constexpr int B = __builtin_ctz(NBK);
    uint32_t b = (c * 2654435761u) >> (32 - B);
    for (int probe = 0; probe < NBK;) {
        const uint4 k4 = *reinterpret_cast<const uint4 *>(&hkey[4 * b]);
        const uint32_t kk[4] = {k4.x, k4.y, k4.z, k4.w};
        int empty = -1;
#pragma unroll
        for (int e = 3; e >= 0; --e) {
            if (kk[e] == kEmptyKey) {
                empty = e;
            } else if ((kk[e] & kColBits) == c) {
                key = kk[e];
                return (int)(4 * b + e);
            }
        }
        if (empty < 0) {
            b = (b + 1) & (NBK - 1);
            ++probe;
            continue;
        }
        const uint32_t old = atomicCAS(&hkey[4 * b + empty], kEmptyKey, c);
        if (old == kEmptyKey) {
            fresh = true;
            key = c;
            return (int)(4 * b + empty);
        }
    }
    return -1;
}

// tfind for two columns of one lane at once (act0/act1: whether to look each up): the bucket
// reads of both go out together, then the claims of both, so the two lookups share their LDS
// round trips.  Same placement rule and results per column as tfind; slot -1 when the table
// is full (or the column was not looked up).  Equal columns would also be found right: both
// lookups claim the same empty slot, one claim wins and the other reads the bucket again.
template <int CAP>
__device__ __forceinline__ void tfind2(uint32_t *hkey, uint32_t c0, bool act0, uint32_t c1, bool act1, int &s0,
                                       int &s1, uint32_t &k0, uint32_t &k1) {
    constexpr int NBK = CAP / 4;
    constexpr int B = __builtin_ctz(NBK);
    uint32_t b0 = (c0 * 2654435761u) >> (32 - B), b1 = (c1 * 2654435761u) >> (32 - B);
    int p0 = 0, p1 = 0;
    bool w0 = act0, w1 = act1;  // still looking
    s0 = -1;
    s1 = -1;
    k0 = 0u;
    k1 = 0u;
    while (w0 || w1) {
        uint4 q0 = make_uint4(0u, 0u, 0u, 0u), q1 = make_uint4(0u, 0u, 0u, 0u);
        if (w0) q0 = *reinterpret_cast<const uint4 *>(&hkey[4 * b0]);
        if (w1) q1 = *reinterpret_cast<const uint4 *>(&hkey[4 * b1]);
        int e0 = -1, e1 = -1;  // smallest empty slot of each bucket
        if (w0) {
            const uint32_t kk[4] = {q0.x, q0.y, q0.z, q0.w};
#pragma unroll
            for (int e = 3; e >= 0; --e) {
                if (kk[e] == kEmptyKey) {
                    e0 = e;
                } else if ((kk[e] & kColBits) == c0) {
                    s0 = (int)(4 * b0 + e);
                    k0 = kk[e];
                }
            }
            if (s0 >= 0) {
                w0 = false;
                e0 = -1;
            } else if (e0 < 0) {  // full bucket without the column: the next one
                b0 = (b0 + 1) & (NBK - 1);
                if (++p0 >= NBK) w0 = false;
            }
        }
        if (w1) {
            const uint32_t kk[4] = {q1.x, q1.y, q1.z, q1.w};
#pragma unroll
            for (int e = 3; e >= 0; --e) {
                if (kk[e] == kEmptyKey) {
                    e1 = e;
                } else if ((kk[e] & kColBits) == c1) {
                    s1 = (int)(4 * b1 + e);
                    k1 = kk[e];
                }
            }
            if (s1 >= 0) {
                w1 = false;
                e1 = -1;
            } else if (e1 < 0) {
                b1 = (b1 + 1) & (NBK - 1);
                if (++p1 >= NBK) w1 = false;
            }
        }
        uint32_t o0 = 0u, o1 = 0u;
        if (e0 >= 0) o0 = atomicCAS(&hkey[4 * b0 + e0], kEmptyKey, c0);
        if (e1 >= 0) o1 = atomicCAS(&hkey[4 * b1 + e1], kEmptyKey, c1);
        // a failed claim means another column took the slot: its bucket is read again
        if (e0 >= 0 && o0 == kEmptyKey) {
            s0 = (int)(4 * b0 + e0);
            k0 = c0;
            w0 = false;
        }
        if (e1 >= 0 && o1 == kEmptyKey) {
            s1 = (int)(4 * b1 + e1);
            k1 = c1;
            w1 = false;
        }
    }
}

// With one row per wavefront (GS = 64) every row-state value is the same in all lanes; read as
// a scalar, a condition or loop bound on it becomes a scalar branch instead of exec-mask
// bookkeeping, and a loop over such a bound a scalar loop instead of a divergent one.  Groups
// of fewer lanes keep their per-group values.
template <int GS>
__device__ __forceinline__ int wu(int v) {
    if constexpr (GS == 64) return __builtin_amdgcn_readfirstlane(v);
    else return v;
}
template <int GS>
__device__ __forceinline__ bool wu(bool b) {
    return wu<GS>(b ? 1 : 0) != 0;
}

template <int GS>
__device__ __forceinline__ uint64_t group_bits(int grp) {
    if constexpr (GS == 64) return ~0ull;
    else return ((1ull << GS) - 1ull) << (grp * GS);
}
// number of set bits of m below this lane
__device__ __forceinline__ int bits_below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// The two largest candidates (|gradient|, key, slot) among this lane's table slots; members
// and empty slots (whose keys carry the member bit) are skipped
template <int GS, int SPL>
__device__ __forceinline__ void top2(const uint32_t *hkey, const double *hval, int gl, double &a1, double &a2,
                                     uint32_t &k1, uint32_t &k2, int &e1, int &e2) {
    a1 = -1.0;
    a2 = -1.0;
    k1 = k2 = kEmptyKey;
    e1 = e2 = 0;
    // unrolled in full only for short scans (16 slots a lane at most for a wavefront per row, 8
    // for smaller groups): the long scans of big tables spill when unrolled in full
#pragma unroll(SPL <= (GS == 64 ? 16 : 8) ? SPL : 4)
    for (int jj = 0; jj < SPL; ++jj) {
        const int e = gl + GS * jj;
        const uint32_t kk = hkey[e];
        const double a = (kk & kMember) ? -1.0 : fabs(hval[e]);
        // value selects only (conditional stores to the pair would become a private array)
        const bool g1 = a > a1, g2 = a > a2;
        a2 = g1 ? a1 : (g2 ? a : a2);
        k2 = g1 ? k1 : (g2 ? kk : k2);
        e2 = g1 ? e1 : (g2 ? e : e2);
        a1 = g1 ? a : a1;
        k1 = g1 ? kk : k1;
        e1 = g1 ? e : e1;
    }
}

template <int GS, int MMAX, int CAP, int NB, bool G32>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(GS == 8 || (GS == 64 && MMAX <= 24 && CAP <= 512) ? 4 : (CAP <= 512 && MMAX <= 48 ? 3 : 1), 8))) void k_rows_w(
    int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, const double *__restrict__ av,
    const float *__restrict__ av32, const double *__restrict__ diag, const int32_t *__restrict__ dlo, int kmax, int s, double eps, double tau,
    int /*gmax*/, const int32_t *__restrict__ list, int nlist, int32_t *__restrict__ counters, int nxcd, int claim,
    int32_t *__restrict__ ell_col, double *__restrict__ ell_val, int ldell, int32_t *__restrict__ m_out,
    double *__restrict__ psi_out, int32_t *__restrict__ steps_out, int32_t *__restrict__ reason_out,
    int8_t *__restrict__ status_out, int32_t *__restrict__ ovf_count, int32_t *__restrict__ ovf_list) {
    using LY = Layout<GS, MMAX, CAP, NB>;
    static_assert(MMAX <= GS && MMAX <= 64, "one lane per pattern position");
    static_assert(CAP <= 65536, "16-bit slots");
    constexpr int RPW = 64 / GS;
    constexpr int SPW = LY::SPW;
    constexpr int SLW = SPW / 2;
    constexpr int SPL = CAP / GS;                 // table slots per lane
    static_assert(12 * MMAX <= CAP * 8, "the selected columns fit in the gradient array");
    constexpr int HMAX = (128 + GS - 1) / GS;     // chunks of a gathered row (rows <= 128 entries)
    constexpr int PF = HMAX < 4 ? HMAX : 4;       // chunks loaded ahead for every gathered row
    constexpr int QB = qb_of(GS);
    using AVT = typename std::conditional<G32, float, double>::type;

    extern __shared__ __align__(16) unsigned char lds_w[];
    __shared__ int32_t s_row;
    const int lane = threadIdx.x;
    const int gl = lane & (GS - 1), grp = lane / GS;
    const int mmx = kmax > 0 ? 1 + kmax * s : 1;  // largest pattern
    unsigned char *gbase = lds_w + grp * LY::bytes(mmx);
    uint32_t *hkey = reinterpret_cast<uint32_t *>(gbase + LY::O_HKEY);
    double *hval = reinterpret_cast<double *>(gbase + LY::O_HVAL);
    double *Wm = reinterpret_cast<double *>(gbase + LY::FIXED);
    Memb *memb = reinterpret_cast<Memb *>(gbase + LY::O_MS);
    int32_t *sel = reinterpret_cast<int32_t *>(gbase + LY::O_SEL);  // [MMAX] selected columns
    int32_t *selb = sel + MMAX;                                     // [MMAX] their row starts
    int32_t *sele = selb + MMAX;                                    // [MMAX] their row ends
    double *NR = LY::ALIAS ? hval : reinterpret_cast<double *>(gbase + LY::O_AL);  // [NB][MMAX]
    double *LV = NR + NB * MMAX;                                                   // [NB+1][MMAX]
    double *NAI = LV + (NB + 1) * MMAX;                                            // [NB]: a_{u,i}
    const uint64_t gm = group_bits<GS>(grp);
    const double tauv = tau;

    const int x = blockIdx.x % nxcd;
    const int64_t per = ((int64_t)nlist + nxcd - 1) / nxcd;
    const int q0 = (int)min<int64_t>(nlist, per * x), q1 = (int)min<int64_t>(nlist, per * (x + 1));
    const int take = claim * RPW;

    int qn = 0, qe = 0;
    for (;;) {
        if (qn >= qe) {
            if (lane == 0) s_row = q0 + atomicAdd(&counters[x], take);
            __syncthreads();
            qn = __builtin_amdgcn_readfirstlane(s_row);  // the block is one wavefront: a scalar
            __syncthreads();
            if (qn >= q1) break;
            qe = min(qn + take, q1);
        }
        const int qi = qn + grp;
        qn += RPW;
        const bool have = qi < qe;
        const int i = have ? (list ? list[qi] : qi) : 0;

        // ---- row state (uniform inside the group) and per-position registers
        int8_t status = ROW_OK;
        int32_t reason = STOP_KMAX;
        int steps = 0, m_o = 0;
        double aii = 1.0;
        int ibeg = 0, ilen = 0;
        if (have) {
            aii = diag[i];
            ibeg = rp[i];
            ilen = dlo[i];
        }
        bool act = have;
        if (act && (!(aii > 0.0) || !isfinite(aii))) {
            status = ROW_NOT_SPD;
            act = false;
        }
        double psi = aii;
        const double psi0 = aii;
        double gi = act ? 1.0 / sqrt(aii) : 0.0;
        int r_col = 0, r_beg = 0, r_len = 0;
        double r_g = 0.0, r_ai = 0.0, r_li = 0.0;
        uint32_t slr[MMAX][SLW];
#pragma unroll
        for (int q = 0; q < MMAX; ++q)
#pragma unroll
            for (int w = 0; w < SLW; ++w) slr[q][w] = 0u;

#pragma unroll
        for (int jj = 0; jj < CAP / GS; ++jj) hkey[gl + GS * jj] = kEmptyKey;
        wsync();
        if (act && kmax > 0) {
            if (ilen > LY::LROW) {
                status = ROW_OVERFLOW;
                act = false;
            }
        }
        if (act && kmax > 0) {
            // row i's entries left of the diagonal: the first candidates
            bool bad = false;
#pragma unroll
            for (int h = 0; h < SPW; ++h) {
                const int o = gl + GS * h;
                if (o < ilen) {
                    bool fresh = false;
                    uint32_t kf;
                    const int slot = tfind<CAP>(hkey, (uint32_t)ci[ibeg + o], fresh, kf);
                    if (slot < 0) bad = true;
                    else slr[0][h >> 1] |= (uint32_t)slot << (16 * (h & 1));
                }
            }
            if (__ballot(bad) & gm) {
                status = ROW_OVERFLOW;
                act = false;
            }
        }

        for (int k = 1; k <= kmax; ++k) {
            if (!__ballot(act)) break;

            // ---- 1. product pass
            if (wu<GS>(act)) {
#pragma unroll
                for (int jj = 0; jj < SPL; ++jj) hval[gl + GS * jj] = 0.0;
                if constexpr (GS < 64) {
                    if (gl == 0) memb[0] = Memb{ibeg, ilen, gi};
                    if (gl < m_o) memb[gl + 1] = Memb{r_beg, r_len, r_g};
                }
            }
            wsync();
            const int mo_u = wu<GS>(m_o);
            if (wu<GS>(act)) {
#pragma unroll
                for (int qb = 0; qb < MMAX; qb += QB) {
                    if (qb <= mo_u) {
                        int slt[QB][SPW];
                        AVT aa[QB][SPW];
                        double gg[QB];
#pragma unroll
                        for (int u = 0; u < QB; ++u) {
                            const int q = qb + u;
                            int beg = 0, len = 0;
                            gg[u] = 0.0;
                            if (q < MMAX && q <= mo_u) {
                                if constexpr (GS == 64) {
                                    // member q: row i (q = 0) or position q - 1, uniform values
                                    if (q == 0) {
                                        beg = ibeg;
                                        len = ilen;
                                        gg[u] = gi;
                                    } else {
                                        beg = rlane(r_beg, q - 1);
                                        len = rlane(r_len, q - 1);
                                        gg[u] = rlane(r_g, q - 1);
                                    }
                                } else {
                                    const Memb mb = memb[q];
                                    beg = mb.beg;
                                    len = mb.len;
                                    gg[u] = mb.g;
                                }
                            }
#pragma unroll
                            for (int h = 0; h < SPW; ++h) {
                                const int o = gl + GS * h;
                                slt[u][h] = -1;
                                aa[u][h] = AVT(0);
                                if (q < MMAX && o < len) {
                                    slt[u][h] = (int)((slr[q < MMAX ? q : 0][h >> 1] >> (16 * (h & 1))) & 0xffffu);
                                    // cached loads (rows are read again at later steps); FP32 values
                                    // for the precision form's gradient
                                    if constexpr (G32) aa[u][h] = av32[beg + o];
                                    else aa[u][h] = av[beg + o];
                                }
                            }
                        }
#pragma unroll
                        for (int u = 0; u < QB; ++u)
#pragma unroll
                            for (int h = 0; h < SPW; ++h)
                                if (slt[u][h] >= 0)
                                    __hip_atomic_fetch_add(&hval[slt[u][h]], (double)aa[u][h] * gg[u], __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                }
            }
            wsync();

            // ---- 2. selection.  One pass over the table keeps each lane's two largest
            //         candidates (value, key, slot).  A round then needs only reductions: with
            //         at most one candidate of each lane in the band of the current maximum, the
            //         smallest key among the lanes' largest candidates in the band wins, and the
            //         winning lane moves up its second (and marks its state as partial: its next
            //         candidate is unknown).  A lane with two candidates in the band, or a partial
            //         lane whose largest is in the band, makes the round exact the slow way: a
            //         pass over the table for the smallest key in the band, then a new first
            //         pass.  Candidates must exceed 2^-40 of the first maximum (eligibility).
            int ns = 0;
            int r_js = 0, r_nb = 0, r_ne = 0;  // lane v: v-th column selected in this step, its row extents
            if (wu<GS>(act)) {
                double a1, a2;
                uint32_t k1, k2;
                int e1, e2;
                top2<GS, SPL>(hkey, hval, gl, a1, a2, k1, k2, e1, e2);
                const double M = gred<GS, OpMax>(a1);
                if (wu<GS>(M > 0.0)) {
                    const double thr = 0x1.0p-40 * M;
                    bool partial = false;
                    for (int round = 0; round < s; ++round) {
                        const double v1 = a1 > thr ? a1 : -1.0;
                        const double v2 = a2 > thr ? a2 : -1.0;
                        const double Mp = round == 0 ? M : gred<GS, OpMax>(v1);
                        if (!wu<GS>(Mp > 0.0)) break;
                        const double band = (1.0 - tauv) * Mp;
                        const bool slow = (__ballot(v2 >= band || (partial && v1 >= band)) & gm) != 0;
                        uint32_t js;
                        if (!slow) {
                            js = gred<GS, OpMinU>(v1 >= band ? k1 : kEmptyKey);
                            const bool won = v1 >= band && k1 == js;
                            if (won) hkey[e1] = js | kMember | ((uint32_t)(m_o + ns) << 24);
                            a1 = won ? a2 : a1;
                            k1 = won ? k2 : k1;
                            e1 = won ? e2 : e1;
                            a2 = won ? -1.0 : a2;
                            k2 = won ? kEmptyKey : k2;
                            partial = partial || won;
                        } else {
                            uint32_t lb = kEmptyKey;
                            int le = 0;
#pragma unroll 4
                            for (int jj = 0; jj < SPL; ++jj) {
                                const int e = gl + GS * jj;
                                const uint32_t kk = hkey[e];
                                const double a = (kk & kMember) ? -1.0 : fabs(hval[e]);
                                if (a > thr && a >= band && kk < lb) {
                                    lb = kk;
                                    le = e;
                                }
                            }
                            js = gred<GS, OpMinU>(lb);
                            if (lb == js) hkey[le] = js | kMember | ((uint32_t)(m_o + ns) << 24);
                            top2<GS, SPL>(hkey, hval, gl, a1, a2, k1, k2, e1, e2);
                            partial = false;
                        }
                        // the new row's extents, loaded while the next rounds run
                        if (gl == ns) {
                            r_js = (int)js;
                            r_nb = rp[js];
                            r_ne = rp[js + 1];
                        }
                        ++ns;
                    }
                }
                if (ns == 0) {
                    reason = STOP_NOCAND;
                    act = false;
                }
            }
            wsync();
            // the selected columns into the gradient array's end (no longer read this step)
            if (act && gl < ns) {
                sel[gl] = r_js;
                selb[gl] = r_nb;
                sele[gl] = r_ne;
            }
            wsync();

            // ---- 3./4. gather the new rows and extend W, NB rows at a time
            bool spd = true;
            double yi = 0.0;  // lane j: (W^T l_i)_j, accumulated over the blocks of this step
            int nsd = 0;
            bool first = true;
            const int nsw = GS == 64 ? wu<GS>(ns)
                                     : __builtin_amdgcn_readfirstlane((int)gred<64, OpMax>((double)(act ? ns : 0)));
            for (int nw = 0; nw < nsw; nw += NB) {
                // old positions of this block (earlier blocks of the step included)
                const int mwb = GS == 64 ? wu<GS>(m_o)
                                         : __builtin_amdgcn_readfirstlane((int)gred<64, OpMax>((double)(act ? m_o : 0)));
                const int mo = wu<GS>(m_o);  // this row's old positions (a scalar with 64 lanes)
                const bool blk = wu<GS>(act && nsd < ns);
                const int nbk = wu<GS>(blk ? min(NB, ns - nsd) : 0);
                if (blk) {
#pragma unroll
                    for (int jj = 0; jj < (NB * MMAX + GS - 1) / GS; ++jj)
                        if (gl + GS * jj < NB * MMAX) NR[gl + GS * jj] = 0.0;
                    if (gl < NB) NAI[gl] = 0.0;
                }
                wsync();
                bool bad = false;
                if (blk) {
                    int gnb[NB], glen[NB];
                    int gc[NB][PF];
                    double ga[NB][PF];
#pragma unroll
                    for (int v = 0; v < NB; ++v) {
                        gnb[v] = 0;
                        glen[v] = 0;
                        if (v < nbk) {
                            gnb[v] = selb[nsd + v];
                            glen[v] = sele[nsd + v] - gnb[v];
                        }
                        if (glen[v] > 128) bad = true;
#pragma unroll
                        for (int h = 0; h < PF; ++h) {
                            const int o = gl + GS * h;
                            gc[v][h] = 0x7fffffff;
                            ga[v][h] = 0.0;
                            if (o < glen[v] && o < 128) {
                                gc[v][h] = ci[gnb[v] + o];
                                ga[v][h] = av[gnb[v] + o];
                            }
                        }
                    }
#pragma unroll
                    for (int v = 0; v < NB; ++v) {
                        if (v < nbk && !bad) {
                            const int p = mo + v;  // position of this new row
                            int nlo = 0;
                            uint32_t pk[SLW];
#pragma unroll
                            for (int w = 0; w < SLW; ++w) pk[w] = 0u;
                            if constexpr (GS == 64) {
                                // both chunks of the row (entries gl and gl + 64, loaded above)
                                // entered in the table by one paired lookup; the second only
                                // when the first lies entirely in the prefix up to column i
                                static_assert(HMAX == 2 && PF == 2 && SLW == 1 && LY::LROW == 128,
                                              "64 lanes: two chunks of a row, one slot word");
                                const int c0 = gc[v][0];
                                const double a0 = ga[v][0];
                                const bool two = glen[v] > GS && (__ballot(c0 <= i) & gm) == gm;
                                const int c1 = two ? gc[v][1] : 0x7fffffff;
                                const double a1 = ga[v][1];
                                if (c0 == i) NAI[v] = a0;
                                if (c1 == i) NAI[v] = a1;
                                const bool l0 = c0 < i, l1 = c1 < i;
                                int s0, s1;
                                uint32_t k0, k1;
                                tfind2<CAP>(hkey, (uint32_t)c0, l0, (uint32_t)c1, l1, s0, s1, k0, k1);
                                if ((l0 && s0 < 0) || (l1 && s1 < 0)) {
                                    bad = true;
                                } else {
                                    if (l0) {
                                        pk[0] |= (uint32_t)s0;
                                        if (k0 & kMember) NR[v * MMAX + (int)((k0 >> 24) & 0x7Fu)] = a0;
                                    }
                                    if (l1) {
                                        pk[0] |= (uint32_t)s1 << 16;
                                        if (k1 & kMember) NR[v * MMAX + (int)((k1 >> 24) & 0x7Fu)] = a1;
                                    }
                                }
                                nlo = __popcll(__ballot(l0) & gm) + __popcll(__ballot(l1) & gm);
                            } else {
#pragma unroll
                            for (int h = 0; h < HMAX; ++h) {
                                if (GS * h < glen[v]) {
                                    const int o = gl + GS * h;
                                    int c = 0x7fffffff;
                                    double a = 0.0;
                                    if (h < PF) {
                                        c = gc[v][h < PF ? h : 0];
                                        a = ga[v][h < PF ? h : 0];
                                    } else if (o < glen[v]) {
                                        c = ci[gnb[v] + o];
                                        a = av[gnb[v] + o];
                                    }
                                    if (c == i) NAI[v] = a;
                                    bool fresh = false;
                                    int slot = -1;
                                    if (c < i) {
                                        if (o >= LY::LROW) {
                                            bad = true;
                                        } else {
                                            uint32_t kf = 0u;
                                            slot = tfind<CAP>(hkey, (uint32_t)c, fresh, kf);
                                            if (slot < 0) {
                                                bad = true;
                                            } else {
                                                if (h < SPW) pk[(h < SPW ? h : 0) >> 1] |= (uint32_t)slot << (16 * (h & 1));
                                                if (kf & kMember) NR[v * MMAX + (int)((kf >> 24) & 0x7Fu)] = a;
                                            }
                                        }
                                    }
                                    nlo += __popcll(__ballot(c < i) & gm);
                                    // the columns up to i form a prefix of the row
                                    if ((__ballot(c <= i) & gm) != gm) break;
                                }
                            }
                            }
                            if (gl == p) {
                                r_beg = gnb[v];
                                r_len = nlo;
                                r_col = sel[nsd + v];
                            }
                            const int qm = p + 1;  // member index of position p
#pragma unroll
                            for (int q8 = 0; q8 < MMAX; q8 += 8) {
                                if (qm >= q8 && qm < q8 + 8) {
#pragma unroll
                                    for (int qq = q8; qq < q8 + 8 && qq < MMAX; ++qq)
                                        if (qq == qm)
#pragma unroll
                                            for (int w = 0; w < SLW; ++w) slr[qq][w] = pk[w];
                                }
                            }
                        }
                    }
                }
                if (__ballot(bad) & gm) {
                    if (blk) {
                        status = ROW_OVERFLOW;
                        act = false;
                    }
                }
                wsync();
                const bool go = blk && act;
                // a_{u,i} of the new positions
                if (go && gl >= mo && gl < mo + nbk) r_ai = NAI[gl - mo];

                // pass A: l_v[t] = sum_{j <= t} W[t][j] a_v[j] for the old positions t < m_o
                double la[NB];
#pragma unroll
                for (int v = 0; v < NB; ++v) la[v] = 0.0;
                {
                    // kPU entries of the row at a time: all loads first (in bounds: at most 7
                    // past the diagonal of the lane's row, or of row 0 for lanes without a row,
                    // within W's padding), then the entries right of the diagonal zeroed
                    const int lim = (go && gl < mo) ? gl : -1;
                    const double *wrow = Wm + tri_w(lim >= 0 ? gl : 0);
                    for (int j0 = 0; j0 < mwb; j0 += kPU) {
                        double wv[kPU];
#pragma unroll
                        for (int u = 0; u < kPU; ++u) wv[u] = wrow[j0 + u];
                        const int d = lim - j0;
#pragma unroll
                        for (int u = 0; u < kPU; ++u) wv[u] = u <= d ? wv[u] : 0.0;
#pragma unroll
                        for (int v = 0; v < NB; ++v)
                            if (v < nbk)
#pragma unroll
                                for (int u = 0; u < kPU; ++u) la[v] = fma(wv[u], NR[v * MMAX + j0 + u], la[v]);
                    }
                }
                if (go && gl < MMAX) {
                    // every entry of the rows (zeros past the old positions) for pass B's
                    // unrolled reads
#pragma unroll
                    for (int v = 0; v < NB; ++v) LV[v * MMAX + gl] = gl < mo ? la[v] : 0.0;
                    LV[NB * MMAX + gl] = (first && gl < mo) ? r_li : 0.0;
                }
                wsync();
                // pass B: y_v[j] = sum_{j <= t < m_o} W[t][j] l_v[t], and the same with l_i
                double yb[NB];
#pragma unroll
                for (int v = 0; v < NB; ++v) yb[v] = 0.0;
                {
                    // all loads first: rows t of the chunk past the old positions read the last
                    // old row, lanes without an old position column 0 (in bounds); then the
                    // entries with t < j or t >= m_o zeroed
                    const int jc = (go && gl < mo) ? gl : 0;
                    const int lo = (go && gl < mo) ? gl : 0x7fffffff;
                    for (int t0 = 0; t0 < mwb; t0 += kPU) {
                        double wv[kPU];
#pragma unroll
                        for (int u = 0; u < kPU; ++u) {
                            const int tc = min(t0 + u, mo - 1);
                            wv[u] = Wm[tri_w(tc) + jc];
                        }
#pragma unroll
                        for (int u = 0; u < kPU; ++u) {
                            const int t = t0 + u;
                            wv[u] = (t >= lo && t < mo) ? wv[u] : 0.0;
                        }
#pragma unroll
                        for (int v = 0; v < NB; ++v)
                            if (v < nbk)
#pragma unroll
                                for (int u = 0; u < kPU; ++u) yb[v] = fma(wv[u], LV[v * MMAX + t0 + u], yb[v]);
#pragma unroll
                        for (int u = 0; u < kPU; ++u) yi = fma(wv[u], LV[NB * MMAX + t0 + u], yi);
                    }
                }
                // the new rows one by one: their coupling inside the block, d_u, and row p of W
                double wn[NB];
#pragma unroll
                for (int v = 0; v < NB; ++v) wn[v] = 0.0;
                if (wu<GS>(go)) {
#pragma unroll
                    for (int v = 0; v < NB; ++v) {
                        if (v < nbk && wu<GS>(spd)) {
                            const int p = mo + v;
                            const double sq = gred<GS, OpSum>(gl < mo ? la[v] * la[v] : 0.0);
                            double d2 = NR[v * MMAX + p] - sq;
                            const double av_l = gl < MMAX ? NR[v * MMAX + (gl < MMAX ? gl : 0)] : 0.0;
                            double cp[NB];
#pragma unroll
                            for (int w = 0; w < NB; ++w) {
                                cp[w] = 0.0;
                                if (w < v) {
                                    cp[w] = gred<GS, OpSum>(wn[w] * av_l);
                                    d2 = d2 - cp[w] * cp[w];
                                }
                            }
                            if (!(d2 > 0.0) || !isfinite(d2)) {
                                spd = false;
                            } else {
                                const double dinv = rsqrt_nr(d2);
                                double y = yb[v];
#pragma unroll
                                for (int w = 0; w < NB; ++w)
                                    if (w < v) y = fma(wn[w], cp[w], y);
                                wn[v] = gl < p ? -(y * dinv) : (gl == p ? dinv : 0.0);
                                if (gl <= p) Wm[tri_w(p) + gl] = wn[v];
                            }
                        }
                    }
                    if (wu<GS>(spd)) {
                        // l_i at the new positions and psi
#pragma unroll
                        for (int w = 0; w < NB; ++w) {
                            if (w < nbk) {
                                const double li = gred<GS, OpSum>(wn[w] * r_ai);
                                if (gl == mo + w) r_li = li;
                                psi = psi - li * li;
                                yi = fma(wn[w], li, yi);
                            }
                        }
                    } else {
                        status = ROW_NOT_SPD;
                        act = false;
                    }
                }
                if (blk) {
                    m_o += nbk;
                    nsd += nbk;
                    first = false;
                }
                wsync();
            }

            // ---- 5. g, psi and the exit test
            if (wu<GS>(act)) {
                if (!(psi > 0.0) || !isfinite(psi)) {
                    status = ROW_NOT_SPD;
                    act = false;
                } else {
                    const double dinv = rsqrt_nr(psi);
                    gi = dinv;
                    r_g = gl < m_o ? -(yi * dinv) : 0.0;
                    steps = k;
                    if (psi <= eps * psi0) {
                        reason = STOP_EPS;
                        act = false;
                    }
                }
            }
        }

        // ---- outputs: the row with ascending columns (i, the largest, last)
        if (wu<GS>(have && status == ROW_OK)) {
            const int col = gl < m_o ? r_col : (gl == m_o ? i : 0x7fffffff);
            if (gl <= m_o) sel[gl] = col;
            wsync();
            int rank = 0;
            const int mo_u = wu<GS>(m_o);
            for (int t = 0; t <= mo_u; ++t) rank += (sel[t] < col) ? 1 : 0;
            if (gl <= m_o) {
                ell_col[(size_t)i * ldell + rank] = col;
                ell_val[(size_t)i * ldell + rank] = gl < m_o ? r_g : gi;
            }
        } else {
            wsync();
        }
        if (have && gl == 0) {
            m_out[i] = (status == ROW_OK) ? m_o + 1 : 0;
            psi_out[i] = psi;
            steps_out[i] = steps;
            reason_out[i] = reason;
            status_out[i] = status;
            if (status == ROW_OVERFLOW) {
                const int pos = atomicAdd(ovf_count, 1);
                ovf_list[pos] = i;
            }
        }
        wsync();
    }
}

}  // namespace wform

// LDS bytes (dynamic) of one block of k_rows_w<GS, MMAX, CAP, NB> for patterns of at most mm
// positions
template <int GS, int MMAX, int CAP, int NB>
__host__ constexpr size_t rows_w_lds_bytes(int mm) {
    return (size_t)(64 / GS) * (size_t)wform::Layout<GS, MMAX, CAP, NB>::bytes(mm);
}

}  // namespace afsai
