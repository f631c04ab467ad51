// Internal helpers shared by the HIP translation units of the adaptive FSAI library:
// error reporting, device properties, XCD-aware block mapping, wavefront reductions and the
// optional per-kernel event timer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/afsai.h"

namespace afsai {

// ---------------------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------------------
void set_error(const char *fmt, ...);
void clear_error();

#define AFSAI_HIP_TRY(expr)                                                                  \
    do {                                                                                     \
        hipError_t _e = (expr);                                                              \
        if (_e != hipSuccess) {                                                              \
            ::afsai::set_error("%s:%d: %s -> %s", __FILE__, __LINE__, #expr,                 \
                               hipGetErrorString(_e));                                       \
            return (_e == hipErrorOutOfMemory) ? AFSAI_ERR_NO_MEMORY : AFSAI_ERR_HIP;        \
        }                                                                                    \
    } while (0)

#define AFSAI_FAIL(code, ...)                                                                \
    do {                                                                                     \
        ::afsai::set_error(__VA_ARGS__);                                                     \
        return (code);                                                                       \
    } while (0)

// value of an afsai_set_option knob (0 = automatic)
int64_t option(int id);

// ---------------------------------------------------------------------------------------
// device properties (cached per device)
// ---------------------------------------------------------------------------------------
struct DeviceInfo {
    int device = -1;
    int num_cus = 256;
    int num_xcds = 8;
};
int device_info(DeviceInfo *out);

// Blocks of a launch are dealt to the XCDs round robin (block b runs on XCD b % num_xcds).
// xcd_block() renumbers them so that each XCD receives one contiguous range of logical
// blocks, which keeps neighbouring rows (and the vector entries they share) in one L2.
__device__ __forceinline__ int xcd_block(int b, int nblocks, int nxcd) {
    if (nxcd <= 1 || nblocks < nxcd) return b;
    const int x = b % nxcd, k = b / nxcd;
    const int per = nblocks / nxcd, extra = nblocks % nxcd;
    // XCD x owns per (+1 for x < extra) consecutive logical blocks
    return x * per + (x < extra ? x : extra) + k;
}
// note: valid because XCD x receives exactly per + (x < extra) physical blocks b = x + k*nxcd.

// ---------------------------------------------------------------------------------------
// wavefront (64-lane) reductions, lane order fixed => deterministic
// ---------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        T o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        T o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}
// inclusive prefix sum over the 64 lanes
__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
    }
    return v;
}

// ---------------------------------------------------------------------------------------
// kernel timer (HIP events around each launch while profiling is on)
// ---------------------------------------------------------------------------------------
bool profiling_on();
// records a start event on `s` and returns a token (or -1 when profiling is off)
int prof_begin(hipStream_t s);
void prof_end(int token, const char *name, hipStream_t s);
// resolves pending events (called at synchronisation points)
void prof_flush();

struct ProfScope {
    int tok;
    const char *name;
    hipStream_t s;
    ProfScope(const char *n, hipStream_t st) : tok(prof_begin(st)), name(n), s(st) {}
    ~ProfScope() { prof_end(tok, name, s); }
};

}  // namespace afsai

// opaque handle
struct afsai_precond_s {
    int device = -1;
    int32_t n = 0;
    int64_t nnz_g = 0;
    int32_t g_prec = AFSAI_F64;
    int32_t mmax = 1;
    // G (lower) and G^T as CSR
    int32_t *g_rp = nullptr, *g_ci = nullptr;
    void *g_val = nullptr;  // double* or float*
    int32_t *gt_rp = nullptr, *gt_ci = nullptr;
    void *gt_val = nullptr;
    // per-row diagnostics (device)
    double *psi = nullptr;
    int32_t *steps = nullptr;
    int32_t *reason = nullptr;
    // workspace for apply (t) and PCG (r, z, p, q, t) and reductions
    double *work = nullptr;
    size_t work_elems = 0;
    afsai_setup_info info{};
};
