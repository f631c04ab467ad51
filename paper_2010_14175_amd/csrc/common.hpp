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
// set_error, returning `code`
int set_error_code(int code, const char *fmt, ...);
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
// device memory: caching allocator (blocks are kept per device and reused by size class;
// afsai_release_cache() returns them to the runtime)
// ---------------------------------------------------------------------------------------
void *pool_alloc(size_t bytes);  // nullptr on failure
void pool_free(void *p);          // p may be nullptr; the caller guarantees no pending use
// pinned host memory from the same kind of cache (hipHostMalloc only on a miss)
void *pinned_alloc(size_t bytes);  // nullptr on failure
void pinned_free(void *p);         // p may be nullptr; the caller guarantees no pending use

// temporary device buffer, returned to the pool when it goes out of scope; the stream is
// synchronised first so that no enqueued kernel still uses it
struct DevBuf {
    void *p = nullptr;
    hipStream_t s = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() {
        if (p) {
            (void)hipStreamSynchronize(s);
            pool_free(p);
        }
    }
    template <typename T>
    T *as() { return (T *)p; }
    void *release() {
        void *q = p;
        p = nullptr;
        return q;
    }
};

inline int dalloc(DevBuf &b, size_t bytes, hipStream_t s) {
    b.s = s;
    b.p = pool_alloc(bytes ? bytes : 16);
    if (!b.p) {
        set_error("out of device memory (%zu bytes)", bytes);
        return AFSAI_ERR_NO_MEMORY;
    }
    return AFSAI_OK;
}

inline int pow2ceil(int64_t v) {
    int64_t p = 1;
    while (p < v) p <<= 1;
    return (int)p;
}

// ---------------------------------------------------------------------------------------
// device properties (cached per device)
// ---------------------------------------------------------------------------------------
struct DeviceInfo {
    int device = -1;
    int num_cus = 256;
    int num_xcds = 8;
};
int device_info(DeviceInfo *out);

// grid for a grid-stride loop over `work` items
inline int grid1d(int64_t work, const DeviceInfo &di, int threads = 256) {
    int64_t b = (work + threads - 1) / threads;
    const int64_t cap = (int64_t)di.num_cus * 16;
    if (b > cap) b = cap;
    return (int)(b < 1 ? 1 : b);
}

// exclusive scan of cnt[0..n) into out[0..n] (out[n] = total, int32); *total (host) gets the
// 64-bit total; synchronous on s
int scan_counts(int n, const int32_t *cnt, int32_t *out, int64_t *total, const DeviceInfo &di, hipStream_t s);

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
// the same operations with DPP lane moves (no LDS-pipe round trip).  GFX9 DPP controls:
// row_shr:k = 0x110+k, row_ror:k = 0x120+k (rows of 16 lanes), row_bcast:15 = 0x142 (lane 15
// of each row to the next row), row_bcast:31 = 0x143 (lane 31 to rows 2 and 3).  Lanes of
// rows outside row_mask keep `old`.
// ---------------------------------------------------------------------------------------
template <int CTRL, int ROWMASK, bool BOUND>
__device__ __forceinline__ int dpp_i32(int old, int v) {
    return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWMASK, 0xF, BOUND);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_f64(double old, double v) {
    const int lo = dpp_i32<CTRL, ROWMASK, false>(__double2loint(old), __double2loint(v));
    const int hi = dpp_i32<CTRL, ROWMASK, false>(__double2hiint(old), __double2hiint(v));
    return __hiloint2double(hi, lo);
}
// maximum over the 64 lanes, returned uniform (read from lane 63)
__device__ __forceinline__ double wave_max_dpp(double v) {
    v = fmax(v, dpp_f64<0x121, 0xF>(v, v));
    v = fmax(v, dpp_f64<0x122, 0xF>(v, v));
    v = fmax(v, dpp_f64<0x124, 0xF>(v, v));
    v = fmax(v, dpp_f64<0x128, 0xF>(v, v));
    v = fmax(v, dpp_f64<0x142, 0xA>(v, v));
    v = fmax(v, dpp_f64<0x143, 0xC>(v, v));
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float wave_max_dpp(float v) {
    v = fmaxf(v, __int_as_float(dpp_i32<0x121, 0xF, false>(__float_as_int(v), __float_as_int(v))));
    v = fmaxf(v, __int_as_float(dpp_i32<0x122, 0xF, false>(__float_as_int(v), __float_as_int(v))));
    v = fmaxf(v, __int_as_float(dpp_i32<0x124, 0xF, false>(__float_as_int(v), __float_as_int(v))));
    v = fmaxf(v, __int_as_float(dpp_i32<0x128, 0xF, false>(__float_as_int(v), __float_as_int(v))));
    v = fmaxf(v, __int_as_float(dpp_i32<0x142, 0xA, false>(__float_as_int(v), __float_as_int(v))));
    v = fmaxf(v, __int_as_float(dpp_i32<0x143, 0xC, false>(__float_as_int(v), __float_as_int(v))));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
// minimum over the 64 lanes (unsigned), returned uniform
__device__ __forceinline__ uint32_t wave_min_dpp(uint32_t v) {
    v = min(v, (uint32_t)dpp_i32<0x121, 0xF, false>((int)v, (int)v));
    v = min(v, (uint32_t)dpp_i32<0x122, 0xF, false>((int)v, (int)v));
    v = min(v, (uint32_t)dpp_i32<0x124, 0xF, false>((int)v, (int)v));
    v = min(v, (uint32_t)dpp_i32<0x128, 0xF, false>((int)v, (int)v));
    v = min(v, (uint32_t)dpp_i32<0x142, 0xA, false>((int)v, (int)v));
    v = min(v, (uint32_t)dpp_i32<0x143, 0xC, false>((int)v, (int)v));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}
// inclusive prefix sum over the 64 lanes
__device__ __forceinline__ int wave_scan_dpp(int v) {
    v += dpp_i32<0x111, 0xF, true>(0, v);
    v += dpp_i32<0x112, 0xF, true>(0, v);
    v += dpp_i32<0x114, 0xF, true>(0, v);
    v += dpp_i32<0x118, 0xF, true>(0, v);
    v += dpp_i32<0x142, 0xA, false>(0, v);
    v += dpp_i32<0x143, 0xC, false>(0, v);
    return v;
}

// ---------------------------------------------------------------------------------------
// kernel timer (HIP events around each launch while profiling is on)
// ---------------------------------------------------------------------------------------
bool profiling_on();
// records a start event on `s` and returns a token (or -1 when profiling is off)
int prof_begin(const char *name, hipStream_t s);
void prof_end(int token, const char *name, hipStream_t s);
// resolves pending events (called at synchronisation points)
void prof_flush();
// position in the list of timed launches not yet resolved, and removal of a range of them
// (launches that returned at once because the iteration had already ended)
int prof_mark();
void prof_drop(int from, int to);

struct ProfScope {
    int tok;
    const char *name;
    hipStream_t s;
    ProfScope(const char *n, hipStream_t st) : tok(prof_begin(n, st)), name(n), s(st) {}
    ~ProfScope() { prof_end(tok, name, s); }
};

}  // namespace afsai

