// Host runtime pieces of the adaptive FSAI library: thread-local error messages, cached
// device properties and the HIP-event kernel timer behind afsai_profile_*.
#include <cstdarg>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace afsai {

static thread_local std::string g_last_error;

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

int set_error_code(int code, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

void clear_error() { g_last_error.clear(); }

static int64_t g_options[16] = {0};

int64_t option(int id) { return (id > 0 && id < 16) ? g_options[id] : 0; }

// ---------------------------------------------------------------------------------------
// caching allocator
// ---------------------------------------------------------------------------------------
namespace {
std::mutex pool_mu;
struct Block {
    size_t size;
    int device;
};
std::map<void *, Block> pool_live;                       // allocated blocks
std::map<int, std::multimap<size_t, void *>> pool_free_; // per device: size -> block

size_t size_class(size_t b) {
    if (b <= (1u << 20)) {
        size_t p = 256;
        while (p < b) p <<= 1;
        return p;
    }
    const size_t g = (size_t)2 << 20;  // 2 MiB granules above 1 MiB
    return (b + g - 1) / g * g;
}
}  // namespace

void *pool_alloc(size_t bytes) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    const size_t sz = size_class(bytes);
    {
        std::lock_guard<std::mutex> lk(pool_mu);
        auto &fl = pool_free_[dev];
        auto it = fl.lower_bound(sz);
        // reuse a cached block of the same class (or up to twice as large)
        if (it != fl.end() && it->first <= 2 * sz) {
            void *p = it->second;
            pool_live[p] = {it->first, dev};
            fl.erase(it);
            return p;
        }
    }
    void *p = nullptr;
    if (hipMalloc(&p, sz) != hipSuccess) {
        (void)hipGetLastError();
        // release cached blocks of this device and retry once
        std::vector<void *> drop;
        {
            std::lock_guard<std::mutex> lk(pool_mu);
            for (auto &kv : pool_free_[dev]) drop.push_back(kv.second);
            pool_free_[dev].clear();
        }
        for (void *q : drop) (void)hipFree(q);
        if (hipMalloc(&p, sz) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    std::lock_guard<std::mutex> lk(pool_mu);
    pool_live[p] = {sz, dev};
    return p;
}

void pool_free(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(pool_mu);
    auto it = pool_live.find(p);
    if (it == pool_live.end()) return;
    pool_free_[it->second.device].emplace(it->second.size, p);
    pool_live.erase(it);
}

// pinned host blocks (device-visible scalars of the solver), cached by size class like the
// device blocks; pinned memory is not tied to a device
namespace {
std::map<void *, size_t> pinned_live;
std::multimap<size_t, void *> pinned_free_;
}  // namespace

void *pinned_alloc(size_t bytes) {
    const size_t sz = size_class(bytes);
    {
        std::lock_guard<std::mutex> lk(pool_mu);
        auto it = pinned_free_.lower_bound(sz);
        if (it != pinned_free_.end() && it->first <= 2 * sz) {
            void *p = it->second;
            pinned_live[p] = it->first;
            pinned_free_.erase(it);
            return p;
        }
    }
    void *p = nullptr;
    if (hipHostMalloc(&p, sz, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(pool_mu);
    pinned_live[p] = sz;
    return p;
}

void pinned_free(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(pool_mu);
    auto it = pinned_live.find(p);
    if (it == pinned_live.end()) return;
    pinned_free_.emplace(it->second, p);
    pinned_live.erase(it);
}

int device_info(DeviceInfo *out) {
    static std::mutex mu;
    static std::map<int, DeviceInfo> cache;
    int dev = 0;
    AFSAI_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it == cache.end()) {
        DeviceInfo d;
        d.device = dev;
        int cus = 0;
        AFSAI_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        d.num_cus = cus > 0 ? cus : 1;
        // MI355X: 256 CUs in 8 XCDs of 32; smaller parts (or partition modes) get one group
        d.num_xcds = (d.num_cus % 8 == 0 && d.num_cus >= 64) ? 8 : 1;
        it = cache.emplace(dev, d).first;
    }
    *out = it->second;
    return AFSAI_OK;
}

// ---------------------------------------------------------------------------------------
// kernel timer
// ---------------------------------------------------------------------------------------
namespace {
struct Pending {
    hipEvent_t a, b;
    std::string name;
};
struct Acc {
    int64_t launches = 0;
    double ms = 0.0;
};
std::mutex prof_mu;
bool prof_enabled = false;
std::vector<std::string> prof_only;  // kernel names to time; empty: all
std::vector<hipEvent_t> event_pool;
std::vector<hipEvent_t> started;  // token -> start event
std::vector<Pending> pending;
std::map<std::string, Acc> totals;

hipEvent_t get_event() {
    if (!event_pool.empty()) {
        hipEvent_t e = event_pool.back();
        event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

bool profiling_on() {
    std::lock_guard<std::mutex> lk(prof_mu);
    return prof_enabled;
}

int prof_begin(const char *name, hipStream_t s) {
    std::lock_guard<std::mutex> lk(prof_mu);
    if (!prof_enabled) return -1;
    if (!prof_only.empty()) {
        bool hit = false;
        for (const std::string &k : prof_only) hit = hit || (name && k == name);
        if (!hit) return -1;
    }
    hipEvent_t e = get_event();
    if (!e) return -1;
    if (hipEventRecord(e, s) != hipSuccess) {
        event_pool.push_back(e);
        return -1;
    }
    started.push_back(e);
    return (int)started.size() - 1;
}

void prof_end(int token, const char *name, hipStream_t s) {
    if (token < 0) return;
    std::lock_guard<std::mutex> lk(prof_mu);
    if (token >= (int)started.size() || !started[token]) return;
    hipEvent_t b = get_event();
    if (!b) return;
    if (hipEventRecord(b, s) != hipSuccess) {
        event_pool.push_back(b);
        return;
    }
    pending.push_back({started[token], b, name});
    started[token] = nullptr;
}

void prof_flush() {
    std::lock_guard<std::mutex> lk(prof_mu);
    for (auto &p : pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            Acc &a = totals[p.name];
            a.launches += 1;
            a.ms += ms;
        }
        event_pool.push_back(p.a);
        event_pool.push_back(p.b);
    }
    pending.clear();
    bool all_done = true;
    for (auto e : started)
        if (e) all_done = false;
    if (all_done) started.clear();
}

int prof_mark() {
    std::lock_guard<std::mutex> lk(prof_mu);
    return (int)pending.size();
}

void prof_drop(int from, int to) {
    std::lock_guard<std::mutex> lk(prof_mu);
    if (from < 0) from = 0;
    if (to > (int)pending.size()) to = (int)pending.size();
    if (from >= to) return;
    for (int k = from; k < to; ++k) {
        (void)hipEventSynchronize(pending[k].b);
        event_pool.push_back(pending[k].a);
        event_pool.push_back(pending[k].b);
    }
    pending.erase(pending.begin() + from, pending.begin() + to);
}

}  // namespace afsai

extern "C" {

const char *afsai_last_error(void) { return afsai::g_last_error.c_str(); }

int afsai_set_option(int32_t opt, int64_t value) {
    auto pow2 = [](int64_t v) { return v > 0 && (v & (v - 1)) == 0; };
    bool ok = false;
    switch (opt) {
        case AFSAI_OPT_SETUP_GROUP: ok = (value >= 0 && value <= 4); break;
        case AFSAI_OPT_SETUP_TABLE: ok = value == 0 || (pow2(value) && value >= 64 && value <= 1024); break;
        case AFSAI_OPT_SPMV_GROUP: ok = value == 0 || (pow2(value) && value >= 4 && value <= 64); break;
        case AFSAI_OPT_SPMV_UNROLL: ok = value == 0 || (pow2(value) && value <= 8); break;
        case AFSAI_OPT_PCG_CSR_A: ok = (value == 0 || value == 1); break;
        case AFSAI_OPT_PCG_FORM: ok = (value >= 0 && value <= 2); break;
        case AFSAI_OPT_SELL_WIDTH: ok = (value >= 0 && value <= 4096); break;
        case AFSAI_OPT_PCG_GRAPH: ok = (value >= 0 && value <= 2); break;
        case AFSAI_OPT_SETUP_SLOTS: ok = (value >= 0 && value <= 2); break;
        case AFSAI_OPT_SELL_TAIL: ok = (value == 0 || value == 1); break;
        case AFSAI_OPT_SELL_UNEVEN: ok = (value == 0 || value == 1); break;
        case AFSAI_OPT_SETUP_FORM: ok = (value >= 0 && value <= 2); break;
        case AFSAI_OPT_SETUP_LANES: ok = value == 0 || (pow2(value) && value >= 8 && value <= 64); break;
        case AFSAI_OPT_SETUP_CLAIM: ok = (value >= 0 && value <= 64); break;
        case AFSAI_OPT_SELL_RUNS: ok = (value == 0 || value == 1); break;
        default: ok = false;
    }
    if (!ok) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_set_option: bad option %d / value %lld", opt, (long long)value);
    afsai::g_options[opt] = value;
    return AFSAI_OK;
}

int afsai_release_cache(void) {
    std::vector<void *> drop, dropped_pinned;
    {
        std::lock_guard<std::mutex> lk(afsai::pool_mu);
        for (auto &dv : afsai::pool_free_)
            for (auto &kv : dv.second) drop.push_back(kv.second);
        afsai::pool_free_.clear();
        for (auto &kv : afsai::pinned_free_) dropped_pinned.push_back(kv.second);
        afsai::pinned_free_.clear();
    }
    for (void *q : drop) AFSAI_HIP_TRY(hipFree(q));
    for (void *q : dropped_pinned) AFSAI_HIP_TRY(hipHostFree(q));
    return AFSAI_OK;
}

int afsai_profile_enable(int32_t on) {
    afsai::prof_flush();
    std::lock_guard<std::mutex> lk(afsai::prof_mu);
    afsai::prof_enabled = (on != 0);
    return AFSAI_OK;
}

int afsai_profile_only(const char *names) {
    std::vector<std::string> v;
    if (names) {
        std::string cur;
        for (const char *c = names;; ++c) {
            if (*c == ',' || *c == '\0') {
                if (!cur.empty()) v.push_back(cur);
                cur.clear();
                if (*c == '\0') break;
            } else {
                cur.push_back(*c);
            }
        }
    }
    std::lock_guard<std::mutex> lk(afsai::prof_mu);
    afsai::prof_only = v;
    return AFSAI_OK;
}

int afsai_profile_read(afsai_kernel_time *out, int32_t cap, int32_t *count, int32_t reset) {
    if (cap < 0 || (cap > 0 && !out)) AFSAI_FAIL(AFSAI_ERR_INVALID_ARG, "afsai_profile_read: bad buffer");
    afsai::prof_flush();
    std::lock_guard<std::mutex> lk(afsai::prof_mu);
    int32_t k = 0;
    for (auto &kv : afsai::totals) {
        if (k < cap) {
            std::memset(out[k].name, 0, sizeof out[k].name);
            std::strncpy(out[k].name, kv.first.c_str(), sizeof out[k].name - 1);
            out[k].launches = kv.second.launches;
            out[k].total_ms = kv.second.ms;
        }
        ++k;
    }
    if (count) *count = k < cap ? k : cap;
    if (reset) afsai::totals.clear();
    return AFSAI_OK;
}

}  // extern "C"
