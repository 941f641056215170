// Internal helpers of libhdm: errors, device buffers, counter-based random numbers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/hdm.h"

namespace hdm {

// An error that maps to an hdm_status at the C boundary.
struct Error : std::runtime_error {
    hdm_status code;
    Error(hdm_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(hdm_status c, const std::string& m) { throw Error(c, m); }

#define HDM_HIP(call)                                                                                  \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            ::hdm::fail(e_ == hipErrorOutOfMemory ? HDM_ENOMEM : HDM_EDEVICE,                         \
                        std::string(#call) + ": " + hipGetErrorString(e_) + " (" + __FILE__ + ":" +     \
                            std::to_string(__LINE__) + ")");                                           \
    } while (0)

#define HDM_CHECK(cond, code, msg)                  \
    do {                                            \
        if (!(cond)) ::hdm::fail((code), (msg));    \
    } while (0)

inline void check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(HDM_EDEVICE, std::string("launch of ") + what + ": " + hipGetErrorString(e));
}

// Device memory behind DevBuf: a per-device cache of released blocks.
// dev_alloc takes the best-fitting cached block or calls hipMalloc.  A block
// released while a PoolScope is alive on the calling thread waits in that
// thread's pending list; when the outermost scope ends it synchronises the
// device and moves the pending blocks into the cache, so a cached block has no
// GPU work left on it.  A release outside any scope frees the block at once.
void* dev_alloc(size_t bytes);
void dev_free(void* p) noexcept;
struct PoolScope {
    PoolScope();
    ~PoolScope();
    PoolScope(const PoolScope&) = delete;
    PoolScope& operator=(const PoolScope&) = delete;
};
// Pinned host memory for an upload made inside a PoolScope, valid until the
// outermost scope ends (after its device synchronisation); nullptr outside a
// scope.  Copies from it are asynchronous, where copies from pageable memory
// are staged by the runtime and return only when done.
void* host_stage(size_t bytes);
// count elements from host memory to device memory on stream s, through
// host_stage when a scope is open
void upload_bytes(void* dst, const void* src, size_t bytes, hipStream_t s);

// Owning device allocation (no copy, movable).
template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    explicit DevBuf(size_t count) { alloc(count); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t count) {
        release();
        if (count == 0) return;
        p = static_cast<T*>(dev_alloc(count * sizeof(T)));
        n = count;
    }
    void release() {
        if (p) dev_free(p);
        p = nullptr;
        n = 0;
    }
    size_t bytes() const { return n * sizeof(T); }
    T* get() const { return p; }
    void upload(const T* host, size_t count, hipStream_t s) {
        if (count) upload_bytes(p, host, count * sizeof(T), s);
    }
    void upload(const std::vector<T>& v, hipStream_t s) {
        if (v.size() > n) alloc(v.size());
        upload(v.data(), v.size(), s);
    }
    void download(T* host, size_t count, hipStream_t s) const {
        if (count) HDM_HIP(hipMemcpyAsync(host, p, count * sizeof(T), hipMemcpyDeviceToHost, s));
    }
};

template <typename T>
DevBuf<T> to_device(const std::vector<T>& v, hipStream_t s) {
    DevBuf<T> b(v.size() ? v.size() : 1);
    b.upload(v.data(), v.size(), s);
    return b;
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11): 10 rounds of two 32x32->64 multiplications with the
// constants 0xD2511F53 / 0xCD9E8D57 and a Weyl key schedule 0x9E3779B9 /
// 0xBB67AE85.  One draw = first output word of counter (i, a, b, purpose) under
// key (seed low, seed high).
// ---------------------------------------------------------------------------
__host__ __device__ inline uint32_t philox_draw(uint64_t seed, uint32_t purpose, uint32_t a, uint32_t b, uint32_t i) {
    uint32_t x0 = i, x1 = a, x2 = b, x3 = purpose;
    uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t m0 = static_cast<uint64_t>(0xD2511F53u) * x0;
        const uint64_t m1 = static_cast<uint64_t>(0xCD9E8D57u) * x2;
        const uint32_t y0 = static_cast<uint32_t>(m1 >> 32) ^ x1 ^ k0;
        const uint32_t y2 = static_cast<uint32_t>(m0 >> 32) ^ x3 ^ k1;
        x1 = static_cast<uint32_t>(m1);
        x3 = static_cast<uint32_t>(m0);
        x0 = y0;
        x2 = y2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return x0;
}

// integer in [0, bound) by multiply-shift of one 32-bit draw
__host__ __device__ inline uint32_t below(uint32_t r, uint32_t bound) {
    return static_cast<uint32_t>((static_cast<uint64_t>(r) * bound) >> 32);
}

enum Purpose : uint32_t { kTreeSample = 1, kKnnPivot = 2, kRowFill = 3, kLanczosStart = 4 };

inline int ceil_div(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

inline size_t dtype_size(int dt) {
    switch (dt) {
        case HDM_F64: return 8;
        case HDM_F32: return 4;
        case HDM_BF16: return 2;
        case HDM_F16: return 2;
        case HDM_U8: return 1;
    }
    return 0;
}

}  // namespace hdm
