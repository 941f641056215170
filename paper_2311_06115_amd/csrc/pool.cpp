// Per-device cache of released device blocks behind DevBuf (see common.hpp).
// Compressing an operator and destroying one allocate and release a few dozen
// buffers each, from a few KB to hundreds of MB; hipMalloc and hipFree cost
// tens to hundreds of microseconds apiece and hipFree waits for the device, so
// repeated compressions spent milliseconds in them.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "common.hpp"

namespace hdm {
namespace {

struct Block {
    int device;
    size_t bytes;
};

struct Pool {
    std::mutex mu;
    std::map<int, std::multimap<size_t, void*>> free_;   // device -> (block bytes -> block)
    std::unordered_map<void*, Block> live;               // every block the pool handed out or holds
    std::map<int, size_t> cached, cap;                   // bytes in the free lists, and their cap, per device
};

Pool& pool() {
    static Pool* P = new Pool();   // never destroyed: blocks outlive static destruction
    return *P;
}

thread_local int t_depth = 0;
thread_local std::vector<void*> t_pending;

// pinned staging blocks of this thread, bump-allocated inside a scope and
// reused after the scope's device synchronisation
struct Stage {
    struct Block {
        char* p;
        size_t size, top;
    };
    std::vector<Block> blocks;
    void reset() {
        for (Block& b : blocks) b.top = 0;
    }
};
thread_local Stage t_stage;

size_t round_up(size_t b) {
    const size_t g = b < (size_t(1) << 20) ? 256 : (size_t(1) << 16);
    return (b + g - 1) / g * g;
}

// free cached blocks of a device, largest first, until at most keep bytes stay; mu held
void trim(Pool& P, int dev, size_t keep) {
    auto& fl = P.free_[dev];
    while (P.cached[dev] > keep && !fl.empty()) {
        auto it = std::prev(fl.end());
        (void)hipFree(it->second);
        P.cached[dev] -= it->first;
        P.live.erase(it->second);
        fl.erase(it);
    }
}

}  // namespace

void* dev_alloc(size_t bytes) {
    int dev = 0;
    HDM_HIP(hipGetDevice(&dev));
    const size_t r = round_up(bytes);
    Pool& P = pool();
    {
        std::lock_guard<std::mutex> g(P.mu);
        auto& fl = P.free_[dev];
        auto it = fl.lower_bound(r);
        // best fit, wasting at most half of a small block or a quarter of a large one
        const size_t limit = r < (size_t(1) << 20) ? 2 * r : r + r / 4;
        if (it != fl.end() && it->first <= limit) {
            void* p = it->second;
            P.cached[dev] -= it->first;
            fl.erase(it);
            return p;
        }
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, r);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        std::lock_guard<std::mutex> g(P.mu);
        trim(P, dev, 0);
        e = hipMalloc(&p, r);
    }
    HDM_HIP(e);
    std::lock_guard<std::mutex> g(P.mu);
    P.live[p] = Block{dev, r};
    return p;
}

void dev_free(void* p) noexcept {
    if (!p) return;
    if (t_depth > 0) {
        t_pending.push_back(p);
        return;
    }
    Pool& P = pool();
    std::lock_guard<std::mutex> g(P.mu);
    P.live.erase(p);
    (void)hipFree(p);
}

void* host_stage(size_t bytes) {
    if (t_depth == 0) return nullptr;
    const size_t need = (bytes + 255) / 256 * 256;
    for (Stage::Block& b : t_stage.blocks)
        if (b.size - b.top >= need) {
            void* p = b.p + b.top;
            b.top += need;
            return p;
        }
    const size_t size = std::max(need, size_t(8) << 20);
    void* p = nullptr;
    if (hipHostMalloc(&p, size, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    t_stage.blocks.push_back(Stage::Block{static_cast<char*>(p), size, need});
    return p;
}

void upload_bytes(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (!bytes) return;
    if (void* h = host_stage(bytes)) {
        std::memcpy(h, src, bytes);
        HDM_HIP(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, s));
    } else {
        HDM_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
    }
}

PoolScope::PoolScope() { ++t_depth; }

PoolScope::~PoolScope() {
    if (--t_depth > 0) return;
    bool staged = false;
    for (const Stage::Block& b : t_stage.blocks) staged = staged || b.top > 0;
    if (t_pending.empty() && !staged) return;
    Pool& P = pool();
    // the blocks may still be read or written, and the staging memory still be
    // copied from, by queued work on any stream
    const bool idle = hipDeviceSynchronize() == hipSuccess;
    if (idle) t_stage.reset();
    else t_stage.blocks.clear();   // in error: leave the staging blocks alone
    std::lock_guard<std::mutex> g(P.mu);
    for (void* p : t_pending) {
        auto it = P.live.find(p);
        if (!idle || it == P.live.end()) {
            // device in error: hipFree as before rather than reuse
            if (it != P.live.end()) P.live.erase(it);
            (void)hipFree(p);
            continue;
        }
        const Block b = it->second;
        if (!P.cap.count(b.device)) {
            size_t fr = 0, tot = 0;
            int cur = 0;
            (void)hipGetDevice(&cur);
            if (cur == b.device && hipMemGetInfo(&fr, &tot) == hipSuccess) P.cap[b.device] = tot / 4;
            else P.cap[b.device] = size_t(16) << 30;
        }
        P.free_[b.device].emplace(b.bytes, p);
        P.cached[b.device] += b.bytes;
    }
    t_pending.clear();
    for (auto& kv : P.cached)
        if (kv.second > P.cap[kv.first]) trim(P, kv.first, P.cap[kv.first]);
}

}  // namespace hdm
