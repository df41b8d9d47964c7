// Device block cache of the TIMEST GPU library.
//
// Tables and temporaries are allocated and released on every call; returning
// them to HIP each time costs milliseconds per call.  Released blocks are kept
// here instead.  A block released on stream S may serve a later allocation on
// S at once (stream order makes that safe) and any other stream once S has
// been synchronised by the library (every entry point synchronises its stream
// before it returns).  Memory goes back to HIP only when an allocation fails
// (after a device synchronisation, so no queued work still uses it).
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "tm_internal.h"

namespace {

struct Block {
    void* p;
    size_t cap;
    hipStream_t st;
    bool synced;
};

constexpr int kMaxDevices = 64;

std::mutex g_mu;
std::vector<Block> g_free[kMaxDevices];
std::unordered_map<void*, size_t> g_used;

// Blocks from a caller's allocator (tm_allocator): returned to it, never cached.
struct UserBlock {
    tm_allocator a;
    size_t bytes;
};
std::unordered_map<void*, UserBlock> g_user;

thread_local const tm_allocator* t_alloc = nullptr;

std::mutex g_stage_mu;
std::vector<void*> g_stage_free;

std::mutex g_ev_mu;
std::vector<hipEvent_t> g_ev_free[kMaxDevices];

size_t size_class(size_t bytes) {
    if (bytes <= 4096) return (bytes + 255) & ~(size_t)255;
    // steps of 1/8 of the enclosing power of two
    size_t p2 = 1;
    while (p2 < bytes) p2 <<= 1;
    const size_t step = p2 >> 4 > 4096 ? p2 >> 4 : 4096;
    return (bytes + step - 1) / step * step;
}

int device_index() {
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= kMaxDevices) return 0;
    return d;
}

}  // namespace

AllocScope::AllocScope(const tm_allocator* a) : prev_(t_alloc) {
    t_alloc = (a && a->alloc && a->free) ? a : nullptr;
}
AllocScope::~AllocScope() { t_alloc = prev_; }

hipError_t dev_alloc(void** p, size_t bytes, hipStream_t st) {
    *p = nullptr;
    if (t_alloc) {
        const tm_allocator a = *t_alloc;
        const size_t want = ((bytes ? bytes : 1) + 255) & ~(size_t)255;
        void* q = a.alloc(a.ctx, want, st);
        if (!q) return hipErrorOutOfMemory;
        std::lock_guard<std::mutex> lk(g_mu);
        g_user[q] = UserBlock{a, want};
        *p = q;
        return hipSuccess;
    }
    const size_t cls = size_class(bytes ? bytes : 1);
    const int dev = device_index();
    {
        std::lock_guard<std::mutex> lk(g_mu);
        std::vector<Block>& fl = g_free[dev];
        int best = -1;
        for (int i = 0; i < (int)fl.size(); ++i) {
            const Block& b = fl[i];
            // small blocks may serve requests down to half their size;
            // large ones only slightly smaller requests
            const size_t slack = cls > ((size_t)64 << 20) ? cls >> 3 : cls;
            if (b.cap < cls || b.cap > cls + slack) continue;
            if (!b.synced && b.st != st) continue;
            if (best < 0 || b.cap < fl[best].cap) best = i;
        }
        if (best >= 0) {
            *p = fl[best].p;
            g_used[*p] = fl[best].cap;
            fl.erase(fl.begin() + best);
            return hipSuccess;
        }
    }
    hipError_t e = hipMalloc(p, cls);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        // give every cached block back and try once more
        dev_cache_trim();
        e = hipMalloc(p, cls);
        if (e != hipSuccess) {
            *p = nullptr;
            return e;
        }
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_used[*p] = cls;
    return hipSuccess;
}

void dev_cache_trim() {
    const int dev = device_index();
    std::vector<Block> drop;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        drop.swap(g_free[dev]);
    }
    if (drop.empty()) return;
    // blocks released on a stream may still be in use by its queued work
    (void)hipDeviceSynchronize();
    for (const Block& b : drop) (void)hipFree(b.p);
}

// While a capture is being recorded on this thread, released blocks are kept
// by the capture's owner: the recorded work reuses them at every replay.
static thread_local std::vector<std::pair<void*, hipStream_t>>* t_defer = nullptr;

void dev_defer_begin(std::vector<std::pair<void*, hipStream_t>>* keep) { t_defer = keep; }
void dev_defer_end() { t_defer = nullptr; }

hipError_t dev_free(void* p, hipStream_t st) {
    if (!p) return hipSuccess;
    if (t_defer) {
        t_defer->push_back({p, st});
        return hipSuccess;
    }
    const int dev = device_index();
    std::unique_lock<std::mutex> lk(g_mu);
    auto ut = g_user.find(p);
    if (ut != g_user.end()) {
        const UserBlock b = ut->second;
        g_user.erase(ut);
        lk.unlock();
        b.a.free(b.a.ctx, p, b.bytes, st);
        return hipSuccess;
    }
    auto it = g_used.find(p);
    if (it == g_used.end()) return hipErrorInvalidValue;
    g_free[dev].push_back(Block{p, it->second, st, false});
    g_used.erase(it);
    return hipSuccess;
}

void dev_stream_synced(hipStream_t st) {
    const int dev = device_index();
    std::lock_guard<std::mutex> lk(g_mu);
    for (Block& b : g_free[dev])
        if (b.st == st) b.synced = true;
}

hipError_t sync_stream(hipStream_t st) {
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess) dev_stream_synced(st);
    return e;
}

void* host_stage_acquire() {
    {
        std::lock_guard<std::mutex> lk(g_stage_mu);
        if (!g_stage_free.empty()) {
            void* p = g_stage_free.back();
            g_stage_free.pop_back();
            return p;
        }
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, kHostStageBytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void host_stage_release(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_stage_mu);
    g_stage_free.push_back(p);
}

hipError_t read_back(const HostRead* r, int n, hipStream_t st) {
    size_t total = 0;
    for (int i = 0; i < n; ++i) total += (r[i].bytes + 15) & ~(size_t)15;
    unsigned char* stage = total <= kHostStageBytes ? static_cast<unsigned char*>(host_stage_acquire()) : nullptr;
    hipError_t e = hipSuccess;
    size_t off = 0;
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        if (r[i].bytes == 0) continue;
        e = hipMemcpyAsync(stage ? stage + off : r[i].host, r[i].dev, r[i].bytes, hipMemcpyDeviceToHost, st);
        off += (r[i].bytes + 15) & ~(size_t)15;
    }
    // the stream is waited for also after a failed enqueue: no copy into the
    // staging block may still be in flight when it goes back to the list
    const hipError_t es = sync_stream(st);
    if (e == hipSuccess) e = es;
    if (stage) {
        off = 0;
        for (int i = 0; i < n && e == hipSuccess; ++i) {
            if (r[i].bytes) std::memcpy(r[i].host, stage + off, r[i].bytes);
            off += (r[i].bytes + 15) & ~(size_t)15;
        }
        host_stage_release(stage);
    }
    return e;
}

hipEvent_t timing_event_acquire(int* dev) {
    *dev = device_index();
    {
        std::lock_guard<std::mutex> lk(g_ev_mu);
        std::vector<hipEvent_t>& fl = g_ev_free[*dev];
        if (!fl.empty()) {
            hipEvent_t e = fl.back();
            fl.pop_back();
            return e;
        }
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

void timing_event_release(hipEvent_t e, int dev) {
    if (!e) return;
    std::lock_guard<std::mutex> lk(g_ev_mu);
    g_ev_free[dev].push_back(e);
}
