// Host runtime of the C ABI in include/gsofa.h: input checks, planning of
// concurrent sources against the device-memory budget, the device memory
// cache, the fill-detection -> assembly -> supernode pipeline for one or many
// matrices, result ownership, and the request server.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "gsofa.h"
#include "gsofa_internal.h"

namespace gsofa {
namespace {

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct HipError {
    hipError_t e;
};

inline void chk(hipError_t e) {
    if (e != hipSuccess) throw HipError{e};
}

struct Status {
    int code;
};

// ------------------------------------------------------ device memory cache
//
// Freed blocks stay cached for later calls. A block is freed while work on its
// stream may still read or write it, so the release records an event on that
// stream and the block is handed out again only on the same stream (stream
// order protects it) or once the event has completed. Engine calls run on one
// stream per thread; t_stream names it.

thread_local hipStream_t t_stream = nullptr;
// Set once a call has synchronised with t_stream for the last time: buffers
// released after that point need no completion event.
thread_local bool t_idle = false;

struct StreamScope {
    hipStream_t prev;
    bool prev_idle;
    explicit StreamScope(hipStream_t s) : prev(t_stream), prev_idle(t_idle) {
        t_stream = s;
        t_idle = false;
    }
    ~StreamScope() {
        t_stream = prev;
        t_idle = prev_idle;
    }
};

void drop_idle_slots();

// process-wide device-memory counters (gsofa_memory_counters)
std::atomic<uint64_t> g_hip_bytes_held{0}, g_hip_mallocs{0}, g_caller_bytes{0}, g_caller_allocs{0},
    g_caller_frees{0};

class DevCache {
   public:
    void* alloc(size_t bytes, hipStream_t st) {
        if (bytes == 0) bytes = 256;
        bytes = (bytes + 255) & ~size_t(255);
        {
            std::lock_guard<std::mutex> g(mu_);
            const size_t limit = bytes * 2 + (64ull << 20);
            for (auto it = free_.lower_bound(bytes); it != free_.end() && it->first <= limit; ++it) {
                Blk& b = it->second;
                const bool ready = b.ev == nullptr || b.st == st || hipEventQuery(b.ev) == hipSuccess;
                if (!ready) continue;
                void* p = b.p;
                if (b.ev) (void)hipEventDestroy(b.ev);
                used_[p] = it->first;
                free_.erase(it);
                return p;
            }
        }
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, bytes);
        g_hip_mallocs.fetch_add(1);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            drop_idle_slots();
            release();
            e = hipMalloc(&p, bytes);
            g_hip_mallocs.fetch_add(1);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                throw Status{GSOFA_ENOMEM};
            }
        }
        g_hip_bytes_held.fetch_add(bytes);
        std::lock_guard<std::mutex> g(mu_);
        used_[p] = bytes;
        return p;
    }
    // synced: no work on the block can still be pending
    void free(void* p, hipStream_t st, bool synced) {
        if (!p) return;
        hipEvent_t ev = nullptr;
        if (!synced) {
            if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
                hipEventRecord(ev, st) != hipSuccess) {
                (void)hipGetLastError();
                if (ev) (void)hipEventDestroy(ev);
                ev = nullptr;
                (void)hipStreamSynchronize(st);
                (void)hipGetLastError();
            }
        }
        std::lock_guard<std::mutex> g(mu_);
        auto it = used_.find(p);
        if (it == used_.end()) {
            if (ev) (void)hipEventDestroy(ev);
            return;
        }
        free_.emplace(it->second, Blk{p, st, ev});
        used_.erase(it);
    }
    // bytes held in idle cached blocks (handed back to the device on pressure)
    size_t idle_bytes() {
        std::lock_guard<std::mutex> g(mu_);
        size_t t = 0;
        for (auto& kv : free_) t += kv.first;
        return t;
    }
    void release() {
        std::lock_guard<std::mutex> g(mu_);
        for (auto& kv : free_) {
            if (kv.second.ev) {
                (void)hipEventSynchronize(kv.second.ev);
                (void)hipEventDestroy(kv.second.ev);
            }
            (void)hipFree(kv.second.p);
            g_hip_bytes_held.fetch_sub(kv.first);
        }
        free_.clear();
        (void)hipGetLastError();
    }

   private:
    struct Blk {
        void* p;
        hipStream_t st;
        hipEvent_t ev;  // completes when the last work on the block is done; null: idle
    };
    std::mutex mu_;
    std::multimap<size_t, Blk> free_;
    std::unordered_map<void*, size_t> used_;
};

DevCache& cache() {
    static DevCache* c = new DevCache();  // lives until process end
    return *c;
}

// The caller's device allocator of one call (gsofa_opts dev_alloc / dev_free).
// Buffers released while the call's device work may still use them are kept
// until flush(), which runs once that work has completed.
struct CallerAlloc {
    gsofa_alloc_fn alloc_fn = nullptr;
    gsofa_free_fn free_fn = nullptr;
    void* ctx = nullptr;
    std::mutex mu;
    std::vector<void*> deferred;

    void* take(size_t bytes) {
        bytes = (bytes + 255) & ~size_t(255);
        void* p = alloc_fn(bytes, ctx);
        if (!p) throw Status{GSOFA_ENOMEM};
        g_caller_allocs.fetch_add(1);
        g_caller_bytes.fetch_add(bytes);
        if (reinterpret_cast<uintptr_t>(p) & 255u) {
            give(p);
            throw Status{GSOFA_EINVAL};  // the allocator must align to 256 bytes
        }
        return p;
    }
    void give(void* p) {
        free_fn(p, ctx);
        g_caller_frees.fetch_add(1);
    }
    // idle: no device work can still use the buffer
    void release(void* p, bool idle) {
        if (idle) {
            give(p);
            return;
        }
        std::lock_guard<std::mutex> g(mu);
        deferred.push_back(p);
    }
    void flush() {
        std::vector<void*> v;
        {
            std::lock_guard<std::mutex> g(mu);
            v.swap(deferred);
        }
        for (void* p : v) give(p);
    }
};

// Set for the length of a call that brought its own allocator.
thread_local std::shared_ptr<CallerAlloc> t_calloc;

// A device buffer taken from the caller's allocator when the call brought one,
// else from the cache on the calling thread's engine stream, returned with that
// stream's ordering on destruction.
struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipStream_t st = nullptr;
    bool synced = false;  // set once no work on the buffer can be pending
    std::shared_ptr<CallerAlloc> ca;
    DBuf() = default;
    explicit DBuf(size_t b) : bytes(b), st(t_stream), ca(t_calloc) {
        p = ca ? ca->take(b) : cache().alloc(b, t_stream);
    }
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    DBuf(DBuf&& o) noexcept : p(o.p), bytes(o.bytes), st(o.st), synced(o.synced), ca(std::move(o.ca)) {
        o.p = nullptr;
    }
    DBuf& operator=(DBuf&& o) noexcept {
        if (this != &o) {
            reset();
            p = o.p;
            bytes = o.bytes;
            st = o.st;
            synced = o.synced;
            ca = std::move(o.ca);
            o.p = nullptr;
        }
        return *this;
    }
    ~DBuf() { reset(); }
    void reset() {
        if (p) {
            const bool idle = synced || (t_idle && st == t_stream);
            if (ca) ca->release(p, idle);
            else cache().free(p, st, idle);
        }
        p = nullptr;
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

// Pinned host memory for uploads, staging and small reads inside a call,
// pooled across calls (pinning pages is slow). A block goes back to the pool
// only once its call's stream is idle; on an error path the release waits for
// the stream first.
class PinnedPool {
   public:
    void* take(size_t bytes) {
        bytes = (bytes + 4095) & ~size_t(4095);
        {
            std::lock_guard<std::mutex> g(mu_);
            auto it = free_.lower_bound(bytes);
            if (it != free_.end() && it->first <= bytes * 2 + (1u << 20)) {
                void* p = it->second;
                size_[p] = it->first;
                pooled_ -= it->first;
                free_.erase(it);
                return p;
            }
        }
        void* p = nullptr;
        chk(hipHostMalloc(&p, bytes, hipHostMallocDefault));
        std::lock_guard<std::mutex> g(mu_);
        size_[p] = bytes;
        return p;
    }
    void give(void* p) {
        if (!t_idle) {
            (void)hipStreamSynchronize(t_stream);
            (void)hipGetLastError();
        }
        std::lock_guard<std::mutex> g(mu_);
        auto it = size_.find(p);
        if (it == size_.end()) return;
        const size_t b = it->second;
        size_.erase(it);
        // keep at most 512 MiB pinned between calls
        if (pooled_ + b > (512ull << 20)) {
            (void)hipHostFree(p);
            return;
        }
        free_.emplace(b, p);
        pooled_ += b;
    }

   private:
    std::mutex mu_;
    std::multimap<size_t, void*> free_;
    std::unordered_map<void*, size_t> size_;
    size_t pooled_ = 0;
};

PinnedPool& pinned_pool() {
    static PinnedPool* p = new PinnedPool();  // lives until process end
    return *p;
}

// Pinned host memory for the worklist / row-buffer overflow of memory-budget
// mode: one block kept between calls (pinning tens of GB takes seconds), owned
// by one call at a time; a call that finds it taken or too small pins its own,
// and the larger of the two stays cached.
class SpillCache {
   public:
    struct Block {
        void* p = nullptr;
        size_t bytes = 0;
    };
    Block take(size_t bytes) {
        {
            std::lock_guard<std::mutex> g(mu_);
            if (cached_.p && cached_.bytes >= bytes) {
                Block b = cached_;
                cached_ = Block{};
                return b;
            }
        }
        Block b;
        b.bytes = (bytes + 4095) & ~size_t(4095);
        chk(hipHostMalloc(&b.p, b.bytes, hipHostMallocDefault));
        return b;
    }
    void give(Block b) {
        if (!b.p) return;
        Block drop;
        {
            std::lock_guard<std::mutex> g(mu_);
            if (!cached_.p || cached_.bytes < b.bytes) {
                drop = cached_;
                cached_ = b;
            } else {
                drop = b;
            }
        }
        if (drop.p) (void)hipHostFree(drop.p);
    }
    void release() {
        Block drop;
        {
            std::lock_guard<std::mutex> g(mu_);
            drop = cached_;
            cached_ = Block{};
        }
        if (drop.p) (void)hipHostFree(drop.p);
    }

   private:
    std::mutex mu_;
    Block cached_;
};

SpillCache& spill_cache() {
    static SpillCache* c = new SpillCache();  // lives until process end
    return *c;
}

// Host memory for results. A result lands in page-locked memory, written by
// the library's copy kernel at the link's rate (690 MB in 13 ms), where fresh
// pageable memory takes 200 ms per 800 MB (each page faults in during the
// copy, and the runtime stages it through its own kernels). Freeing
// page-locked memory waits for all work on the device, so released blocks are
// kept for later results (best fit within twice the size), up to
// kResultIdleMax bytes; only beyond that does a release free, and wait. Where
// no page-locked memory is left, a block comes from malloc, and so does a
// result below kResultPinnedMin bytes (many small results kept by a caller
// would otherwise lock memory by the 64 KiB block).
constexpr size_t kResultIdleMax = 8ull << 30;
constexpr size_t kResultPinnedMin = 1u << 20;

class ResultBlocks {
   public:
    struct Block {
        void* p = nullptr;
        bool pinned = false;
    };
    Block take(size_t bytes) {
        if (bytes < kResultPinnedMin) return {std::malloc(bytes), false};
        bytes = (bytes + 65535) & ~size_t(65535);
        {
            std::lock_guard<std::mutex> g(mu_);
            auto it = idle_.lower_bound(bytes);
            if (it != idle_.end() && it->first <= bytes * 2 + (1u << 20)) {
                void* p = it->second;
                size_[p] = it->first;
                pooled_ -= it->first;
                idle_.erase(it);
                return {p, true};
            }
        }
        void* p = nullptr;
        if (hipHostMalloc(&p, bytes, hipHostMallocDefault) == hipSuccess && p) {
            std::lock_guard<std::mutex> g(mu_);
            size_[p] = bytes;
            return {p, true};
        }
        (void)hipGetLastError();
        return {std::malloc(bytes), false};
    }
    // p came from take() as page-locked; the call that filled it has synchronised
    void give(void* p) {
        std::vector<void*> drop;
        {
            std::lock_guard<std::mutex> g(mu_);
            auto it = size_.find(p);
            if (it == size_.end()) return;
            idle_.emplace(it->second, p);
            pooled_ += it->second;
            size_.erase(it);
            while (pooled_ > kResultIdleMax) {
                auto big = std::prev(idle_.end());
                pooled_ -= big->first;
                drop.push_back(big->second);
                idle_.erase(big);
            }
        }
        for (void* q : drop) (void)hipHostFree(q);
    }

   private:
    std::mutex mu_;
    std::multimap<size_t, void*> idle_;
    std::unordered_map<void*, size_t> size_;
    size_t pooled_ = 0;
};

ResultBlocks& result_blocks() {
    static ResultBlocks* r = new ResultBlocks();  // lives until process end
    return *r;
}

struct PinnedBuf {
    void* p = nullptr;
    explicit PinnedBuf(size_t b) : p(pinned_pool().take(std::max<size_t>(b, 8))) {}
    PinnedBuf(const PinnedBuf&) = delete;
    PinnedBuf& operator=(const PinnedBuf&) = delete;
    ~PinnedBuf() {
        if (p) pinned_pool().give(p);
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

// Transfers of a call's small arrays run as copy kernels of this library
// (256-thread workgroups, a few registers each). The runtime copies host and
// device memory with kernels of 512- and 1,024-thread workgroups, which wait
// for a compute unit with that much room, and there is none while persistent
// traversals of other calls hold the device: a 2,000-row server request's
// input upload waited 0.4 s behind two 64^3 traversals. Larger uploads go
// from pinned staging by hipMemcpyAsync, which runs on the copy engine; results
// of any size come back through the copy kernel into page-locked blocks.
constexpr size_t kKernelCopyMax = 8u << 20;

// ------------------------------------------------------------ HIP graphs
//
// The device work of a call between two host synchronisations (a phase) is
// captured on a private stream and replayed as one graph launch on the call's
// stream. Executable graphs are kept per phase and updated in place with the
// next call's launch parameters; a graph whose node structure changed is
// instantiated again. Everything a phase touches is allocated before its
// capture starts and released only after the call has synchronised, and no
// captured phase contains a memset node (buffers are cleared by kernels).

enum PhaseId { kPhaseTraverse = 0, kPhaseScan, kPhaseSort, kPhaseSupernodes, kPhaseColumns, kPhaseCount };

struct GraphPool {
    std::mutex mu;
    std::vector<hipStream_t> streams;  // idle capture streams
    // idle executable graphs: (phase, node count) -> exec
    std::vector<std::pair<std::pair<int, size_t>, hipGraphExec_t>> execs;
    std::vector<hipEvent_t> events;  // idle timing events
};

// Never destroyed: graphs, streams and events must not be released while the
// runtime shuts down at process exit.
GraphPool& graph_pool() {
    static GraphPool* p = new GraphPool();
    return *p;
}

std::atomic<uint64_t> g_graph_instantiations{0}, g_graph_updates{0}, g_graph_launches{0};

class Phase {
  public:
    Phase(int id, bool use_graph, hipStream_t run) : id_(id), graph_(use_graph), run_(run) {
        if (!graph_) return;
        {
            std::lock_guard<std::mutex> g(graph_pool().mu);
            auto& v = graph_pool().streams;
            if (!v.empty()) {
                cap_ = v.back();
                v.pop_back();
            }
        }
        if (!cap_) chk(hipStreamCreateWithFlags(&cap_, hipStreamNonBlocking));
        chk(hipStreamBeginCapture(cap_, hipStreamCaptureModeRelaxed));
        capturing_ = true;
    }
    Phase(const Phase&) = delete;
    Phase& operator=(const Phase&) = delete;

    // stream the phase's work is enqueued on
    hipStream_t stream() const { return graph_ ? cap_ : run_; }

    // end the capture and launch the phase's graph on the call's stream
    void launch() {
        if (!graph_) return;
        hipGraph_t g = nullptr;
        capturing_ = false;
        chk(hipStreamEndCapture(cap_, &g));
        struct GraphGuard {
            hipGraph_t g;
            ~GraphGuard() {
                if (g) (void)hipGraphDestroy(g);
            }
        } gg{g};
        size_t nodes = 0;
        chk(hipGraphGetNodes(g, nullptr, &nodes));
        if (nodes == 0) return;
        key_ = {id_, nodes};
        {
            std::lock_guard<std::mutex> lk(graph_pool().mu);
            auto& v = graph_pool().execs;
            for (size_t i = 0; i < v.size(); ++i)
                if (v[i].first == key_) {
                    exec_ = v[i].second;
                    v.erase(v.begin() + (long)i);
                    break;
                }
        }
        if (exec_) {
            hipGraphNode_t bad = nullptr;
            hipGraphExecUpdateResult res = hipGraphExecUpdateSuccess;
            if (hipGraphExecUpdate(exec_, g, &bad, &res) != hipSuccess || res != hipGraphExecUpdateSuccess) {
                (void)hipGetLastError();
                (void)hipGraphExecDestroy(exec_);
                exec_ = nullptr;
            } else {
                g_graph_updates.fetch_add(1);
            }
        }
        if (!exec_) {
            chk(hipGraphInstantiate(&exec_, g, nullptr, nullptr, 0));
            g_graph_instantiations.fetch_add(1);
        }
        chk(hipGraphLaunch(exec_, run_));
        g_graph_launches.fetch_add(1);
        launched_ = true;
    }

    // the caller has synchronised with the call's stream: the graph is idle
    void done() { finished_ = true; }

    ~Phase() {
        if (capturing_) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(cap_, &g);
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
        }
        if (exec_) {
            if (launched_ && !finished_) (void)hipStreamSynchronize(run_);
            std::lock_guard<std::mutex> lk(graph_pool().mu);
            auto& v = graph_pool().execs;
            v.emplace_back(key_, exec_);
            // bounded: at most 64 idle executable graphs
            if (v.size() > 64) {
                (void)hipGraphExecDestroy(v.front().second);
                v.erase(v.begin());
            }
        }
        if (cap_) {
            std::lock_guard<std::mutex> lk(graph_pool().mu);
            graph_pool().streams.push_back(cap_);
        }
    }

  private:
    int id_;
    bool graph_;
    hipStream_t run_;
    hipStream_t cap_ = nullptr;
    hipGraphExec_t exec_ = nullptr;
    std::pair<int, size_t> key_{-1, 0};
    bool capturing_ = false, launched_ = false, finished_ = false;
};

// Five timing events taken from a process-wide pool for the length of a call.
struct EventSet {
    hipEvent_t e[5] = {};
    EventSet() {
        std::lock_guard<std::mutex> lk(graph_pool().mu);
        auto& v = graph_pool().events;
        for (auto& x : e) {
            if (!v.empty()) {
                x = v.back();
                v.pop_back();
            }
        }
    }
    EventSet(const EventSet&) = delete;
    EventSet& operator=(const EventSet&) = delete;
    hipEvent_t operator[](int i) {
        if (!e[i]) chk(hipEventCreate(&e[i]));
        return e[i];
    }
    ~EventSet() {
        std::lock_guard<std::mutex> lk(graph_pool().mu);
        for (auto x : e)
            if (x) graph_pool().events.push_back(x);
    }
};

// Slot state is kept initialised between calls: every source leaves its
// pending bitmap clear and its labels in a used-up range, so a later call with
// the same layout can start at once.
struct SlotSet {
    DBuf buf;
    SlotLayout lay{};
    int32_t nslots = 0;
    int mode = 0;  // 0: 32-bit labels, 1: byte states
};

std::mutex g_slot_mu;
std::vector<std::unique_ptr<SlotSet>>& idle_slots() {
    static auto* v = new std::vector<std::unique_ptr<SlotSet>>();
    return *v;
}

std::unique_ptr<SlotSet> take_slots(const SlotLayout& lay, int32_t nslots, int mode, hipStream_t st) {
    if (!t_calloc) {
        std::lock_guard<std::mutex> g(g_slot_mu);
        auto& v = idle_slots();
        for (size_t i = 0; i < v.size(); ++i) {
            // a set laid out for up to twice the size serves smaller matrices too,
            // and one with at least 7/8 of the slots asked for is used as it is
            // (the caller runs min(asked, set) sources) rather than reallocated
            if (v[i]->lay.N >= lay.N && v[i]->lay.N <= 2 * lay.N && (int64_t)v[i]->nslots * 8 >= (int64_t)nslots * 7) {
                auto s = std::move(v[i]);
                v.erase(v.begin() + i);
                s->buf.st = st;
                s->buf.synced = false;
                // 32-bit labels left behind do not read as "not reached" bytes
                if (s->mode != mode) chk(launch_init_slots(s->buf.as<uint8_t>(), s->nslots, s->lay, st));
                s->mode = mode;
                return s;
            }
        }
    }
    auto s = std::make_unique<SlotSet>();
    s->buf = DBuf((size_t)lay.bytes_per_slot * nslots);
    s->lay = lay;
    s->nslots = nslots;
    s->mode = mode;
    chk(launch_init_slots(s->buf.as<uint8_t>(), nslots, lay, st));
    return s;
}

// Called once the traversal that used the slots has completed.
void give_slots(std::unique_ptr<SlotSet> s) {
    s->buf.synced = true;
    if (s->buf.ca) return;  // the caller's memory goes straight back
    std::vector<std::unique_ptr<SlotSet>> drop;
    {
        std::lock_guard<std::mutex> g(g_slot_mu);
        auto& v = idle_slots();
        v.push_back(std::move(s));
        // keep the cache bounded: at most 4 idle sets
        while (v.size() > 4) {
            drop.push_back(std::move(v.front()));
            v.erase(v.begin());
        }
    }
}

void drop_idle_slots() {
    std::vector<std::unique_ptr<SlotSet>> drop;
    std::lock_guard<std::mutex> g(g_slot_mu);
    drop.swap(idle_slots());
}

size_t idle_slot_bytes() {
    std::lock_guard<std::mutex> g(g_slot_mu);
    size_t t = 0;
    for (auto& s : idle_slots()) t += s->buf.bytes;
    return t;
}

struct DeviceInfo {
    int cus = 256;
    size_t free_b = 0, total_b = 0;
    size_t reclaimable = 0;  // idle memory this library caches and gives back on demand
};

DeviceInfo device_info() {
    DeviceInfo d;
    int dev = 0;
    chk(hipGetDevice(&dev));
    // compute-unit counts per device, queried once
    static std::mutex mu;
    static std::map<int, int> cus;
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cus.find(dev);
        if (it != cus.end()) d.cus = it->second;
        else {
            int c = 0;
            chk(hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev));
            cus[dev] = d.cus = c;
        }
    }
    chk(hipMemGetInfo(&d.free_b, &d.total_b));
    d.reclaimable = cache().idle_bytes() + idle_slot_bytes();
    return d;
}

// ------------------------------------------------------------ input checks

int check_csr_host(int32_t n, const int32_t* rp, const int32_t* ci, std::vector<uint32_t>& stamp) {
    if (n < 0 || n > GSOFA_MAX_N) return GSOFA_EINVAL;
    if (n == 0) return GSOFA_OK;
    if (!rp || rp[0] != 0) return GSOFA_EINVAL;
    for (int32_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i]) return GSOFA_EINVAL;
    if (rp[n] > 0 && !ci) return GSOFA_EINVAL;
    if ((int64_t)stamp.size() < n) stamp.assign(n, 0u);
    else std::fill(stamp.begin(), stamp.begin() + n, 0u);
    for (int32_t i = 0; i < n; ++i) {
        const uint32_t tag = (uint32_t)i + 1u;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            const int32_t c = ci[e];
            if (c < 0 || c >= n) return GSOFA_EINVAL;
            if (stamp[c] == tag) return GSOFA_EINVAL;  // repeated column
            stamp[c] = tag;
        }
    }
    return GSOFA_OK;
}

// ------------------------------------------------------------------ results

struct ResultOwner {
    // the host block or the device buffers shared by the results of one call
    std::shared_ptr<void> shared_host;
    std::shared_ptr<std::vector<DBuf>> dev;
};

gsofa_result* new_result() {
    auto* r = static_cast<gsofa_result*>(std::calloc(1, sizeof(gsofa_result)));
    if (!r) throw Status{GSOFA_ENOMEM};
    r->internal_ = new ResultOwner();
    return r;
}

// ------------------------------------------------------------ the pipeline

struct MatIn {
    int32_t n;
    const int32_t* rp;
    const int32_t* ci;
};

// Largest order of a one-matrix call that launches its phases eagerly.
constexpr int64_t kEagerMaxRows = 65536;

// Calls with fewer sources are latency-bound and use the defaults untuned.
constexpr int64_t kTuneMinSources = 65536;
// Memory-budget mode: pinned host memory for worklist and row-buffer overflow,
// at most this much per band (it bounds the sources in flight as well).
constexpr int64_t kSpillHostBytes = int64_t(32) << 30;

struct Plan {
    int32_t window;
    int32_t nslots;
    int32_t max_super;  // <= 0: unbounded
    uint32_t flags;
    int64_t budget;
    int32_t queue_cap;  // memory-budget mode: device entries per worklist and row buffer
    int32_t slot_div;   // the tuner's choice of sources in flight: planned count / slot_div
    bool window_auto;   // window span, mapping and sources in flight are the tuner's
    bool allow_trials;  // the tuner may time trial launches in this call
};

// Traversal mapping. One wavefront per source with 32-bit labels is the
// default: per-source frontiers are small (a window holds a few dozen
// vertices), so a workgroup per source leaves most of its wavefronts idle and
// was 3-5x slower on the 64^3 and 1000^2 stencils, and byte states were 1.5x
// slower on the 64^3 stencil (byte updates need compare-and-swap loops). The
// others stay available as tuning knobs and tuner candidates. Byte states
// (mapping 3) need windows of at most 253 ids and keep no label for vertices
// already in the structure, so the paper's order (window = n) and the
// line-9.5-off ablation always run on 32-bit labels.
int choose_mapping(uint32_t flags, int32_t window) {
    if (flags & GSOFA_BUDGET_MODE) return 5;
    if (flags & GSOFA_MAP_THREAD) return 6;
    if (flags & GSOFA_MAP_WG16) return 1;
    if (flags & GSOFA_MAP_WG8) return 2;
    if (flags & GSOFA_MAP_WAVE32) return 0;
    if (flags & GSOFA_MAP_WAVE32_7) return 4;
    const bool ablation = window > 253 || (flags & (GSOFA_NO_LINE95 | GSOFA_LEVEL_ORDER));
    if ((flags & GSOFA_MAP_BYTE) && !ablation) return 3;
    return 0;
}

int32_t auto_window(int64_t sources) {
    // Window span for the traversal schedule. Small spans keep revisits low,
    // wider ones need fewer levels. A call with many sources is bound by
    // throughput, and 16 was best on the 64^3 and 1000^2 stencils and on the
    // 4,096-matrix batch; a call with few sources is bound by the latency of
    // its longest source, and 64 was best for single matrices of a few
    // thousand rows (2.3 ms against 3.4 ms at 16).
    return sources >= kTuneMinSources ? 16 : 64;
}

// ------------------------------------------------------------ autotuner
//
// Window span and traversal mapping change only the speed, never the result.
// For a size class that has not been seen yet (device, log2 of the largest n,
// mean row length, batch size) and a call with enough sources, the tuner times
// every candidate on a stratified sample of the call's sources
// (kTuneScreenPerSlot per slot), times the kTuneFinalists fastest again on a
// larger one (kTuneSamplesPerSlot per slot), keeps the fastest of those, and
// reuses it for later calls of the class. Smaller calls use the defaults.
// Sources in flight enter only as all resident wavefronts or half of them,
// both with the same number of sources per slot: on a sample a few sources per
// slot long, fewer slots win by balancing the tail better, while at full size
// they were twice as slow.

struct TuneKey {
    int cus, n_log2, deg_bucket, batch_log2;
    bool operator<(const TuneKey& o) const {
        return std::tie(cus, n_log2, deg_bucket, batch_log2) < std::tie(o.cus, o.n_log2, o.deg_bucket, o.batch_log2);
    }
};

struct TuneChoice {
    int mapping;     // 0 32-bit labels (eight wavefronts per SIMD), 4 the same at seven, 3 byte states
    int32_t window;  // threshold-window span
    uint32_t flags;  // extra flags: GSOFA_NO_LINE95 (the access-order check switched off)
    int32_t div;     // sources in flight: the planned count divided by div (#C)
};

constexpr TuneChoice kTuneCandidates[] = {
    // order is a prior: a later candidate replaces the best only if 5 % faster.
    // Seven wavefronts per SIMD with window 8 comes second: where window 8 wins
    // clearly (the 1000^2 9-point stencil) it also wins at seven by ~4 %, which
    // the margin would hide if it came after window 8 at eight. Windows 4 and 2
    // cut revisits on 2D stencils (1.31x edges at window 8, 1.12x at 4, 1.03x
    // at 2 on the 1000^2 9-point stencil; 249 -> 216 ms at 4). The last four
    // are the paper's other two ablations as tuner dimensions: line 9.5 off
    // (Section 4, access-order paragraph) and half the sources in flight
    // (#C, the chunk-size study of the Evaluation section).
    {0, 16, 0, 1}, {4, 8, 0, 1}, {0, 32, 0, 1}, {0, 64, 0, 1}, {0, 8, 0, 1}, {4, 16, 0, 1}, {3, 16, 0, 1},
    {0, 4, 0, 1}, {0, 2, 0, 1}, {4, 4, 0, 1},
    {0, 16, GSOFA_NO_LINE95, 1}, {4, 8, GSOFA_NO_LINE95, 1}, {0, 16, 0, 2}, {4, 8, 0, 2},
};
constexpr int kTuneSamplesPerSlot = 24;  // final sample: sources per slot
constexpr int kTuneScreenPerSlot = 8;    // first (screening) sample
constexpr int kTuneFinalists = 3;        // candidates timed on the final sample

std::mutex g_tune_mu;
std::map<TuneKey, TuneChoice>& tune_table() {
    static auto* t = new std::map<TuneKey, TuneChoice>();
    return *t;
}

// sources in flight divided by d, in whole blocks of four wavefronts
int64_t div_slots(int64_t ns, int32_t d) {
    if (d <= 1) return ns;
    int64_t r = ns / d;
    if (r > 4) r = r / 4 * 4;
    return std::max<int64_t>(r, 1);
}

int ceil_log2(int64_t v) {
    int b = 0;
    while (b < 62 && (int64_t(1) << b) < v) ++b;
    return b;
}

struct EngineOut {
    int status = GSOFA_OK;
    std::vector<int> job_status;
};

// Per-launch fill-ratio memory used to size the output pool of later calls.
std::atomic<double> g_fill_ratio{48.0};
// The same per size class (the tuner's key): a batch of small 3D stencils fills
// more per stored entry than a large 2D stencil, and a pool sized from the other
// class's ratio overflowed and cost a second traversal pass (418 ms on the
// 4,096-matrix batch after the 1000^2 stencil).
std::mutex g_fill_mu;
std::map<TuneKey, double>& fill_ratios() {
    static auto* m = new std::map<TuneKey, double>();
    return *m;
}
double fill_ratio_for(const TuneKey& k) {
    std::lock_guard<std::mutex> g(g_fill_mu);
    auto it = fill_ratios().find(k);
    return it != fill_ratios().end() ? it->second : 48.0;
}
void note_fill_ratio(const TuneKey& k, double r) {
    std::lock_guard<std::mutex> g(g_fill_mu);
    fill_ratios()[k] = r;
    g_fill_ratio.store(r);
}

// Device bytes a launch needs besides slots and output pool: inputs, per-row
// arrays, assembly buffers, scratch.
int64_t fixed_bytes(int64_t nrows, int64_t nnz) { return nrows * 40 + nnz * 8 + (64ll << 20); }

// Output-pool entries expected for nnz stored entries.
int64_t pool_estimate(int64_t nrows, int64_t nnz, double ratio = -1.0) {
    if (ratio <= 0) ratio = g_fill_ratio.load();
    return std::max<int64_t>((int64_t)(ratio * (double)nnz * 1.15) + nrows, 1 << 20);
}

// Budget under which the planner below gives nslots slots and the expected
// pool: half of the room after fixed_bytes goes to slots, and the pool may
// take up to a third of the rest in 4-byte entries.
int64_t budget_for(int64_t nrows, int64_t nnz, int64_t nslots, const SlotLayout& lay) {
    return fixed_bytes(nrows, nnz) + 2 * nslots * lay.bytes_per_slot + 12 * pool_estimate(nrows, nnz);
}

// out[j] = row_ptr_j[n_j]: the entry count of every matrix of a batch.
__global__ void k_gather_last(int32_t njobs, const Job* jobs, int64_t* out) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= njobs) return;
    out[j] = jobs[j].n > 0 ? (int64_t)jobs[j].row_ptr[jobs[j].n] : 0;
}

// out[j] = a[job_row_base[j]] for j < njobs, out[njobs] = a[nrows]: the values
// of a global pointer array at the matrix boundaries.
__global__ void k_gather_bounds(int32_t njobs, const int64_t* job_row_base, int64_t nrows, const int64_t* a,
                                int64_t* out) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > njobs) return;
    out[j] = a[j < njobs ? job_row_base[j] : nrows];
}

__global__ void k_rebase_ptr(int32_t njobs, const int64_t* job_row_base, const int32_t* job_n,
                             const int64_t* g, int64_t* out) {
    // out[row_base_j + j + i] = g[row_base_j + i] - g[row_base_j], i in [0, n_j]
    const int32_t j = blockIdx.y;
    if (j >= njobs) return;
    const int64_t b = job_row_base[j];
    const int64_t g0 = g[b];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= job_n[j];
         i += (int64_t)gridDim.x * blockDim.x)
        out[b + j + i] = g[b + i] - g0;
}

// A served request's link to the server's work-item admission. The traversal
// launches poll `flag` (fine-grained host memory) before each work item; the
// server sets it when it admits another request onto a full device, the launch
// then stops taking items, and the engine relaunches from the work counter once
// `before_resume` returns (the admitted request's traversal is enqueued by
// then, or a bounded wait has passed). `enqueued` runs once the first traversal
// launch of the call is on the stream, `finished` once the traversal is done.
// `before_traverse` runs before the traversal is enqueued (the call's uploads
// and sorts are on the stream by then) and may wait.
struct YieldHooks {
    uint32_t* flag = nullptr;
    std::function<void()> enqueued, finished, before_resume, before_traverse;
};

struct Engine {
    std::vector<MatIn> mats;
    bool on_device = false;
    gsofa_opts o{};
    Plan plan{};
    hipStream_t st = nullptr;
    const YieldHooks* yh = nullptr;  // server requests only

    // outputs
    std::vector<gsofa_result*> results;

    int run() {
        const double t0 = now_ms();
        StreamScope scope(st);
        // staging blocks of this call's uploads; released (after the stream is
        // idle) when the call ends
        std::vector<std::unique_ptr<PinnedBuf>> staged;
        auto h2d = [&](void* dst, const void* src, size_t bytes, hipStream_t s, bool src_pinned) {
            if (bytes == 0) return;
            if (bytes > kKernelCopyMax || bytes % 4 != 0) {
                chk(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
                return;
            }
            if (!src_pinned) {
                staged.push_back(std::make_unique<PinnedBuf>(bytes));
                std::memcpy(staged.back()->p, src, bytes);
                src = staged.back()->p;
            }
            chk(launch_copy_from_host(dst, src, bytes, s));
        };
        const int32_t nj = (int32_t)mats.size();
        results.assign(nj, nullptr);
        std::vector<int> jstat(nj, GSOFA_OK);

        // ---- inputs to the device
        std::vector<int64_t> nnz(nj, 0);
        std::vector<int64_t> row_base(nj, 0);
        int64_t nrows = 0, total_nnz = 0, N = 1;
        for (int32_t j = 0; j < nj; ++j) {
            row_base[j] = nrows;
            nrows += mats[j].n;
            N = std::max<int64_t>(N, mats[j].n);
        }
        std::vector<Job> jobs(nj);
        DBuf in_rp, in_ci;
        if (on_device) {
            // every matrix's entry count (row_ptr[n]) in one gather and one copy
            for (int32_t j = 0; j < nj; ++j) {
                jobs[j].row_ptr = mats[j].rp;
                jobs[j].col_idx = mats[j].ci;
                jobs[j].n = mats[j].n;
            }
            DBuf d_tab(sizeof(Job) * std::max(nj, 1)), d_last(8 * std::max(nj, 1));
            PinnedBuf h_last(8 * std::max(nj, 1));
            h2d(d_tab.p, jobs.data(), sizeof(Job) * nj, st, false);
            if (nj > 0)
                hipLaunchKernelGGL(k_gather_last, dim3((nj + 255) / 256), dim3(256), 0, st, nj, d_tab.as<Job>(),
                                   d_last.as<int64_t>());
            chk(hipGetLastError());
            chk(launch_copy_to_host(h_last.p, d_last.p, 8 * nj, st));
            chk(hipStreamSynchronize(st));
            for (int32_t j = 0; j < nj; ++j) {
                const int64_t last = h_last.as<int64_t>()[j];
                // a negative count, or entries with no column array, is malformed
                if (last < 0 || (last > 0 && !mats[j].ci)) jstat[j] = GSOFA_EINVAL;
                nnz[j] = std::max<int64_t>(last, 0);
            }
            // nothing may read such a matrix's arrays: fail before the validation kernel
            for (int32_t j = 0; j < nj; ++j)
                if (jstat[j] != GSOFA_OK) return finish_failed(jstat, t0);
        } else {
            std::vector<int64_t> rp_off(nj), ci_off(nj);
            int64_t rp_tot = 0, ci_tot = 0;
            for (int32_t j = 0; j < nj; ++j) {
                nnz[j] = mats[j].n > 0 ? mats[j].rp[mats[j].n] : 0;
                rp_off[j] = rp_tot;
                ci_off[j] = ci_tot;
                rp_tot += mats[j].n + 1;
                ci_tot += nnz[j];
            }
            in_rp = DBuf(4 * (size_t)std::max<int64_t>(rp_tot, 1));
            in_ci = DBuf(4 * (size_t)std::max<int64_t>(ci_tot, 1));
            // pack through a pinned staging buffer, kept to the end of the call
            // (its copies complete by the traversal's synchronisation)
            const size_t stage_b = 4 * (size_t)(rp_tot + ci_tot);
            staged.push_back(std::make_unique<PinnedBuf>(std::max<size_t>(stage_b, 4)));
            int32_t* sp = staged.back()->as<int32_t>();
            for (int32_t j = 0; j < nj; ++j) {
                if (mats[j].n > 0) {
                    std::memcpy(sp + rp_off[j], mats[j].rp, 4 * (size_t)(mats[j].n + 1));
                    if (nnz[j] > 0) std::memcpy(sp + rp_tot + ci_off[j], mats[j].ci, 4 * (size_t)nnz[j]);
                } else {
                    sp[rp_off[j]] = 0;
                }
            }
            h2d(in_rp.p, sp, 4 * (size_t)rp_tot, st, true);
            h2d(in_ci.p, sp + rp_tot, 4 * (size_t)ci_tot, st, true);
            for (int32_t j = 0; j < nj; ++j) {
                jobs[j].row_ptr = in_rp.as<int32_t>() + rp_off[j];
                jobs[j].col_idx = in_ci.as<int32_t>() + ci_off[j];
            }
        }
        for (int32_t j = 0; j < nj; ++j) total_nnz += nnz[j];

        // work order: larger matrices first; inside a matrix, larger row ids first
        std::vector<int32_t> ord(nj);
        for (int32_t j = 0; j < nj; ++j) ord[j] = j;
        std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return mats[a].n > mats[b].n; });
        // the kernel maps items to jobs by item_base, so the job table is in work order
        std::vector<Job> jt(nj);
        std::vector<int32_t> jt_of(nj);  // job-table index of matrix j
        int64_t items = 0;
        for (int32_t q = 0; q < nj; ++q) {
            const int32_t j = ord[q];
            jt[q] = jobs[j];
            jt[q].n = mats[j].n;
            jt[q].row_base = row_base[j];
            jt[q].item_base = items;
            jt_of[j] = q;
            items += mats[j].n;
        }
        DBuf d_jobs(sizeof(Job) * std::max(nj, 1));
        h2d(d_jobs.p, jt.data(), sizeof(Job) * nj, st, false);

        if (on_device) {
            DBuf bad(4 * std::max(nj, 1));
            chk(launch_zero_i32(bad.as<int32_t>(), nj, st));
            chk(launch_validate(d_jobs.as<Job>(), nj, N, bad.as<int32_t>(), st));
            PinnedBuf h_bad(4 * (size_t)std::max(nj, 1));
            chk(launch_copy_to_host(h_bad.p, bad.p, 4 * (size_t)nj, st));
            chk(hipStreamSynchronize(st));
            const int32_t* hb = h_bad.as<int32_t>();
            for (int32_t q = 0; q < nj; ++q)
                if (hb[q]) jstat[ord[q]] = GSOFA_EINVAL;
            bool any_bad = false;
            for (int32_t j = 0; j < nj; ++j) any_bad |= jstat[j] != GSOFA_OK;
            if (any_bad) return finish_failed(jstat, t0);
        }

        // ---- plan the concurrent sources
        const SlotLayout lay = slot_layout(N);
        const DeviceInfo di = device_info();
        // default budget: free device memory plus what this library holds idle
        int64_t budget = plan.budget > 0 ? plan.budget : (int64_t)((di.free_b + di.reclaimable) * 0.9);
        const int64_t fixed = fixed_bytes(nrows, total_nnz);
        // memory-budget mode: the budget caps the source-slot state alone (the
        // paper's shared arena of frontier queues, labels and stamps); inputs,
        // per-row arrays and the output are outside it
        const bool budget_mode = (plan.flags & GSOFA_BUDGET_MODE) != 0;
        if (!budget_mode && budget < fixed + lay.bytes_per_slot) throw Status{GSOFA_ENOMEM};
        const int64_t slot_fit = budget_mode ? 1 : std::max<int64_t>((budget - fixed) / 2 / lay.bytes_per_slot, 1);
        // sources in flight for a mapping: the resident wavefronts (or blocks),
        // within half of the memory left after the fixed part
        auto plan_slots = [&](int map) {
            // every resident slot, but at most 16 GiB of label arrays in flight:
            // the 64^3 stencil (1 MB per source) is fastest with all resident
            // slots (8,192), the 1000^2 stencil (4 MB per source) gained nothing
            // beyond 4,096
            int64_t want = plan.nslots > 0 ? plan.nslots : (int64_t)traverse_resident_slots(di.cus, map);
            if (plan.nslots <= 0 && (map == 0 || map == 3 || map == 4 || map == 6))
                want = std::min<int64_t>(want, std::max<int64_t>(1024, (int64_t(16) << 30) / (4 * N)));
            want = std::min<int64_t>(want, std::max<int64_t>(items, 1));
            int64_t ns = std::max<int64_t>(std::min<int64_t>(want, slot_fit), 1);
            // coarse steps, so that small budget changes between calls keep the
            // cached slot set; the one-wavefront mappings launch whole blocks of 4
            if (plan.nslots <= 0 && ns > 1024) ns = ns / 256 * 256;
            if ((map == 0 || map == 3 || map == 4) && ns > 4) ns = ns / 4 * 4;
            return ns;
        };
        int mapping = choose_mapping(plan.flags, plan.window);
        double t_tune = 0;
        const TuneKey key{di.cus, ceil_log2(N), ceil_log2(std::max<int64_t>(total_nnz * 4 / std::max<int64_t>(nrows, 1), 1)),
                          nj > 1 ? ceil_log2(nj) : 0};
        const double fill_ratio = fill_ratio_for(key);
        if (plan.window_auto) {
            bool found = false;
            {
                std::lock_guard<std::mutex> lk(g_tune_mu);
                auto it = tune_table().find(key);
                if (it != tune_table().end()) {
                    mapping = it->second.mapping;
                    plan.window = it->second.window;
                    plan.flags |= it->second.flags;
                    plan.slot_div = plan.nslots > 0 ? 1 : it->second.div;
                    found = true;
                }
            }
            const bool force = (plan.flags & GSOFA_TUNE_NOW) != 0;
            if ((!found || force) && plan.allow_trials && (items >= kTuneMinSources || force)) {
                const double tt0 = now_ms();
                const TuneChoice c = tune(jt, nj, N, items, lay, budget, fixed, total_nnz, nrows, d_jobs, plan_slots);
                t_tune = now_ms() - tt0;
                mapping = c.mapping;
                plan.window = c.window;
                plan.flags = (plan.flags & ~(uint32_t)GSOFA_NO_LINE95) | c.flags;
                plan.slot_div = c.div;
                std::lock_guard<std::mutex> lk(g_tune_mu);
                tune_table()[key] = c;
            }
        }
        const int64_t nslots = budget_mode ? 0 : div_slots(plan_slots(mapping), plan.slot_div);

        int64_t pool_cap = pool_estimate(nrows, total_nnz, fill_ratio);
        if (!budget_mode) {
            const int64_t pool_room = (budget - fixed - nslots * lay.bytes_per_slot) / 4 / 3;
            pool_cap = std::max<int64_t>(std::min<int64_t>(pool_cap, pool_room), nrows + 1024);
        }

        // slot modes: 0 32-bit labels, 1 byte states, 2 visit stamps of the
        // one-thread-per-source kernel (a different mode re-initialises a set)
        std::unique_ptr<SlotSet> slots;
        if (!budget_mode) slots = take_slots(lay, (int32_t)nslots, mapping == 3 ? 1 : mapping == 6 ? 2 : 0, st);
        // a call on one small matrix launches eagerly: capturing and updating
        // its phases costs more host time than the graph launches save (40x40
        // stencil: 0.65 ms per call with graphs, 0.60 ms eager; equal from
        // 4,000 rows up, while graphs are 2 % faster on a 4,096-matrix batch)
        const bool graphs = (plan.flags & GSOFA_EAGER) == 0 && !budget_mode && !(nj == 1 && N <= kEagerMaxRows);

        DBuf row_off(8 * (size_t)std::max<int64_t>(nrows, 1));
        DBuf row_cnt(4 * (size_t)std::max<int64_t>(nrows, 1));
        DBuf row_lcnt(4 * (size_t)std::max<int64_t>(nrows, 1));
        DBuf counters(64);  // [0] item counter, [1] pool tail
        DBuf jst(sizeof(JobStats) * std::max(nj, 1));
        DBuf pool(4 * (size_t)pool_cap);
        DBuf d_row_job, d_item_job;
        if (nj > 1) {
            d_row_job = DBuf(4 * (size_t)std::max<int64_t>(nrows, 1));
            d_item_job = DBuf(4 * (size_t)std::max<int64_t>(nrows, 1));
        }
        DBuf row_stats(sizeof(RowStat) * (size_t)std::max<int64_t>(nrows, 1));
        // job statistics and the pool tail come back through pinned memory
        PinnedBuf h_stats(sizeof(JobStats) * (size_t)std::max(nj, 1) + 64);
        JobStats* hst = h_stats.as<JobStats>();
        unsigned long long* h_tail =
            reinterpret_cast<unsigned long long*>(h_stats.as<char>() + sizeof(JobStats) * (size_t)std::max(nj, 1));
        unsigned long long* h_items = h_tail + 1;  // work counter after the traversal

        // ev[0]/ev[4]: traversal phase; ev[1]..ev[3]: emit, supernode and column phases
        EventSet ev;

        TraverseArgs ta{};
        ta.jobs = d_jobs.as<Job>();
        ta.njobs = nj;
        if (slots) {
            ta.nslots = slots->nslots < nslots ? slots->nslots : (int32_t)nslots;
            ta.slots = slots->buf.as<uint8_t>();
            ta.lay = slots->lay;
        }
        ta.nitems = items;
        ta.item_rows = nullptr;
        ta.row_job = d_row_job.as<int32_t>();
        ta.item_job = d_item_job.as<int32_t>();
        ta.row_stats = row_stats.as<RowStat>();
        ta.item_counter = counters.as<unsigned long long>();
        ta.row_off = row_off.as<int64_t>();
        ta.row_cnt = row_cnt.as<int32_t>();
        ta.row_lcnt = row_lcnt.as<int32_t>();
        ta.pool = pool.as<int32_t>();
        ta.pool_tail = counters.as<unsigned long long>() + 1;
        ta.pool_cap = pool_cap;
        ta.jstats = jst.as<JobStats>();
        ta.window = plan.window;
        ta.flags = plan.flags;
        ta.mapping = mapping;

        // Memory-budget mode (Space Optimization section). Sources run in bands
        // of decreasing ids, each band one launch whose slots hold labels, level
        // stamps and the pending bitmap for the ids below the band's largest
        // source only (bubble removal), so a band of smaller ids fits more
        // sources into the same budget (dynamic space allocation); the budget
        // gets as many slots as fit, at most the resident wavefronts, and a band
        // reaching that many takes all remaining sources. Worklists and row
        // buffers keep queue_cap entries on the device and spill the rest to
        // pinned host memory (external frontier management).
        int32_t band_launches = 0;
        int32_t trav_launches = 1;  // default mode: the first launch, plus relaunches after yields
        int32_t budget_max_c = 0;
        int64_t budget_peak_slots = 0;
        const int64_t slot_budget =
            plan.budget > 0 ? plan.budget
                            : std::max<int64_t>((int64_t)((di.free_b + di.reclaimable) * 0.9) - fixed - 4 * pool_cap,
                                                int64_t(64) << 20);
        auto run_budget = [&](const std::vector<int32_t>& rows, const std::vector<int32_t>& local) {
            // rows: global rows; local: their ids inside their matrix; both in
            // order of decreasing local id
            if (rows.empty()) return;
            const int64_t R5 = traverse_resident_slots(di.cus, 5);
            // plan the bands: [lo, hi) of local ids, layout, sources in flight
            struct Band {
                size_t pos, end;
                SlotLayout lay;
                int64_t ns;
            };
            std::vector<Band> bands;
            size_t spill_entries = 1;
            {
                size_t pos = 0;
                int64_t hi = (int64_t)local[0] + 1;
                while (pos < rows.size()) {
                    const SlotLayout lb = slot_layout_budget(N, hi, plan.queue_cap > 0 ? plan.queue_cap : 8192);
                    int64_t C = std::min<int64_t>(R5, slot_budget / lb.bytes_per_slot);
                    C = std::min<int64_t>(C, kSpillHostBytes / std::max<int64_t>(4 * lb.h_stride, 1));
                    if (plan.nslots > 0) C = std::min<int64_t>(C, plan.nslots);
                    if (C < 1) throw Status{GSOFA_ENOMEM};
                    const int64_t lo = (C >= R5 || hi <= 4096) ? 0 : hi / 2;
                    size_t end = pos;
                    while (end < rows.size() && local[end] >= lo) ++end;
                    int64_t ns = std::min<int64_t>(C, (int64_t)(end - pos));
                    if (ns > 4) ns = ns / 4 * 4;
                    if (end > pos) {
                        bands.push_back(Band{pos, end, lb, ns});
                        spill_entries = std::max<size_t>(spill_entries, (size_t)(ns * lb.h_stride));
                    }
                    pos = end;
                    hi = lo;
                }
            }
            DBuf d_rows(4 * rows.size());
            h2d(d_rows.p, rows.data(), 4 * rows.size(), st, false);
            // one spill area serves every band (bands run one after another)
            struct SpillHold {
                SpillCache::Block b;
                hipStream_t st;
                ~SpillHold() {
                    (void)hipStreamSynchronize(st);
                    (void)hipGetLastError();
                    spill_cache().give(b);
                }
            } spill{spill_cache().take(4 * spill_entries), st};
            for (const Band& bd : bands) {
                DBuf sl((size_t)bd.ns * (size_t)bd.lay.bytes_per_slot);
                chk(launch_init_slots(sl.as<uint8_t>(), (int32_t)bd.ns, bd.lay, st));
                TraverseArgs tb = ta;
                tb.slots = sl.as<uint8_t>();
                tb.lay = bd.lay;
                tb.nslots = (int32_t)bd.ns;
                tb.item_rows = d_rows.as<int32_t>() + bd.pos;
                tb.nitems = (int64_t)(bd.end - bd.pos);
                tb.item_job = nullptr;
                tb.row_job = nj > 1 ? d_row_job.as<int32_t>() : nullptr;
                tb.host_spill = static_cast<int32_t*>(spill.b.p);
                tb.mapping = 5;
                chk(launch_zero_i32(counters.as<int32_t>(), 2, st));  // the item counter only
                chk(launch_traverse(tb, st));
                ++band_launches;
                budget_max_c = std::max<int32_t>(budget_max_c, (int32_t)bd.ns);
                budget_peak_slots = std::max<int64_t>(budget_peak_slots, bd.ns * bd.lay.bytes_per_slot);
            }
            chk(hipStreamSynchronize(st));
        };
        // local id of a global row (matrices in the user's order, row_base increasing)
        auto local_of = [&](int32_t r) -> int32_t {
            const auto it = std::upper_bound(row_base.begin(), row_base.end(), (int64_t)r);
            return (int32_t)(r - *(it - 1));
        };

        if (yh && yh->before_traverse) yh->before_traverse();
        chk(hipEventRecord(ev[0], st));
        if (budget_mode) {
            if (nj > 1) chk(launch_row_job(d_jobs.as<Job>(), nj, N, d_row_job.as<int32_t>(), st));
            chk(launch_zero_i32(counters.as<int32_t>(), 16, st));
            chk(launch_zero_i32(jst.as<int32_t>(), (int64_t)(sizeof(JobStats) / 4) * nj, st));
            // every source, largest ids first (the job table is sorted by size)
            std::vector<int32_t> rows, local;
            rows.reserve((size_t)items);
            local.reserve((size_t)items);
            for (int64_t sid = N - 1; sid >= 0; --sid)
                for (int32_t q = 0; q < nj && jt[q].n > sid; ++q) {
                    rows.push_back((int32_t)(jt[q].row_base + sid));
                    local.push_back((int32_t)sid);
                }
            run_budget(rows, local);
            chk(launch_job_stats(d_jobs.as<Job>(), nj, N, row_stats.as<RowStat>(), jst.as<JobStats>(), st));
            chk(launch_copy_to_host(hst, jst.p, sizeof(JobStats) * nj, st));
            chk(launch_copy_to_host(h_tail, counters.as<unsigned long long>() + 1, 8, st));
            chk(hipEventRecord(ev[4], st));
            chk(hipStreamSynchronize(st));
        } else {
            // phase 1: one persistent traversal launch over every source of every matrix
            Phase ph(kPhaseTraverse, graphs, st);
            const hipStream_t s = ph.stream();
            if (nj > 1) {
                chk(launch_row_job(d_jobs.as<Job>(), nj, N, d_row_job.as<int32_t>(), s));
                chk(launch_row_job(d_jobs.as<Job>(), nj, N, d_item_job.as<int32_t>(), s, true));
            }
            chk(launch_zero_i32(counters.as<int32_t>(), 16, s));
            chk(launch_zero_i32(jst.as<int32_t>(), (int64_t)(sizeof(JobStats) / 4) * nj, s));
            ta.yield = yh ? yh->flag : nullptr;
            chk(launch_traverse(ta, s));
            chk(launch_job_stats(d_jobs.as<Job>(), nj, N, row_stats.as<RowStat>(), jst.as<JobStats>(), s));
            chk(launch_copy_to_host(hst, jst.p, sizeof(JobStats) * nj, s));
            chk(launch_copy_to_host(h_tail, counters.as<unsigned long long>() + 1, 8, s));
            chk(launch_copy_to_host(h_items, counters.as<unsigned long long>(), 8, s));
            ph.launch();
            if (yh && yh->enqueued) yh->enqueued();
            chk(hipEventRecord(ev[4], st));
            chk(hipStreamSynchronize(st));
            ph.done();
            // A launch asked to yield stopped taking work items: every item below
            // the counter is done, relaunch for the rest. Two launches in a row
            // that take nothing (the flag keeps being set) end the yielding.
            int32_t idle = 0;
            std::vector<int32_t> err_seen(ta.yield ? (size_t)nj : 0, 0);
            while (ta.yield && *h_items < (unsigned long long)items) {
                const unsigned long long before = *h_items;
                // the statistics are summed again after the relaunch; error bits of
                // rows done so far are kept on the host
                for (int32_t q = 0; q < nj; ++q) err_seen[(size_t)q] |= hst[q].err;
                if (yh->before_resume) yh->before_resume();
                __atomic_store_n(yh->flag, 0u, __ATOMIC_RELEASE);
                if (idle >= 2) ta.yield = nullptr;
                chk(launch_zero_i32(jst.as<int32_t>(), (int64_t)(sizeof(JobStats) / 4) * nj, st));
                chk(launch_traverse(ta, st));
                ++trav_launches;
                chk(launch_job_stats(d_jobs.as<Job>(), nj, N, row_stats.as<RowStat>(), jst.as<JobStats>(), st));
                chk(launch_copy_to_host(hst, jst.p, sizeof(JobStats) * nj, st));
                chk(launch_copy_to_host(h_tail, counters.as<unsigned long long>() + 1, 8, st));
                chk(launch_copy_to_host(h_items, counters.as<unsigned long long>(), 8, st));
                chk(hipEventRecord(ev[4], st));
                chk(hipStreamSynchronize(st));
                idle = *h_items == before ? idle + 1 : 0;
            }
            for (size_t q = 0; q < err_seen.size(); ++q) hst[q].err |= err_seen[q];
            ta.yield = nullptr;
            if (yh && yh->finished) yh->finished();
        }

        bool overflow = false;
        float t_trav_extra = 0;
        int32_t n_launches = budget_mode ? band_launches : trav_launches;
        for (int32_t q = 0; q < nj; ++q) {
            if (hst[q].err & kErrDuplicate) jstat[ord[q]] = GSOFA_EINVAL;
            if (hst[q].err & kErrOverflow) overflow = true;
        }
        if (overflow) {
            // rows that did not fit: grow the pool, keep what fits, redo the rest
            // per-row offsets and counts: through copy kernels and pinned memory
            // when small, the runtime's copies into pageable memory otherwise
            const size_t rows_b = 12 * (size_t)std::max<int64_t>(nrows, 1);
            std::unique_ptr<PinnedBuf> h_rows;
            std::vector<char> h_rows_big;
            char* hr = nullptr;
            if (rows_b <= kKernelCopyMax) {
                h_rows = std::make_unique<PinnedBuf>(rows_b);
                hr = h_rows->as<char>();
                chk(launch_copy_to_host(hr, row_off.p, 8 * (size_t)nrows, st));
                chk(launch_copy_to_host(hr + 8 * (size_t)nrows, row_cnt.p, 4 * (size_t)nrows, st));
            } else {
                h_rows_big.resize(rows_b);
                hr = h_rows_big.data();
                chk(hipMemcpyAsync(hr, row_off.p, 8 * (size_t)nrows, hipMemcpyDeviceToHost, st));
                chk(hipMemcpyAsync(hr + 8 * (size_t)nrows, row_cnt.p, 4 * (size_t)nrows, hipMemcpyDeviceToHost, st));
            }
            chk(hipStreamSynchronize(st));
            const int64_t* h_off = reinterpret_cast<const int64_t*>(hr);
            const int32_t* h_cnt = reinterpret_cast<const int32_t*>(hr + 8 * (size_t)nrows);
            std::vector<int32_t> redo;
            int64_t need = 0;
            for (int64_t r = 0; r < nrows; ++r)
                if (h_off[r] < 0) {
                    redo.push_back((int32_t)r);
                    need += h_cnt[r];
                }
            const int64_t new_cap = pool_cap + need;
            DBuf pool2(4 * (size_t)new_cap);
            chk(launch_copy_device(pool2.p, pool.p, 4 * (size_t)pool_cap, st));
            pool = std::move(pool2);
            DBuf d_redo(4 * redo.size());
            h2d(d_redo.p, redo.data(), 4 * redo.size(), st, false);
            unsigned long long cnt2[2] = {0ull, (unsigned long long)pool_cap};
            h2d(counters.p, cnt2, 16, st, false);
            ta.item_rows = d_redo.as<int32_t>();
            ta.nitems = (int64_t)redo.size();
            ta.pool = pool.as<int32_t>();
            ta.pool_cap = new_cap;
            // redone rows store the same per-source statistics again
            chk(launch_zero_i32(jst.as<int32_t>(), (int64_t)(sizeof(JobStats) / 4) * nj, st));
            float first_ms = 0;
            chk(hipEventElapsedTime(&first_ms, ev[0], ev[4]));
            t_trav_extra += first_ms;
            chk(hipEventRecord(ev[0], st));
            if (budget_mode) {
                std::vector<int32_t> loc(redo.size());
                for (size_t i = 0; i < redo.size(); ++i) loc[i] = local_of(redo[i]);
                std::vector<size_t> perm(redo.size());
                for (size_t i = 0; i < perm.size(); ++i) perm[i] = i;
                std::stable_sort(perm.begin(), perm.end(), [&](size_t x, size_t y) { return loc[x] > loc[y]; });
                std::vector<int32_t> rr(redo.size()), ll(redo.size());
                for (size_t i = 0; i < perm.size(); ++i) {
                    rr[i] = redo[perm[i]];
                    ll[i] = loc[perm[i]];
                }
                const int32_t before = band_launches;
                run_budget(rr, ll);
                n_launches += band_launches - before;
            } else {
                chk(launch_traverse(ta, st));
                ++n_launches;
            }
            chk(hipEventRecord(ev[4], st));
            chk(launch_job_stats(d_jobs.as<Job>(), nj, N, row_stats.as<RowStat>(), jst.as<JobStats>(), st));
            chk(launch_copy_to_host(hst, jst.p, sizeof(JobStats) * nj, st));
            chk(launch_copy_to_host(h_tail, counters.as<unsigned long long>() + 1, 8, st));
            chk(hipStreamSynchronize(st));
            for (int32_t q = 0; q < nj; ++q) {
                if (hst[q].err & kErrOverflow) throw Status{GSOFA_ENOMEM};
                if (hst[q].err & kErrDuplicate) jstat[ord[q]] = GSOFA_EINVAL;
            }
            pool_cap = new_cap;
        }
        chk(hipEventRecord(ev[1], st));
        if (slots) give_slots(std::move(slots));
        if (total_nnz > 0)
            note_fill_ratio(key, std::max(4.0, (double)*h_tail / (double)total_nnz));

        // ---- phase 2: counts -> row pointers of U and L, and the totals
        DBuf scan_scr(8 * (size_t)scan_scratch_elems(nrows + 1) + 64);
        DBuf u_ptr(8 * (size_t)(nrows + 1)), l_rptr(8 * (size_t)(nrows + 1));
        PinnedBuf h_tot(16);
        {
            Phase ph(kPhaseScan, graphs, st);
            const hipStream_t s = ph.stream();
            chk(launch_scan_counts(row_cnt.as<int32_t>(), row_lcnt.as<int32_t>(), nrows, u_ptr.as<int64_t>(),
                                   scan_scr.as<int64_t>(), s));
            chk(launch_scan_counts(row_lcnt.as<int32_t>(), nullptr, nrows, l_rptr.as<int64_t>(),
                                   scan_scr.as<int64_t>(), s));
            chk(launch_copy_to_host(h_tot.as<int64_t>(), u_ptr.as<int64_t>() + nrows, 8, s));
            chk(launch_copy_to_host(h_tot.as<int64_t>() + 1, l_rptr.as<int64_t>() + nrows, 8, s));
            ph.launch();
            chk(hipStreamSynchronize(st));
            ph.done();
        }
        const int64_t nnz_u = h_tot.as<int64_t>()[0], nnz_l = h_tot.as<int64_t>()[1];

        // ---- everything the remaining phases touch is allocated up front, so
        // that they can be captured and replayed without host work in between
        const bool want_sn = (plan.flags & GSOFA_NO_SUPERNODES) == 0;
        const bool have_sn = want_sn && nrows > 0;
        const bool l_csr = (plan.flags & GSOFA_L_CSR) != 0;
        DBuf u_idx(4 * (size_t)std::max<int64_t>(nnz_u, 1)), l_ridx(4 * (size_t)std::max<int64_t>(nnz_l, 1));
        DBuf big_list(4 * (size_t)std::max<int64_t>(nrows, 1)), big_cnt(64);

        // small host tables in one pinned block and one upload: row bases and
        // sizes per matrix, a job table in the user's order, supernode blocks
        std::vector<int64_t> bf;
        std::vector<int32_t> bl;
        if (have_sn)
            for (int32_t j = 0; j < nj; ++j) {
                const int64_t M = plan.max_super > 0 ? plan.max_super : std::max<int64_t>(mats[j].n, 1);
                for (int64_t b = 0; b < mats[j].n; b += M) {
                    bf.push_back(row_base[j] + b);
                    bl.push_back((int32_t)std::min<int64_t>(M, mats[j].n - b));
                }
            }
        const int64_t nbk = (int64_t)bf.size();
        auto up8 = [](int64_t b) { return (b + 15) & ~int64_t(15); };
        const int64_t o_jrb = 0, o_jn = o_jrb + up8(8 * (int64_t)nj), o_ju = o_jn + up8(4 * (int64_t)nj),
                      o_bf = o_ju + up8((int64_t)sizeof(Job) * nj), o_bl = o_bf + up8(8 * nbk),
                      up_bytes = o_bl + up8(4 * nbk) + 16;
        PinnedBuf h_up((size_t)up_bytes);
        DBuf d_up((size_t)up_bytes);
        {
            char* c = h_up.as<char>();
            int64_t* jrb = reinterpret_cast<int64_t*>(c + o_jrb);
            int32_t* jn = reinterpret_cast<int32_t*>(c + o_jn);
            Job* ju = reinterpret_cast<Job*>(c + o_ju);
            for (int32_t j = 0; j < nj; ++j) {
                jrb[j] = row_base[j];
                jn[j] = mats[j].n;
                ju[j] = jobs[j];
                ju[j].n = mats[j].n;
                ju[j].row_base = row_base[j];
            }
            if (nbk) {
                std::memcpy(c + o_bf, bf.data(), 8 * (size_t)nbk);
                std::memcpy(c + o_bl, bl.data(), 4 * (size_t)nbk);
            }
        }
        const int64_t* d_jrb = reinterpret_cast<const int64_t*>(d_up.as<char>() + o_jrb);
        const int32_t* d_jn = reinterpret_cast<const int32_t*>(d_up.as<char>() + o_jn);
        const Job* d_ju = reinterpret_cast<const Job*>(d_up.as<char>() + o_ju);
        const int64_t* d_bf = reinterpret_cast<const int64_t*>(d_up.as<char>() + o_bf);
        const int32_t* d_bl = reinterpret_cast<const int32_t*>(d_up.as<char>() + o_bl);

        // rows of the global row space -> matrix in the user's order
        DBuf row_job_user;
        RowSpace rs{nrows, nullptr, nullptr};
        if (nj > 1) {
            row_job_user = DBuf(4 * (size_t)std::max<int64_t>(nrows, 1));
            rs.row_job = row_job_user.as<int32_t>();
            rs.job_row_base = d_jrb;
        }
        DBuf is_start, start_scan, xsup_all, supno_all;
        if (have_sn) {
            is_start = DBuf(4 * (size_t)nrows);
            start_scan = DBuf(8 * (size_t)(nrows + 1));
            xsup_all = DBuf(4 * (size_t)(nrows + nj));
            supno_all = DBuf(4 * (size_t)nrows);
        }
        DBuf l_cptr, l_cidx, col_cnt, cursor, ctmp;
        if (!l_csr) {
            l_cptr = DBuf(8 * (size_t)(nrows + 1));
            l_cidx = DBuf(4 * (size_t)std::max<int64_t>(nnz_l, 1));
            col_cnt = DBuf(4 * (size_t)std::max<int64_t>(nrows, 1));
            cursor = DBuf(4 * (size_t)std::max<int64_t>(nrows, 1));
            ctmp = DBuf(4 * (size_t)std::max<int64_t>(nnz_l, 1));
        }
        const int64_t* Lp = l_csr ? l_rptr.as<int64_t>() : l_cptr.as<int64_t>();
        const int32_t* Li = l_csr ? l_ridx.as<int32_t>() : l_cidx.as<int32_t>();
        // per-matrix pointer arrays (each starting at 0) side by side: matrix j
        // owns entries [row_base_j + j, row_base_j + j + n_j]
        DBuf u_ptr_loc, l_ptr_loc;
        const int64_t* Up_loc = u_ptr.as<int64_t>();
        const int64_t* Lp_loc = Lp;
        if (nj > 1) {
            u_ptr_loc = DBuf(8 * (size_t)(nrows + nj));
            l_ptr_loc = DBuf(8 * (size_t)(nrows + nj));
            Up_loc = u_ptr_loc.as<int64_t>();
            Lp_loc = l_ptr_loc.as<int64_t>();
        }
        // pointer values at the matrix boundaries, for the result headers
        DBuf d_b(8 * 3 * (size_t)(nj + 1));
        PinnedBuf h_b(8 * 3 * (size_t)(nj + 1));

        // ---- phase 3: sorted rows of U (CSR) and L (CSR)
        Phase ph_sort(kPhaseSort, graphs, st);
        {
            const hipStream_t s = ph_sort.stream();
            h2d(d_up.p, h_up.p, (size_t)up_bytes, s, true);
            if (nj > 1) chk(launch_row_job(d_ju, nj, N, row_job_user.as<int32_t>(), s));
            chk(launch_sort_rows(rs, row_off.as<int64_t>(), row_cnt.as<int32_t>(), row_lcnt.as<int32_t>(),
                                 pool.as<int32_t>(), u_ptr.as<int64_t>(), u_idx.as<int32_t>(),
                                 l_rptr.as<int64_t>(), l_ridx.as<int32_t>(), big_list.as<int32_t>(),
                                 big_cnt.as<int32_t>(), s));
            ph_sort.launch();
        }
        chk(hipEventRecord(ev[2], st));

        // ---- phase 4: supernodes (Definition T3 per block of max_supernode rows)
        Phase ph_sn(kPhaseSupernodes, graphs, st);
        if (have_sn) {
            const hipStream_t s = ph_sn.stream();
            chk(launch_supernodes(rs, nbk, d_bf, d_bl, u_ptr.as<int64_t>(), l_rptr.as<int64_t>(),
                                  l_ridx.as<int32_t>(), is_start.as<int32_t>(), s));
            chk(launch_scan_counts(is_start.as<int32_t>(), nullptr, nrows, start_scan.as<int64_t>(),
                                   scan_scr.as<int64_t>(), s));
            chk(launch_supernode_assemble(rs, nj, is_start.as<int32_t>(), start_scan.as<int64_t>(),
                                          xsup_all.as<int32_t>(), supno_all.as<int32_t>(), s));
            chk(launch_supernode_terminals(nj, d_jrb, d_jn, start_scan.as<int64_t>(), xsup_all.as<int32_t>(), s));
        }
        ph_sn.launch();
        chk(hipEventRecord(ev[3], st));

        // ---- phase 5: L column-wise, per-matrix pointers, boundary values
        Phase ph_col(kPhaseColumns, graphs, st);
        {
            const hipStream_t s = ph_col.stream();
            if (!l_csr)
                chk(launch_transpose_l(rs, l_rptr.as<int64_t>(), l_ridx.as<int32_t>(), col_cnt.as<int32_t>(),
                                       l_cptr.as<int64_t>(), l_cidx.as<int32_t>(), scan_scr.as<int64_t>(),
                                       cursor.as<int32_t>(), ctmp.as<int32_t>(), big_list.as<int32_t>(),
                                       big_cnt.as<int32_t>(), s));
            if (nj > 1) {
                const unsigned gx = (unsigned)std::min<int64_t>((N + 256) / 256, 64);
                hipLaunchKernelGGL(k_rebase_ptr, dim3(gx, nj), dim3(256), 0, s, nj, d_jrb, d_jn,
                                   u_ptr.as<int64_t>(), u_ptr_loc.as<int64_t>());
                hipLaunchKernelGGL(k_rebase_ptr, dim3(gx, nj), dim3(256), 0, s, nj, d_jrb, d_jn, Lp,
                                   l_ptr_loc.as<int64_t>());
            }
            const dim3 gb((nj + 1 + 255) / 256);
            hipLaunchKernelGGL(k_gather_bounds, gb, dim3(256), 0, s, nj, d_jrb, nrows, u_ptr.as<int64_t>(),
                               d_b.as<int64_t>());
            hipLaunchKernelGGL(k_gather_bounds, gb, dim3(256), 0, s, nj, d_jrb, nrows, Lp,
                               d_b.as<int64_t>() + (nj + 1));
            if (have_sn)
                hipLaunchKernelGGL(k_gather_bounds, gb, dim3(256), 0, s, nj, d_jrb, nrows, start_scan.as<int64_t>(),
                                   d_b.as<int64_t>() + 2 * (nj + 1));
            chk(hipGetLastError());
            chk(launch_copy_to_host(h_b.p, d_b.p, 8 * 3 * (size_t)(nj + 1), s));
            ph_col.launch();
        }
        chk(hipStreamSynchronize(st));
        ph_sort.done();
        ph_sn.done();
        ph_col.done();
        pool.reset();

        float t_trav = 0, t_emit = 0, t_sn = 0;
        chk(hipEventElapsedTime(&t_trav, ev[0], ev[4]));
        t_trav += t_trav_extra;
        chk(hipEventElapsedTime(&t_emit, ev[1], ev[2]));
        chk(hipEventElapsedTime(&t_sn, ev[2], ev[3]));

        // ---- results
        const bool dev_out = (plan.flags & GSOFA_RESULT_ON_DEVICE) != 0;
        std::vector<int64_t> ujb(nj + 1), ljb(nj + 1), sjb(nj + 1, 0);
        {
            const int64_t* hb = h_b.as<int64_t>();
            for (int32_t j = 0; j <= nj; ++j) {
                ujb[j] = hb[j];
                ljb[j] = hb[nj + 1 + j];
                if (have_sn) sjb[j] = hb[2 * (nj + 1) + j];
            }
        }
        const int64_t nptr = nrows + std::max(nj, 1);

        // host results: every array copied once into one block shared by the
        // results of this call (freed with the last of them)
        std::shared_ptr<void> hblock;
        int64_t *h_up_ptr = nullptr, *h_lp_ptr = nullptr;
        int32_t *h_ui = nullptr, *h_li = nullptr, *h_xs = nullptr, *h_sn = nullptr;
        std::shared_ptr<std::vector<DBuf>> keep;
        if (!dev_out) {
            const size_t bytes = 8 * 2 * (size_t)nptr + 4 * (size_t)(nnz_u + nnz_l) +
                                 (have_sn ? 4 * (size_t)(nrows + nj + nrows) : 0) + 64;
            const ResultBlocks::Block rb = result_blocks().take(bytes);
            void* blk = rb.p;
            if (!blk) throw Status{GSOFA_ENOMEM};
            // until the copies into it have completed, an error returns the block
            // only after the stream has drained
            struct Guard {
                ResultBlocks::Block b;
                hipStream_t st;
                bool armed = true;
                ~Guard() {
                    if (!armed) return;
                    (void)hipStreamSynchronize(st);
                    (void)hipGetLastError();
                    if (b.pinned) result_blocks().give(b.p);
                    else std::free(b.p);
                }
            } guard{rb, st};
            h_up_ptr = static_cast<int64_t*>(blk);
            h_lp_ptr = h_up_ptr + nptr;
            h_ui = reinterpret_cast<int32_t*>(h_lp_ptr + nptr);
            h_li = h_ui + nnz_u;
            h_xs = h_li + nnz_l;
            h_sn = h_xs + (have_sn ? nrows + nj : 0);
            // into page-locked memory every result comes back through the copy
            // kernel (as fast as the runtime's copy, which dispatched 512- and
            // 1,024-thread workgroups that wait for room next to running
            // traversals); into pageable memory a small one through the copy
            // kernel and a pinned block, a large one through the runtime's
            // staged copies
            struct Piece {
                void* dst;
                const void* src;
                size_t bytes;
            };
            std::vector<Piece> pieces{{h_up_ptr, Up_loc, 8 * (size_t)nptr}, {h_lp_ptr, Lp_loc, 8 * (size_t)nptr},
                                      {h_ui, u_idx.p, 4 * (size_t)nnz_u}, {h_li, Li, 4 * (size_t)nnz_l}};
            if (have_sn) {
                pieces.push_back({h_xs, xsup_all.p, 4 * (size_t)(nrows + nj)});
                pieces.push_back({h_sn, supno_all.p, 4 * (size_t)nrows});
            }
            size_t small_b = 0;
            for (auto& pc : pieces) small_b += pc.bytes;
            if (rb.pinned) {
                for (auto& pc : pieces)
                    if (pc.bytes) chk(launch_copy_to_host(pc.dst, pc.src, pc.bytes, st));
                chk(hipStreamSynchronize(st));
            } else if (small_b <= kKernelCopyMax) {
                PinnedBuf out_stage(std::max<size_t>(small_b, 4));
                size_t off = 0;
                for (auto& pc : pieces) {
                    chk(launch_copy_to_host(out_stage.as<char>() + off, pc.src, pc.bytes, st));
                    off += pc.bytes;
                }
                chk(hipStreamSynchronize(st));
                off = 0;
                for (auto& pc : pieces) {
                    if (pc.bytes) std::memcpy(pc.dst, out_stage.as<char>() + off, pc.bytes);
                    off += pc.bytes;
                }
            } else {
                for (auto& pc : pieces)
                    if (pc.bytes) chk(hipMemcpyAsync(pc.dst, pc.src, pc.bytes, hipMemcpyDeviceToHost, st));
                chk(hipStreamSynchronize(st));
            }
            guard.armed = false;
            if (rb.pinned)
                hblock = std::shared_ptr<void>(blk, [](void* q) { result_blocks().give(q); });
            else
                hblock = std::shared_ptr<void>(blk, [](void* q) { std::free(q); });
        } else {
            keep = std::make_shared<std::vector<DBuf>>();
        }
        // no more device work in this call: buffers released from here on are idle
        t_idle = true;

        static int32_t zero_xsup = 0;
        for (int32_t j = 0; j < nj; ++j) {
            gsofa_result* r = new_result();
            results[j] = r;
            const int32_t q = jt_of[j];
            r->n = mats[j].n;
            r->flags = plan.flags;
            r->stats.status = jstat[j];
            r->stats.edges_alg = hst[q].edges_alg;
            r->stats.edges_gpu = hst[q].edges_gpu;
            r->stats.iterations = hst[q].iterations;
            r->stats.windows = hst[q].windows;
            r->stats.concurrent_sources = budget_mode ? budget_max_c : ta.nslots;
            r->stats.peak_device_bytes =
                (uint64_t)((budget_mode ? budget_peak_slots : nslots * lay.bytes_per_slot) + pool_cap * 4 + nrows * 48 +
                           (nnz_u + 3 * nnz_l) * 4);
            r->stats.t_traverse_ms = t_trav;
            r->stats.t_emit_ms = t_emit;
            r->stats.t_supernode_ms = t_sn;
            r->stats.window = plan.window;
            r->stats.mapping = mapping;
            r->stats.t_tune_ms = t_tune;
            r->stats.launches = n_launches;
            r->stats.spilled_entries = hst[q].spilled;
            if (jstat[j] != GSOFA_OK) continue;
            const int64_t n = mats[j].n, b = row_base[j];
            r->nnz_a = nnz[j];
            r->nnz_u = ujb[j + 1] - ujb[j];
            r->nnz_l = ljb[j + 1] - ljb[j];
            r->fills = r->nnz_u + r->nnz_l - (nnz[j] + n - (int64_t)hst[q].diag);
            r->nsuper = want_sn ? (int32_t)(sjb[j + 1] - sjb[j]) : 0;
            auto* own = static_cast<ResultOwner*>(r->internal_);
            if (!dev_out) {
                own->shared_host = hblock;
                r->u_ptr = h_up_ptr + b + j;
                r->l_ptr = h_lp_ptr + b + j;
                r->u_idx = h_ui + ujb[j];
                r->l_idx = h_li + ljb[j];
                if (want_sn) {
                    // an empty matrix has the one-entry partition {0}
                    r->xsup = have_sn ? h_xs + sjb[j] + j : &zero_xsup;
                    r->supno = have_sn ? h_sn + b : nullptr;
                }
            } else {
                own->dev = keep;
                r->u_ptr = const_cast<int64_t*>(Up_loc) + b + j;
                r->l_ptr = const_cast<int64_t*>(Lp_loc) + b + j;
                r->u_idx = u_idx.as<int32_t>() + ujb[j];
                r->l_idx = const_cast<int32_t*>(Li) + ljb[j];
                if (want_sn && n > 0) {
                    r->xsup = xsup_all.as<int32_t>() + sjb[j] + j;
                    r->supno = supno_all.as<int32_t>() + b;
                }
            }
        }
        if (dev_out) {
            for (DBuf* db : {&u_idx, &u_ptr, &l_rptr, &l_ridx, &l_cptr, &l_cidx, &xsup_all, &supno_all,
                             &u_ptr_loc, &l_ptr_loc})
                db->synced = true;
            keep->push_back(std::move(u_idx));
            keep->push_back(std::move(u_ptr));
            if (l_csr) {
                keep->push_back(std::move(l_rptr));
                keep->push_back(std::move(l_ridx));
            } else {
                keep->push_back(std::move(l_cptr));
                keep->push_back(std::move(l_cidx));
            }
            keep->push_back(std::move(xsup_all));
            keep->push_back(std::move(supno_all));
            keep->push_back(std::move(u_ptr_loc));
            keep->push_back(std::move(l_ptr_loc));
        }
        const double t1 = now_ms();
        int first_bad = GSOFA_OK;
        for (int32_t j = 0; j < nj; ++j) {
            results[j]->stats.t_total_ms = t1 - t0;
            if (jstat[j] != GSOFA_OK && first_bad == GSOFA_OK) first_bad = jstat[j];
        }
        return first_bad;
    }

    // Times every tuner candidate on one stratified sample of the call's
    // sources (largest ids first inside each matrix, as in the real order) and
    // returns the fastest; a candidate must beat the current best by 5% to
    // replace it, so near-ties keep the earlier (default) one. The sample's
    // rows go to scratch arrays; the slot sets are left clean for the real run.
    template <typename PlanSlots>
    TuneChoice tune(const std::vector<Job>& jt, int32_t nj, int64_t N, int64_t items, const SlotLayout& lay,
                    int64_t budget, int64_t fixed, int64_t total_nnz, int64_t nrows, const DBuf& d_jobs,
                    PlanSlots plan_slots) {
        const int64_t R = plan_slots(0);
        // Successive halving: every candidate on a first sample of
        // kTuneScreenPerSlot sources per slot, the kTuneFinalists best of them
        // on the full sample of kTuneSamplesPerSlot. Each sample is stratified
        // over the call's sources; the candidates with half the sources in flight
        // run every other entry of it (the same number of sources per slot, so
        // the tail weighs the same; candidates are compared by edges per second).
        const int64_t S = std::min<int64_t>(items, std::max<int64_t>(R * kTuneSamplesPerSlot, 1));
        const int64_t S2 = std::max<int64_t>(S / 2, 1);
        const int64_t T = std::min<int64_t>(items - items / 64, std::max<int64_t>(R * kTuneScreenPerSlot, 1));
        const int64_t T2 = std::max<int64_t>(T / 2, 1);
        PinnedBuf h_s(4 * (size_t)(S + S2 + T + T2));
        int32_t* smp = h_s.as<int32_t>();
        // The screening sample skips the first 1/64 of the work items (the
        // highest source ids): in a nested-dissection order those are the top
        // separators, whose sources reach most of the matrix. In a full launch
        // they run first and overlap everything else, but in a short trial they
        // set its length on their own (2D 9-point stencil: trials of ~200 ms
        // where the sources' mean cost predicted ~20 ms). The final sample keeps
        // them: without them a near-tie on the 64^3 27-point stencil went to a
        // candidate 5 % slower at full size.
        auto stratified = [&](int32_t* out, int64_t count, int64_t head) {
            const int64_t span = std::max<int64_t>(items - head, 1);
            int32_t q = 0;
            for (int64_t i = 0; i < count; ++i) {
                const int64_t k = head + (int64_t)((__int128)i * span / count);
                while (q + 1 < nj && jt[q + 1].item_base <= k) ++q;
                out[i] = (int32_t)(jt[q].row_base + (jt[q].n - 1 - (k - jt[q].item_base)));
            }
        };
        stratified(smp, S, 0);
        for (int64_t i = 0; i < S2; ++i) smp[S + i] = smp[std::min<int64_t>(2 * i, S - 1)];
        stratified(smp + S + S2, T, items / 64);
        for (int64_t i = 0; i < T2; ++i) smp[S + S2 + T + i] = smp[S + S2 + std::min<int64_t>(2 * i, T - 1)];
        DBuf d_s(4 * (size_t)(S + S2 + T + T2)), tcnt(64), tjst(sizeof(JobStats) * (size_t)std::max(nj, 1));
        DBuf t_off(8 * (size_t)std::max<int64_t>(nrows, 1)), t_cnt(4 * (size_t)std::max<int64_t>(nrows, 1)),
            t_lcnt(4 * (size_t)std::max<int64_t>(nrows, 1)),
            t_rs(sizeof(RowStat) * (size_t)std::max<int64_t>(nrows, 1));
        chk(launch_copy_from_host(d_s.p, h_s.p, 4 * (size_t)(S + S2 + T + T2), st));
        DBuf d_rj;
        if (nj > 1) {
            d_rj = DBuf(4 * (size_t)std::max<int64_t>(nrows, 1));
            chk(launch_row_job(d_jobs.as<Job>(), nj, N, d_rj.as<int32_t>(), st));
        }
        // scratch output pool for the sample; rows that do not fit are only flagged
        const int64_t want_pool =
            pool_estimate(nrows, total_nnz, fill_ratio_for(TuneKey{device_info().cus, ceil_log2(N),
                                                                  ceil_log2(std::max<int64_t>(total_nnz * 4 / std::max<int64_t>(nrows, 1), 1)),
                                                                  nj > 1 ? ceil_log2(nj) : 0})) /
                std::max<int64_t>(items, 1) * S * 2 +
            (1 << 20);
        const int64_t room = (budget - fixed - R * lay.bytes_per_slot) / 4 / 3;
        const int64_t pcap = std::max<int64_t>(std::min<int64_t>(want_pool, room), 1 << 16);
        DBuf tpool(4 * (size_t)pcap);
        PinnedBuf h_js(sizeof(JobStats) * (size_t)std::max(nj, 1));
        EventSet ev;
        // one trial: edges per millisecond of candidate c on the full or the
        // first sample
        auto trial = [&](const TuneChoice& c, bool full) -> double {
            const int64_t ns = div_slots(plan_slots(c.mapping), c.div);
            auto ss = take_slots(lay, (int32_t)ns, c.mapping == 3 ? 1 : 0, st);
            TraverseArgs ta{};
            ta.jobs = d_jobs.as<Job>();
            ta.njobs = nj;
            ta.nslots = (int32_t)std::min<int64_t>(ns, ss->nslots);
            ta.nitems = full ? (c.div == 2 ? S2 : S) : (c.div == 2 ? T2 : T);
            ta.item_rows = d_s.as<int32_t>() + (full ? (c.div == 2 ? S : 0) : (c.div == 2 ? S + S2 + T : S + S2));
            ta.row_job = d_rj.as<int32_t>();
            ta.item_job = nullptr;
            ta.row_stats = t_rs.as<RowStat>();
            ta.item_counter = tcnt.as<unsigned long long>();
            ta.slots = ss->buf.as<uint8_t>();
            ta.lay = ss->lay;
            ta.row_off = t_off.as<int64_t>();
            ta.row_cnt = t_cnt.as<int32_t>();
            ta.row_lcnt = t_lcnt.as<int32_t>();
            ta.pool = tpool.as<int32_t>();
            ta.pool_tail = tcnt.as<unsigned long long>() + 1;
            ta.pool_cap = pcap;
            ta.jstats = tjst.as<JobStats>();
            ta.window = c.window;
            ta.flags = (plan.flags & ~(uint32_t)GSOFA_NO_LINE95) | c.flags;
            ta.mapping = c.mapping;
            chk(launch_zero_i32(tcnt.as<int32_t>(), 16, st));
            chk(launch_zero_i32(tjst.as<int32_t>(), (int64_t)(sizeof(JobStats) / 4) * nj, st));
            chk(launch_zero_i32(t_rs.as<int32_t>(), (int64_t)(sizeof(RowStat) / 4) * nrows, st));
            chk(hipEventRecord(ev[0], st));
            chk(launch_traverse(ta, st));
            chk(hipEventRecord(ev[1], st));
            chk(launch_job_stats(d_jobs.as<Job>(), nj, N, t_rs.as<RowStat>(), tjst.as<JobStats>(), st));
            chk(launch_copy_to_host(h_js.p, tjst.p, sizeof(JobStats) * nj, st));
            chk(hipStreamSynchronize(st));
            give_slots(std::move(ss));
            float ms = 0;
            chk(hipEventElapsedTime(&ms, ev[0], ev[1]));
            double edges = 0;
            for (int32_t jj = 0; jj < nj; ++jj) edges += (double)h_js.as<JobStats>()[jj].edges_alg;
            return edges / std::max(1e-3, (double)ms);
        };
        constexpr int kCand = (int)(sizeof(kTuneCandidates) / sizeof(kTuneCandidates[0]));
        // The first candidate runs once untimed: the first launch on a new slot
        // set also pays for touching its memory, which made that candidate lose
        // by ~7 % to an equal one on the 64^3 27-point stencil.
        (void)trial(kTuneCandidates[0], false);
        std::vector<std::pair<double, int>> screen;
        for (int t = 0; t < kCand; ++t) screen.push_back({trial(kTuneCandidates[t], false), t});
        std::stable_sort(screen.begin(), screen.end(),
                         [](const std::pair<double, int>& x, const std::pair<double, int>& y) { return x.first > y.first; });
        // finalists: the first candidate (the prior's choice, replaced only by a
        // finalist 5 % faster on the final sample) and the kTuneFinalists best
        // of the screening. Short screening trials are noisy near ties: without
        // the first candidate in the final, the 64^3 27-point stencil went to
        // one 5 % slower at full size in four tunings out of five.
        std::vector<int> fin{0};
        for (int i = 0; i < kCand && (int)fin.size() <= kTuneFinalists; ++i)
            if (screen[(size_t)i].second != 0) fin.push_back(screen[(size_t)i].second);
        std::sort(fin.begin(), fin.end());  // candidate order is the prior
        TuneChoice best = kTuneCandidates[fin[0]];
        double best_rate = 0;
        bool have = false;
        for (int t : fin) {
            const double rate = trial(kTuneCandidates[t], true);
            if (!have || rate > best_rate * 1.05) {
                best = kTuneCandidates[t];
                best_rate = rate;
                have = true;
            }
        }
        return best;
    }

    int finish_failed(const std::vector<int>& jstat, double t0) {
        int first_bad = GSOFA_OK;
        for (size_t j = 0; j < jstat.size(); ++j) {
            gsofa_result* r = new_result();
            r->n = mats[j].n;
            r->stats.status = jstat[j];
            r->stats.t_total_ms = now_ms() - t0;
            results[j] = r;
            if (jstat[j] != GSOFA_OK && first_bad == GSOFA_OK) first_bad = jstat[j];
        }
        return first_bad;
    }
};

void free_result(gsofa_result* r) {
    if (!r) return;
    auto* own = static_cast<ResultOwner*>(r->internal_);
    delete own;
    std::free(r);
}

Plan make_plan(const gsofa_opts* o) {
    Plan p{};
    p.window = 0;
    p.nslots = 0;
    p.max_super = 128;
    p.flags = 0;
    p.budget = 0;
    p.window_auto = false;
    p.allow_trials = true;
    p.queue_cap = 0;
    p.slot_div = 1;
    if (o) {
        p.flags = o->flags;
        p.budget = o->mem_budget_bytes;
        p.nslots = o->concurrent_sources;
        if (o->max_supernode > 0) p.max_super = o->max_supernode;
        else if (o->max_supernode < 0) p.max_super = 0;
        p.window = o->window;
        p.queue_cap = o->queue_cap;
    }
    return p;
}

int check_opts(const gsofa_opts* o) {
    if (!o) return GSOFA_OK;
    if (o->struct_size != 0 && o->struct_size < sizeof(gsofa_opts)) return GSOFA_EINVAL;
    if (o->mem_budget_bytes < 0 || o->window < 0 || o->concurrent_sources < 0) return GSOFA_EINVAL;
    if ((o->dev_alloc == nullptr) != (o->dev_free == nullptr)) return GSOFA_EINVAL;
    if (o->queue_cap < 0) return GSOFA_EINVAL;
    return GSOFA_OK;
}

std::mutex g_api_mu;  // one call at a time per process for the plain entry points

int run_engine(std::vector<MatIn> mats, const gsofa_opts* o, std::vector<gsofa_result*>& outs,
               bool allow_trials = true, bool tuned_with_slots = false, const YieldHooks* yh = nullptr) {
    Engine eng;
    eng.mats = std::move(mats);
    eng.plan = make_plan(o);
    eng.yh = yh;
    eng.plan.allow_trials = allow_trials && !(eng.plan.flags & GSOFA_NO_TUNE);
    eng.on_device = o && (o->flags & GSOFA_INPUT_ON_DEVICE);
    eng.st = o ? static_cast<hipStream_t>(o->stream) : nullptr;
    int64_t N = 1, rows = 0;
    for (auto& m : eng.mats) {
        N = std::max<int64_t>(N, m.n);
        rows += std::max<int32_t>(m.n, 0);
    }
    // the server gives a request its sources in flight and still takes the
    // cached mapping and window of its size class
    eng.plan.window_auto = eng.plan.window <= 0 && (eng.plan.nslots <= 0 || tuned_with_slots) &&
                           (eng.plan.flags & (GSOFA_MAP_WAVE32 | GSOFA_MAP_WAVE32_7 | GSOFA_MAP_WG8 | GSOFA_MAP_WG16 | GSOFA_MAP_BYTE |
                                              GSOFA_LEVEL_ORDER | GSOFA_NO_LINE95 | GSOFA_BUDGET_MODE | GSOFA_MAP_THREAD |
                                              GSOFA_RESET_LABELS)) == 0;
    if (eng.plan.window <= 0) eng.plan.window = auto_window(rows);
    if (eng.plan.flags & GSOFA_LEVEL_ORDER) eng.plan.window = (int32_t)std::min<int64_t>(N, 0x7FFFFFFF);
    // a caller allocator serves every device buffer of this call; buffers it
    // releases early go back once the call's device work has completed
    struct AllocScope {
        std::shared_ptr<CallerAlloc> prev, cur;
        hipStream_t st;
        ~AllocScope() {
            if (cur) {
                (void)hipStreamSynchronize(st);
                (void)hipGetLastError();
                cur->flush();
            }
            t_calloc = prev;
        }
    } as{t_calloc, nullptr, eng.st};
    if (o && o->dev_alloc) {
        as.cur = std::make_shared<CallerAlloc>();
        as.cur->alloc_fn = o->dev_alloc;
        as.cur->free_fn = o->dev_free;
        as.cur->ctx = o->alloc_ctx;
    }
    t_calloc = as.cur;
    int rc;
    try {
        rc = eng.run();
    } catch (const HipError&) {
        (void)hipGetLastError();
        for (auto* r : eng.results) free_result(r);
        return GSOFA_EDEVICE;
    } catch (const Status& s) {
        for (auto* r : eng.results) free_result(r);
        return s.code;
    } catch (const std::bad_alloc&) {
        for (auto* r : eng.results) free_result(r);
        return GSOFA_ENOMEM;
    }
    outs = eng.results;
    return rc;
}

}  // namespace
}  // namespace gsofa

using namespace gsofa;

// ------------------------------------------------------------------ the ABI

extern "C" GSOFA_API int gsofa_symbolic(int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
                              const gsofa_opts* opts, gsofa_result** out) {
    if (!out) return GSOFA_EINVAL;
    int rc = check_opts(opts);
    if (rc != GSOFA_OK) return rc;
    if (n < 0 || n > GSOFA_MAX_N) return GSOFA_EINVAL;
    const bool on_dev = opts && (opts->flags & GSOFA_INPUT_ON_DEVICE);
    if (n > 0 && (!row_ptr || !col_idx)) {
        // col_idx may be NULL only for an empty pattern
        if (!row_ptr) return GSOFA_EINVAL;
        if (!on_dev && row_ptr[n] != 0) return GSOFA_EINVAL;
    }
    if (!on_dev) {
        std::vector<uint32_t> stamp;
        rc = check_csr_host(n, row_ptr, col_idx, stamp);
        if (rc != GSOFA_OK) return rc;
    }
    std::lock_guard<std::mutex> g(g_api_mu);
    std::vector<gsofa_result*> outs;
    rc = run_engine({MatIn{n, row_ptr, col_idx}}, opts, outs);
    if (rc != GSOFA_OK) {
        for (auto* r : outs) free_result(r);
        return rc;
    }
    *out = outs[0];
    return GSOFA_OK;
}

extern "C" GSOFA_API int gsofa_batch(int32_t count, const gsofa_csr* mats, const gsofa_opts* opts,
                           gsofa_result** outs) {
    if (count < 0 || (count > 0 && (!mats || !outs))) return GSOFA_EINVAL;
    int rc = check_opts(opts);
    if (rc != GSOFA_OK) return rc;
    if (count == 0) return GSOFA_OK;
    const bool on_dev = opts && (opts->flags & GSOFA_INPUT_ON_DEVICE);
    std::vector<MatIn> in;
    std::vector<int> pre(count, GSOFA_OK);
    std::vector<uint32_t> stamp;
    for (int32_t i = 0; i < count; ++i) {
        if (!on_dev) pre[i] = check_csr_host(mats[i].n, mats[i].row_ptr, mats[i].col_idx, stamp);
        else if (mats[i].n < 0 || mats[i].n > GSOFA_MAX_N || (mats[i].n > 0 && !mats[i].row_ptr))
            pre[i] = GSOFA_EINVAL;
    }
    std::vector<int32_t> idx;
    for (int32_t i = 0; i < count; ++i)
        if (pre[i] == GSOFA_OK) {
            in.push_back(MatIn{mats[i].n, mats[i].row_ptr, mats[i].col_idx});
            idx.push_back(i);
        }
    std::lock_guard<std::mutex> g(g_api_mu);
    std::vector<gsofa_result*> res;
    int first_bad = GSOFA_OK;
    if (!in.empty()) {
        rc = run_engine(in, opts, res);
        if (res.empty()) return rc;  // device or memory failure: nothing produced
        if (rc != GSOFA_OK) first_bad = rc;
    }
    size_t k = 0;
    for (int32_t i = 0; i < count; ++i) {
        if (pre[i] == GSOFA_OK) {
            outs[i] = res[k++];
        } else {
            gsofa_result* r = nullptr;
            try {
                r = new_result();
            } catch (...) {
                return GSOFA_ENOMEM;
            }
            r->n = mats[i].n;
            r->stats.status = pre[i];
            outs[i] = r;
            if (first_bad == GSOFA_OK) first_bad = pre[i];
        }
    }
    return first_bad;
}

extern "C" GSOFA_API void gsofa_result_free(gsofa_result* r) { free_result(r); }

extern "C" GSOFA_API const char* gsofa_strerror(int s) {
    switch (s) {
        case GSOFA_OK: return "ok";
        case GSOFA_EINVAL: return "invalid argument or malformed CSR";
        case GSOFA_ENOMEM: return "device memory budget too small";
        case GSOFA_EDEVICE: return "HIP runtime failure";
        case GSOFA_EAGAIN: return "request not finished";
        case GSOFA_ECAPACITY: return "request exceeds the admission budget";
        case GSOFA_ENOTFOUND: return "unknown ticket";
        default: return "unknown status";
    }
}

extern "C" GSOFA_API int gsofa_release_cache(void) {
    std::lock_guard<std::mutex> g(g_api_mu);
    drop_idle_slots();
    cache().release();
    spill_cache().release();
    return GSOFA_OK;
}

extern "C" GSOFA_API int gsofa_memory_counters(uint64_t* out) {
    if (!out) return GSOFA_EINVAL;
    out[0] = g_hip_bytes_held.load();
    out[1] = g_hip_mallocs.load();
    out[2] = g_caller_bytes.load();
    out[3] = g_caller_allocs.load();
    out[4] = g_caller_frees.load();
    return GSOFA_OK;
}

extern "C" GSOFA_API int gsofa_graph_counters(uint64_t* out) {
    if (!out) return GSOFA_EINVAL;
    out[0] = g_graph_instantiations.load();
    out[1] = g_graph_updates.load();
    out[2] = g_graph_launches.load();
    return GSOFA_OK;
}

// ------------------------------------------------------------ the server
//
// Continuous batching: max_inflight worker threads, each with its own stream,
// take the oldest queued request whose memory estimate fits what is left of the
// budget (serve_pick), together with later small ones that fit. Requests that
// arrive while others run are admitted as soon as a worker and memory are free,
// and their kernels overlap on the device with the running ones. A finished
// request returns its memory to the budget and wakes the waiting workers.

struct gsofa_server {
    gsofa_opts opts{};
    int32_t max_inflight = 4;
    int64_t budget = 0;
    std::mutex mu;
    std::condition_variable cv;
    bool closing = false;
    uint64_t next_ticket = 1;
    struct Req {
        uint64_t ticket;
        int32_t n;
        std::vector<int32_t> rp, ci;
        int64_t est;
        int32_t nslots;  // sources in flight for this request
        int32_t passed = 0;  // times a later request was admitted before this one
    };
    std::deque<Req> queue;
    int32_t inflight = 0;
    int64_t mem_in_use = 0;
    std::map<uint64_t, std::pair<int, gsofa_result*>> done;
    std::map<uint64_t, bool> known;  // tickets not yet collected
    std::vector<hipStream_t> streams;
    std::vector<std::thread> workers;
    int device = 0;
    int32_t slots_total = 5120;
    // work-item admission: per worker, its yield flag (one 64-byte line of
    // fine-grained pinned host memory each) and the state of its traversal
    struct Worker {
        uint32_t* flag = nullptr;
        bool traversing = false;   // its traversal launches hold wave slots
        bool yieldable = false;    // its current call polls the flag (a large request)
        int32_t slots = 0;         // sources in flight of its current call
        bool alone = false;        // its call was given the idle device's wave slots
        bool alone_trav = false;   // ... and its traversal has not ended yet
        double last_yield_ms = -1e300;
        uint64_t wait_for = 0;     // the admission it last yielded to
    };
    std::vector<Worker> wk;
    void* flag_mem = nullptr;
    uint64_t admit_seq = 0;
    std::map<uint64_t, bool> admits_pending;  // admissions whose traversal is not enqueued yet
    uint64_t yields = 0;                       // yield requests made (statistics)
};

namespace {

int64_t estimate_request_bytes(int32_t n, int64_t nnz, int32_t nslots) {
    const SlotLayout lay = slot_layout(std::max<int64_t>(n, 1));
    return budget_for(n, nnz, nslots, lay);
}

// Wave slots no request's traversal takes by default: the row sorts, the L
// transpose and the supernode kernels of a request admitted while large
// traversals run find room there instead of waiting for their next yield.
constexpr int32_t kServeReserveSlots = 256;

// Sources in flight for one request: a share of the resident wavefronts less
// the reserve (two requests' kernels fill the rest), never more than the
// request has rows, and few enough that the request's estimate fits the whole
// budget; 0 if even one source does not fit.
int32_t serve_slots_for(const gsofa_server* s, int32_t n, int64_t nnz) {
    int32_t want;
    if (s->opts.concurrent_sources > 0) {
        want = std::min(s->opts.concurrent_sources, std::max(n, 1));
    } else {
        const int32_t share = (s->slots_total - kServeReserveSlots) / std::max(1, s->max_inflight / 2) / 4 * 4;
        want = std::min(std::max(share, 64), std::max(n, 1));
    }
    const SlotLayout lay = slot_layout(std::max<int64_t>(n, 1));
    const int64_t rest = s->budget - budget_for(n, nnz, 0, lay);
    const int64_t fit = rest > 0 ? rest / (2 * lay.bytes_per_slot) : 0;
    return (int32_t)std::min<int64_t>(want, fit);
}

// Sources in flight for a request admitted onto an idle server (nothing running,
// nothing queued): every resident wavefront but the reserve, within the budget.
// The share above assumes two large requests at once; a lone one would leave
// half the device idle (the largest request of a 1-per-second stream took
// 141 ms against 110 ms as a plain call).
int32_t serve_slots_alone(const gsofa_server* s, int32_t n, int64_t nnz) {
    const int32_t want = std::min((s->slots_total - kServeReserveSlots) / 4 * 4, std::max(n, 1));
    const SlotLayout lay = slot_layout(std::max<int64_t>(n, 1));
    const int64_t rest = s->budget - s->mem_in_use - budget_for(n, nnz, 0, lay);
    const int64_t fit = rest > 0 ? rest / (2 * lay.bytes_per_slot) : 0;
    return (int32_t)std::min<int64_t>(want, fit);
}

// Requests of at most kServeSmallRows rows admitted together share one engine
// call: one persistent traversal launch over all their sources, as in
// gsofa_batch. Larger requests run alone (their own launch fills the device).
constexpr int32_t kServeSmallRows = 65536;
constexpr size_t kServeMaxGroup = 64;
constexpr int64_t kServeGroupRows = 1 << 20;

// Admission order: the oldest queued request that fits the memory left, so a
// large request waiting for memory does not block smaller ones behind it; once
// the oldest has been passed kServeMaxPassed times, nothing passes it any more
// and it is admitted as soon as its memory is free.
constexpr int32_t kServeMaxPassed = 32;

// Work-item admission (GSOFA_SERVE_YIELD): when a worker admits a request and
// the traversals already running hold so many wave slots that its own would
// find no room, it sets their yield flags. Each running launch then takes no further source,
// finishes the ones it holds and ends; its engine relaunches from the work
// counter once the new request's traversal is on its stream (or after
// kServeResumeWaitMs), so the new request's wavefronts are dispatched first. A
// traversal is asked at most once per kServeYieldGapMs, which bounds what a
// stream of small requests costs a large one (a drain of about half a source
// per slot each time).
constexpr double kServeYieldGapMs = 20.0;
constexpr int kServeResumeWaitMs = 20;

long serve_pick(const gsofa_server* s) {
    if (s->queue.empty()) return -1;
    const auto fits = [&](const gsofa_server::Req& r) { return s->mem_in_use + r.est <= s->budget; };
    if (s->queue.front().passed >= kServeMaxPassed) return fits(s->queue.front()) ? 0 : -1;
    for (size_t i = 0; i < s->queue.size(); ++i)
        if (fits(s->queue[i])) return (long)i;
    return -1;
}

void serve_worker(gsofa_server* s, int sid) {
    (void)hipSetDevice(s->device);
    gsofa_server::Worker& me = s->wk[(size_t)sid];
    for (;;) {
        std::vector<gsofa_server::Req> grp;
        int64_t grp_est = 0;
        int32_t want = 0;
        uint64_t my_admit = 0;  // set if this admission asked running traversals to yield
        {
            std::unique_lock<std::mutex> lk(s->mu);
            long pick = -1;
            s->cv.wait(lk, [&] {
                if (s->queue.empty()) return s->closing;
                pick = serve_pick(s);
                return pick >= 0;
            });
            if (s->queue.empty()) return;  // closing and drained
            if (pick > 0) s->queue.front().passed++;
            grp.push_back(std::move(s->queue[(size_t)pick]));
            s->queue.erase(s->queue.begin() + pick);
            grp_est = grp[0].est;
            if (grp[0].n <= kServeSmallRows) {
                // later small requests that fit the memory budget join, in arrival order
                int64_t rows = grp[0].n;
                for (auto it = s->queue.begin(); it != s->queue.end() && grp.size() < kServeMaxGroup;) {
                    if (it->n <= kServeSmallRows && rows + it->n <= kServeGroupRows &&
                        s->mem_in_use + grp_est + it->est <= s->budget) {
                        rows += it->n;
                        grp_est += it->est;
                        grp.push_back(std::move(*it));
                        it = s->queue.erase(it);
                    } else {
                        ++it;
                    }
                }
            }
            if (grp.size() == 1 && s->inflight == 0 && s->queue.empty() && s->opts.concurrent_sources <= 0) {
                const int32_t slots = serve_slots_alone(s, grp[0].n, (int64_t)grp[0].ci.size());
                if (slots > grp[0].nslots) {
                    me.alone = me.alone_trav = true;
                    grp[0].nslots = slots;
                    grp[0].est = estimate_request_bytes(grp[0].n, (int64_t)grp[0].ci.size(), slots);
                    grp_est = grp[0].est;
                }
            }
            s->inflight++;
            s->mem_in_use += grp_est;
            int64_t rows = 0;
            for (auto& r : grp) rows += r.n;
            want = grp.size() == 1 ? grp[0].nslots : (int32_t)std::min<int64_t>(rows, s->slots_total);
            int64_t busy = 0;
            bool gated = false;  // waits for a lone request's traversal (below): nothing to yield to
            for (auto& w : s->wk) {
                if (w.traversing) busy += w.slots;
                if (w.alone_trav && !me.alone && grp.size() == 1 && grp[0].n > kServeSmallRows) gated = true;
            }
            if ((s->opts.flags & GSOFA_SERVE_YIELD) && !gated && busy + want > s->slots_total - kServeReserveSlots) {
                const double now = now_ms();
                const uint64_t id = ++s->admit_seq;
                for (auto& w : s->wk)
                    if (w.traversing && w.yieldable && now - w.last_yield_ms >= kServeYieldGapMs) {
                        __atomic_store_n(w.flag, 1u, __ATOMIC_RELEASE);
                        w.last_yield_ms = now;
                        w.wait_for = id;
                        my_admit = id;
                        s->yields++;
                    }
                if (my_admit) s->admits_pending[my_admit] = true;
            }
            s->wk[(size_t)sid].slots = want;
            // only a lone large request polls the flag: its sources take
            // milliseconds each, so one host-memory read per source costs
            // nothing, while a group of small requests would poll millions of
            // times a second (and finishes soon anyway)
            s->wk[(size_t)sid].yieldable =
                (s->opts.flags & GSOFA_SERVE_YIELD) && grp.size() == 1 && grp[0].n > kServeSmallRows;
        }
        gsofa_opts o = s->opts;
        o.stream = s->streams[sid];
        o.flags &= ~(uint32_t)GSOFA_INPUT_ON_DEVICE;
        o.mem_budget_bytes = grp_est;
        // a lone request keeps its planned share of sources; a group plans from its budget
        o.concurrent_sources = grp.size() == 1 ? grp[0].nslots : 0;
        std::vector<MatIn> mats;
        for (auto& r : grp) mats.push_back(MatIn{r.n, r.rp.data(), r.ci.data()});
        std::vector<gsofa_result*> outs;
        // no tuner trials inside a request (they would add to its latency), but
        // the size class's cached choice of mapping and window applies
        YieldHooks hooks;
        hooks.flag = me.yieldable ? me.flag : nullptr;
        // a request set it after this worker's previous traversal had ended
        __atomic_store_n(me.flag, 0u, __ATOMIC_RELEASE);
        // the traversal is on the stream: it holds wave slots, and the
        // traversals that yielded to this admission may resume
        auto admitted_done = [&] {
            if (my_admit) {
                s->admits_pending.erase(my_admit);
                my_admit = 0;
                s->cv.notify_all();
            }
        };
        hooks.enqueued = [&] {
            std::lock_guard<std::mutex> g(s->mu);
            me.traversing = true;
            admitted_done();
        };
        hooks.finished = [&] {
            std::lock_guard<std::mutex> g(s->mu);
            me.traversing = false;
            if (me.alone_trav) {
                me.alone_trav = false;
                s->cv.notify_all();
            }
        };
        // A large request admitted while one that was given the idle device
        // traverses uploads and sorts at once but starts its traversal when that
        // traversal ends: its wavefronts could only queue behind it, and would
        // take the reserve the small requests need as they got room.
        if (!me.alone && grp.size() == 1 && grp[0].n > kServeSmallRows)
            hooks.before_traverse = [&] {
                std::unique_lock<std::mutex> lk(s->mu);
                s->cv.wait(lk, [&] {
                    for (auto& w : s->wk)
                        if (w.alone_trav) return false;
                    return true;
                });
            };
        hooks.before_resume = [&] {
            std::unique_lock<std::mutex> lk(s->mu);
            const uint64_t id = me.wait_for;
            s->cv.wait_for(lk, std::chrono::milliseconds(kServeResumeWaitMs),
                           [&] { return s->closing || s->admits_pending.count(id) == 0; });
        };
        const int rc = run_engine(std::move(mats), &o, outs, false, true, &hooks);
        std::lock_guard<std::mutex> g(s->mu);
        me.traversing = false;
        admitted_done();
        for (size_t i = 0; i < grp.size(); ++i) {
            gsofa_result* res = i < outs.size() ? outs[i] : nullptr;
            int st = res ? res->stats.status : (rc != GSOFA_OK ? rc : GSOFA_EDEVICE);
            if (res && st != GSOFA_OK) {
                free_result(res);
                res = nullptr;
            }
            s->done[grp[i].ticket] = {st, res};
        }
        s->inflight--;
        me.alone = me.alone_trav = false;
        s->mem_in_use -= grp_est;
        s->cv.notify_all();
    }
}

}  // namespace

extern "C" GSOFA_API int gsofa_serve_open(const gsofa_opts* opts, int32_t max_inflight, gsofa_server** srv) {
    if (!srv || max_inflight < 0) return GSOFA_EINVAL;
    int rc = check_opts(opts);
    if (rc != GSOFA_OK) return rc;
    auto* s = new (std::nothrow) gsofa_server();
    if (!s) return GSOFA_ENOMEM;
    if (opts) s->opts = *opts;
    s->opts.stream = nullptr;
    s->max_inflight = max_inflight > 0 ? max_inflight : 4;
    try {
        (void)hipGetDevice(&s->device);
        DeviceInfo di = device_info();
        s->slots_total = traverse_resident_slots(di.cus, 0);
        s->budget = s->opts.mem_budget_bytes > 0 ? s->opts.mem_budget_bytes
                                                 : (int64_t)((di.free_b + di.reclaimable) * 0.85);
        s->streams.assign(s->max_inflight, nullptr);
        for (auto& st : s->streams) chk(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        // yield flags: fine-grained (coherent) pinned memory, so that a running
        // kernel sees the host's store
        chk(hipHostMalloc(&s->flag_mem, 64 * (size_t)s->max_inflight, hipHostMallocCoherent));
        std::memset(s->flag_mem, 0, 64 * (size_t)s->max_inflight);
        s->wk.resize((size_t)s->max_inflight);
        for (int i = 0; i < s->max_inflight; ++i)
            s->wk[(size_t)i].flag = reinterpret_cast<uint32_t*>(static_cast<char*>(s->flag_mem) + 64 * i);
    } catch (...) {
        for (auto st : s->streams)
            if (st) (void)hipStreamDestroy(st);
        if (s->flag_mem) (void)hipHostFree(s->flag_mem);
        delete s;
        return GSOFA_EDEVICE;
    }
    for (int i = 0; i < s->max_inflight; ++i) s->workers.emplace_back(serve_worker, s, i);
    *srv = s;
    return GSOFA_OK;
}

extern "C" GSOFA_API int gsofa_serve_submit(gsofa_server* s, const gsofa_csr* m, uint64_t* ticket) {
    if (!s || !m || !ticket) return GSOFA_EINVAL;
    std::vector<uint32_t> stamp;
    int rc = check_csr_host(m->n, m->row_ptr, m->col_idx, stamp);
    if (rc != GSOFA_OK) return rc;
    gsofa_server::Req r;
    r.n = m->n;
    const int64_t nnz = m->n > 0 ? m->row_ptr[m->n] : 0;
    try {
        if (m->n > 0) {
            r.rp.assign(m->row_ptr, m->row_ptr + m->n + 1);
            r.ci.assign(m->col_idx, m->col_idx + nnz);
        } else {
            r.rp.assign(1, 0);
        }
    } catch (const std::bad_alloc&) {
        return GSOFA_ENOMEM;
    }
    r.nslots = serve_slots_for(s, m->n, nnz);
    if (r.nslots < 1) return GSOFA_ECAPACITY;
    r.est = estimate_request_bytes(m->n, nnz, r.nslots);
    std::lock_guard<std::mutex> g(s->mu);
    if (s->closing) return GSOFA_EINVAL;
    if (r.est > s->budget) return GSOFA_ECAPACITY;
    r.ticket = s->next_ticket++;
    *ticket = r.ticket;
    s->known[r.ticket] = true;
    s->queue.push_back(std::move(r));
    s->cv.notify_all();
    return GSOFA_OK;
}

extern "C" GSOFA_API int gsofa_serve_poll(gsofa_server* s, uint64_t ticket, int32_t timeout_us, gsofa_result** out) {
    if (!s || !out) return GSOFA_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (!s->known.count(ticket)) return GSOFA_ENOTFOUND;
    auto ready = [&] { return s->done.count(ticket) > 0; };
    if (!ready()) {
        if (timeout_us == 0) return GSOFA_EAGAIN;
        if (timeout_us < 0) s->cv.wait(lk, ready);
        else if (!s->cv.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) return GSOFA_EAGAIN;
    }
    auto it = s->done.find(ticket);
    const int rc = it->second.first;
    gsofa_result* r = it->second.second;
    s->done.erase(it);
    s->known.erase(ticket);
    if (rc == GSOFA_OK) *out = r;
    return rc;
}

extern "C" GSOFA_API int gsofa_serve_close(gsofa_server* s) {
    if (!s) return GSOFA_EINVAL;
    {
        // requests not admitted yet are dropped; running ones finish
        std::lock_guard<std::mutex> g(s->mu);
        s->closing = true;
        for (auto& r : s->queue) s->known.erase(r.ticket);
        s->queue.clear();
        s->cv.notify_all();
    }
    for (auto& t : s->workers)
        if (t.joinable()) t.join();
    for (auto& kv : s->done) free_result(kv.second.second);
    for (auto st : s->streams) (void)hipStreamDestroy(st);
    if (s->flag_mem) (void)hipHostFree(s->flag_mem);
    delete s;
    return GSOFA_OK;
}
