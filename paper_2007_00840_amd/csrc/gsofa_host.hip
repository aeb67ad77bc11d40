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
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
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

struct StreamScope {
    hipStream_t prev;
    explicit StreamScope(hipStream_t s) : prev(t_stream) { t_stream = s; }
    ~StreamScope() { t_stream = prev; }
};

void drop_idle_slots();

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
        if (e != hipSuccess) {
            (void)hipGetLastError();
            drop_idle_slots();
            release();
            e = hipMalloc(&p, bytes);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                throw Status{GSOFA_ENOMEM};
            }
        }
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
    void release() {
        std::lock_guard<std::mutex> g(mu_);
        for (auto& kv : free_) {
            if (kv.second.ev) {
                (void)hipEventSynchronize(kv.second.ev);
                (void)hipEventDestroy(kv.second.ev);
            }
            (void)hipFree(kv.second.p);
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

// A device buffer taken from the cache on the calling thread's engine stream,
// returned with that stream's ordering on destruction.
struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipStream_t st = nullptr;
    bool synced = false;  // set once no work on the buffer can be pending
    DBuf() = default;
    explicit DBuf(size_t b) : p(cache().alloc(b, t_stream)), bytes(b), st(t_stream) {}
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    DBuf(DBuf&& o) noexcept : p(o.p), bytes(o.bytes), st(o.st), synced(o.synced) { o.p = nullptr; }
    DBuf& operator=(DBuf&& o) noexcept {
        if (this != &o) {
            reset();
            p = o.p;
            bytes = o.bytes;
            st = o.st;
            synced = o.synced;
            o.p = nullptr;
        }
        return *this;
    }
    ~DBuf() { reset(); }
    void reset() {
        if (p) cache().free(p, st, synced);
        p = nullptr;
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
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
    {
        std::lock_guard<std::mutex> g(g_slot_mu);
        auto& v = idle_slots();
        for (size_t i = 0; i < v.size(); ++i) {
            if (v[i]->lay.N == lay.N && v[i]->nslots >= nslots) {
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

struct DeviceInfo {
    int cus = 256;
    size_t free_b = 0, total_b = 0;
};

DeviceInfo device_info() {
    DeviceInfo d;
    int dev = 0;
    chk(hipGetDevice(&dev));
    hipDeviceProp_t p;
    chk(hipGetDeviceProperties(&p, dev));
    d.cus = p.multiProcessorCount;
    chk(hipMemGetInfo(&d.free_b, &d.total_b));
    return d;
}

// ------------------------------------------------------------ input checks

int check_csr_host(int32_t n, const int32_t* rp, const int32_t* ci, std::vector<uint32_t>& stamp) {
    if (n < 0) return GSOFA_EINVAL;
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
    // host arrays (malloc) or device buffers shared by the results of one call
    std::vector<void*> host;
    std::shared_ptr<std::vector<DBuf>> dev;
};

gsofa_result* new_result() {
    auto* r = static_cast<gsofa_result*>(std::calloc(1, sizeof(gsofa_result)));
    if (!r) throw Status{GSOFA_ENOMEM};
    r->internal_ = new ResultOwner();
    return r;
}

template <typename T>
T* host_array(gsofa_result* r, int64_t count) {
    void* p = std::malloc(sizeof(T) * (size_t)std::max<int64_t>(count, 1));
    if (!p) throw Status{GSOFA_ENOMEM};
    static_cast<ResultOwner*>(r->internal_)->host.push_back(p);
    return static_cast<T*>(p);
}

// ------------------------------------------------------------ the pipeline

struct MatIn {
    int32_t n;
    const int32_t* rp;
    const int32_t* ci;
};

struct Plan {
    int32_t window;
    int32_t nslots;
    int32_t max_super;  // <= 0: unbounded
    uint32_t flags;
    int64_t budget;
};

// Traversal mapping. One wavefront per source is the default: per-source
// frontiers are small (a window holds a few dozen vertices), so a workgroup per
// source leaves most of its wavefronts idle and was 3-5x slower on the 64^3
// and 1000^2 stencils. The workgroup variants stay available as tuning knobs.
// Byte states (mapping 3) need windows of at most 253 ids and keep no label
// for vertices already in the structure, so the paper's order (window = n) and
// the line-9.5-off ablation run on 32-bit labels (mapping 0).
int choose_mapping(uint32_t flags, int32_t window) {
    if (flags & GSOFA_MAP_WG16) return 1;
    if (flags & GSOFA_MAP_WG8) return 2;
    if (flags & GSOFA_MAP_WAVE32) return 0;
    if (window > 253 || (flags & (GSOFA_NO_LINE95 | GSOFA_LEVEL_ORDER))) return 0;
    return 3;
}

int32_t auto_window(int64_t N) {
    // Window span for the traversal schedule. Small spans keep revisits low,
    // wider ones give fuller wavefronts; 16 was the best measured trade-off on
    // 2D and 3D stencils in nested-dissection order.
    (void)N;
    return 16;
}

struct EngineOut {
    int status = GSOFA_OK;
    std::vector<int> job_status;
};

// Per-launch fill-ratio memory used to size the output pool of later calls.
std::atomic<double> g_fill_ratio{48.0};

// Device bytes a launch needs besides slots and output pool: inputs, per-row
// arrays, assembly buffers, scratch.
int64_t fixed_bytes(int64_t nrows, int64_t nnz) { return nrows * 40 + nnz * 8 + (64ll << 20); }

// Output-pool entries expected for nnz stored entries.
int64_t pool_estimate(int64_t nrows, int64_t nnz) {
    return std::max<int64_t>((int64_t)(g_fill_ratio.load() * (double)nnz * 1.15) + nrows, 1 << 20);
}

// Budget under which the planner below gives nslots slots and the expected
// pool: half of the room after fixed_bytes goes to slots, and the pool may
// take up to a third of the rest in 4-byte entries.
int64_t budget_for(int64_t nrows, int64_t nnz, int64_t nslots, const SlotLayout& lay) {
    return fixed_bytes(nrows, nnz) + 2 * nslots * lay.bytes_per_slot + 12 * pool_estimate(nrows, nnz);
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

struct Engine {
    std::vector<MatIn> mats;
    bool on_device = false;
    gsofa_opts o{};
    Plan plan{};
    hipStream_t st = nullptr;

    // outputs
    std::vector<gsofa_result*> results;

    int run() {
        const double t0 = now_ms();
        StreamScope scope(st);
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
            for (int32_t j = 0; j < nj; ++j) {
                int32_t last = 0;
                if (mats[j].n > 0) chk(hipMemcpyAsync(&last, mats[j].rp + mats[j].n, 4, hipMemcpyDeviceToHost, st));
                chk(hipStreamSynchronize(st));
                if (last < 0) jstat[j] = GSOFA_EINVAL;
                nnz[j] = last;
                jobs[j].row_ptr = mats[j].rp;
                jobs[j].col_idx = mats[j].ci;
            }
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
            // pack through a pinned staging buffer
            const size_t stage_b = 4 * (size_t)(rp_tot + ci_tot);
            void* stage = nullptr;
            chk(hipHostMalloc(&stage, std::max<size_t>(stage_b, 4), hipHostMallocDefault));
            int32_t* sp = static_cast<int32_t*>(stage);
            for (int32_t j = 0; j < nj; ++j) {
                if (mats[j].n > 0) {
                    std::memcpy(sp + rp_off[j], mats[j].rp, 4 * (size_t)(mats[j].n + 1));
                    if (nnz[j] > 0) std::memcpy(sp + rp_tot + ci_off[j], mats[j].ci, 4 * (size_t)nnz[j]);
                } else {
                    sp[rp_off[j]] = 0;
                }
            }
            chk(hipMemcpyAsync(in_rp.p, sp, 4 * (size_t)rp_tot, hipMemcpyHostToDevice, st));
            if (ci_tot > 0)
                chk(hipMemcpyAsync(in_ci.p, sp + rp_tot, 4 * (size_t)ci_tot, hipMemcpyHostToDevice, st));
            chk(hipStreamSynchronize(st));
            (void)hipHostFree(stage);
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
        chk(hipMemcpyAsync(d_jobs.p, jt.data(), sizeof(Job) * nj, hipMemcpyHostToDevice, st));

        if (on_device) {
            DBuf bad(4 * std::max(nj, 1));
            chk(launch_zero_i32(bad.as<int32_t>(), nj, st));
            chk(launch_validate(d_jobs.as<Job>(), nj, N, bad.as<int32_t>(), st));
            std::vector<int32_t> hb(nj);
            chk(hipMemcpyAsync(hb.data(), bad.p, 4 * nj, hipMemcpyDeviceToHost, st));
            chk(hipStreamSynchronize(st));
            for (int32_t q = 0; q < nj; ++q)
                if (hb[q]) jstat[ord[q]] = GSOFA_EINVAL;
            bool any_bad = false;
            for (int32_t j = 0; j < nj; ++j) any_bad |= jstat[j] != GSOFA_OK;
            if (any_bad) return finish_failed(jstat, t0);
        }

        // ---- plan the concurrent sources
        const SlotLayout lay = slot_layout(N);
        const DeviceInfo di = device_info();
        int64_t budget = plan.budget > 0 ? plan.budget : (int64_t)(di.free_b * 0.9);
        const int64_t fixed = fixed_bytes(nrows, total_nnz);
        if (budget < fixed + lay.bytes_per_slot) throw Status{GSOFA_ENOMEM};
        const int mapping = choose_mapping(plan.flags, plan.window);
        int64_t want = plan.nslots > 0 ? plan.nslots : (int64_t)traverse_resident_slots(di.cus, mapping);
        want = std::min<int64_t>(want, std::max<int64_t>(items, 1));
        const int64_t slot_room = (budget - fixed) / 2;  // half of the rest for slots
        int64_t nslots = std::min<int64_t>(want, std::max<int64_t>(slot_room / lay.bytes_per_slot, 1));
        nslots = std::max<int64_t>(nslots, 1);
        // the one-wavefront mapping launches whole blocks of 4 wavefronts
        if ((mapping == 0 || mapping == 3) && nslots > 4) nslots = nslots / 4 * 4;

        int64_t pool_cap = pool_estimate(nrows, total_nnz);
        const int64_t pool_room = (budget - fixed - nslots * lay.bytes_per_slot) / 4 / 3;
        pool_cap = std::max<int64_t>(std::min<int64_t>(pool_cap, pool_room), nrows + 1024);

        auto slots = take_slots(lay, (int32_t)nslots, mapping == 3 ? 1 : 0, st);

        DBuf row_off(8 * (size_t)std::max<int64_t>(nrows, 1));
        DBuf row_cnt(4 * (size_t)std::max<int64_t>(nrows, 1));
        DBuf row_lcnt(4 * (size_t)std::max<int64_t>(nrows, 1));
        DBuf counters(64);  // [0] item counter, [1] pool tail
        DBuf jst(sizeof(JobStats) * std::max(nj, 1));
        DBuf pool(4 * (size_t)pool_cap);
        DBuf d_row_job;
        if (nj > 1) {
            d_row_job = DBuf(4 * (size_t)std::max<int64_t>(nrows, 1));
            chk(launch_row_job(d_jobs.as<Job>(), nj, N, d_row_job.as<int32_t>(), st));
        }
        chk(launch_zero_i32(counters.as<int32_t>(), 16, st));
        chk(launch_zero_i32(jst.as<int32_t>(), (int64_t)(sizeof(JobStats) / 4) * nj, st));

        // ev[0]/ev[4]: traversal kernel; ev[1]..ev[3]: assembly and supernode phases
        hipEvent_t ev[5];
        for (auto& e : ev) chk(hipEventCreate(&e));
        struct EvGuard {
            hipEvent_t* e;
            ~EvGuard() {
                for (int i = 0; i < 5; ++i) (void)hipEventDestroy(e[i]);
            }
        } evg{ev};

        TraverseArgs ta{};
        ta.jobs = d_jobs.as<Job>();
        ta.njobs = nj;
        ta.nslots = slots->nslots < nslots ? slots->nslots : (int32_t)nslots;
        ta.nitems = items;
        ta.item_rows = nullptr;
        ta.row_job = d_row_job.as<int32_t>();
        ta.item_counter = counters.as<unsigned long long>();
        ta.slots = slots->buf.as<uint8_t>();
        ta.lay = lay;
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
        chk(hipEventRecord(ev[0], st));
        chk(launch_traverse(ta, st));
        chk(hipEventRecord(ev[4], st));

        std::vector<JobStats> hst(nj);
        unsigned long long tail = 0;
        chk(hipMemcpyAsync(hst.data(), jst.p, sizeof(JobStats) * nj, hipMemcpyDeviceToHost, st));
        chk(hipMemcpyAsync(&tail, counters.as<unsigned long long>() + 1, 8, hipMemcpyDeviceToHost, st));
        chk(hipStreamSynchronize(st));

        bool overflow = false;
        float t_trav_extra = 0;
        for (int32_t q = 0; q < nj; ++q) {
            if (hst[q].err & kErrDuplicate) jstat[ord[q]] = GSOFA_EINVAL;
            if (hst[q].err & kErrOverflow) overflow = true;
        }
        if (overflow) {
            // rows that did not fit: grow the pool, keep what fits, redo the rest
            std::vector<int64_t> h_off(nrows);
            std::vector<int32_t> h_cnt(nrows);
            chk(hipMemcpyAsync(h_off.data(), row_off.p, 8 * nrows, hipMemcpyDeviceToHost, st));
            chk(hipMemcpyAsync(h_cnt.data(), row_cnt.p, 4 * nrows, hipMemcpyDeviceToHost, st));
            chk(hipStreamSynchronize(st));
            std::vector<int32_t> redo;
            int64_t need = 0;
            for (int64_t r = 0; r < nrows; ++r)
                if (h_off[r] < 0) {
                    redo.push_back((int32_t)r);
                    need += h_cnt[r];
                }
            const int64_t new_cap = pool_cap + need;
            DBuf pool2(4 * (size_t)new_cap);
            chk(hipMemcpyAsync(pool2.p, pool.p, 4 * (size_t)pool_cap, hipMemcpyDeviceToDevice, st));
            pool = std::move(pool2);
            DBuf d_redo(4 * redo.size());
            chk(hipMemcpyAsync(d_redo.p, redo.data(), 4 * redo.size(), hipMemcpyHostToDevice, st));
            unsigned long long cnt2[2] = {0ull, (unsigned long long)pool_cap};
            chk(hipMemcpyAsync(counters.p, cnt2, 16, hipMemcpyHostToDevice, st));
            ta.item_rows = d_redo.as<int32_t>();
            ta.nitems = (int64_t)redo.size();
            ta.pool = pool.as<int32_t>();
            ta.pool_cap = new_cap;
            // stats were already counted for these rows in the first pass: keep a copy
            std::vector<JobStats> keep = hst;
            chk(launch_zero_i32(jst.as<int32_t>(), (int64_t)(sizeof(JobStats) / 4) * nj, st));
            float first_ms = 0;
            chk(hipEventElapsedTime(&first_ms, ev[0], ev[4]));
            t_trav_extra += first_ms;
            chk(hipEventRecord(ev[0], st));
            chk(launch_traverse(ta, st));
            chk(hipEventRecord(ev[4], st));
            chk(hipMemcpyAsync(hst.data(), jst.p, sizeof(JobStats) * nj, hipMemcpyDeviceToHost, st));
            chk(hipMemcpyAsync(&tail, counters.as<unsigned long long>() + 1, 8, hipMemcpyDeviceToHost, st));
            chk(hipStreamSynchronize(st));
            for (int32_t q = 0; q < nj; ++q) {
                if (hst[q].err & kErrOverflow) throw Status{GSOFA_ENOMEM};
                if (hst[q].err & kErrDuplicate) jstat[ord[q]] = GSOFA_EINVAL;
                // the first pass already counted the redone rows' edges once
                hst[q].edges_alg = keep[q].edges_alg;
                hst[q].edges_gpu = keep[q].edges_gpu;
                hst[q].iterations = keep[q].iterations;
                hst[q].windows = keep[q].windows;
                hst[q].diag = keep[q].diag;
            }
            pool_cap = new_cap;
        }
        chk(hipEventRecord(ev[1], st));
        give_slots(std::move(slots));
        if (total_nnz > 0)
            g_fill_ratio.store(std::max(4.0, (double)tail / (double)total_nnz));

        // ---- assembly: counts -> pointers -> sorted rows (U CSR, L CSR)
        DBuf scan_scr(8 * (size_t)scan_scratch_elems(nrows + 1) + 64);
        DBuf u_ptr(8 * (size_t)(nrows + 1)), l_rptr(8 * (size_t)(nrows + 1));
        chk(launch_scan_counts(row_cnt.as<int32_t>(), row_lcnt.as<int32_t>(), nrows, u_ptr.as<int64_t>(),
                               scan_scr.as<int64_t>(), st));
        chk(launch_scan_counts(row_lcnt.as<int32_t>(), nullptr, nrows, l_rptr.as<int64_t>(),
                               scan_scr.as<int64_t>(), st));
        int64_t tot[2] = {0, 0};
        chk(hipMemcpyAsync(&tot[0], u_ptr.as<int64_t>() + nrows, 8, hipMemcpyDeviceToHost, st));
        chk(hipMemcpyAsync(&tot[1], l_rptr.as<int64_t>() + nrows, 8, hipMemcpyDeviceToHost, st));
        chk(hipStreamSynchronize(st));
        const int64_t nnz_u = tot[0], nnz_l = tot[1];
        DBuf u_idx(4 * (size_t)std::max<int64_t>(nnz_u, 1)), l_ridx(4 * (size_t)std::max<int64_t>(nnz_l, 1));
        DBuf big_list(4 * (size_t)std::max<int64_t>(nrows, 1)), big_cnt(64);
        DBuf d_jrb(8 * std::max(nj, 1)), d_jn(4 * std::max(nj, 1));
        std::vector<int32_t> jn(nj);
        for (int32_t j = 0; j < nj; ++j) jn[j] = mats[j].n;
        chk(hipMemcpyAsync(d_jrb.p, row_base.data(), 8 * nj, hipMemcpyHostToDevice, st));
        chk(hipMemcpyAsync(d_jn.p, jn.data(), 4 * nj, hipMemcpyHostToDevice, st));
        // rows of the global row space -> job in the user's order
        DBuf row_job_user;
        RowSpace rs{nrows, nullptr, nullptr};
        if (nj > 1) {
            row_job_user = DBuf(4 * (size_t)std::max<int64_t>(nrows, 1));
            // a job table in user order for k_row_job
            std::vector<Job> ju(nj);
            for (int32_t j = 0; j < nj; ++j) {
                ju[j] = jobs[j];
                ju[j].n = mats[j].n;
                ju[j].row_base = row_base[j];
            }
            DBuf d_ju(sizeof(Job) * nj);
            chk(hipMemcpyAsync(d_ju.p, ju.data(), sizeof(Job) * nj, hipMemcpyHostToDevice, st));
            chk(launch_row_job(d_ju.as<Job>(), nj, N, row_job_user.as<int32_t>(), st));
            chk(hipStreamSynchronize(st));
            rs.row_job = row_job_user.as<int32_t>();
            rs.job_row_base = d_jrb.as<int64_t>();
        }
        chk(launch_sort_rows(rs, row_off.as<int64_t>(), row_cnt.as<int32_t>(), row_lcnt.as<int32_t>(),
                             pool.as<int32_t>(), u_ptr.as<int64_t>(), u_idx.as<int32_t>(), l_rptr.as<int64_t>(),
                             l_ridx.as<int32_t>(), big_list.as<int32_t>(), big_cnt.as<int32_t>(), st));
        pool.reset();

        // ---- supernodes (Definition T3 per block of max_supernode rows)
        const bool want_sn = (plan.flags & GSOFA_NO_SUPERNODES) == 0;
        DBuf is_start, start_scan, xsup_all, supno_all;
        chk(hipEventRecord(ev[2], st));
        if (want_sn && nrows > 0) {
            std::vector<int64_t> bf;
            std::vector<int32_t> bl;
            for (int32_t j = 0; j < nj; ++j) {
                const int64_t M = plan.max_super > 0 ? plan.max_super : std::max<int64_t>(mats[j].n, 1);
                for (int64_t b = 0; b < mats[j].n; b += M) {
                    bf.push_back(row_base[j] + b);
                    bl.push_back((int32_t)std::min<int64_t>(M, mats[j].n - b));
                }
            }
            DBuf d_bf(8 * bf.size()), d_bl(4 * bl.size());
            chk(hipMemcpyAsync(d_bf.p, bf.data(), 8 * bf.size(), hipMemcpyHostToDevice, st));
            chk(hipMemcpyAsync(d_bl.p, bl.data(), 4 * bl.size(), hipMemcpyHostToDevice, st));
            is_start = DBuf(4 * (size_t)nrows);
            start_scan = DBuf(8 * (size_t)(nrows + 1));
            xsup_all = DBuf(4 * (size_t)(nrows + nj));
            supno_all = DBuf(4 * (size_t)nrows);
            chk(launch_supernodes(rs, (int64_t)bf.size(), d_bf.as<int64_t>(), d_bl.as<int32_t>(),
                                  u_ptr.as<int64_t>(), l_rptr.as<int64_t>(), l_ridx.as<int32_t>(),
                                  is_start.as<int32_t>(), st));
            chk(launch_scan_counts(is_start.as<int32_t>(), nullptr, nrows, start_scan.as<int64_t>(),
                                   scan_scr.as<int64_t>(), st));
            chk(launch_supernode_assemble(rs, nj, is_start.as<int32_t>(), start_scan.as<int64_t>(),
                                          xsup_all.as<int32_t>(), supno_all.as<int32_t>(), st));
            chk(launch_supernode_terminals(nj, d_jrb.as<int64_t>(), d_jn.as<int32_t>(), start_scan.as<int64_t>(),
                                           xsup_all.as<int32_t>(), st));
            chk(hipStreamSynchronize(st));
        }
        chk(hipEventRecord(ev[3], st));

        // ---- L column-wise
        const bool l_csr = (plan.flags & GSOFA_L_CSR) != 0;
        DBuf l_cptr, l_cidx;
        if (!l_csr) {
            l_cptr = DBuf(8 * (size_t)(nrows + 1));
            l_cidx = DBuf(4 * (size_t)std::max<int64_t>(nnz_l, 1));
            DBuf col_cnt(4 * (size_t)std::max<int64_t>(nrows, 1)), cursor(4 * (size_t)std::max<int64_t>(nrows, 1));
            DBuf tmp(4 * (size_t)std::max<int64_t>(nnz_l, 1));
            chk(launch_transpose_l(rs, l_rptr.as<int64_t>(), l_ridx.as<int32_t>(), col_cnt.as<int32_t>(),
                                   l_cptr.as<int64_t>(), l_cidx.as<int32_t>(), scan_scr.as<int64_t>(),
                                   cursor.as<int32_t>(), tmp.as<int32_t>(), big_list.as<int32_t>(),
                                   big_cnt.as<int32_t>(), st));
            chk(hipStreamSynchronize(st));
        }
        float t_trav = 0, t_emit = 0, t_sn = 0, t_l = 0;
        chk(hipEventSynchronize(ev[3]));
        chk(hipEventElapsedTime(&t_trav, ev[0], ev[4]));
        t_trav += t_trav_extra;
        chk(hipEventElapsedTime(&t_emit, ev[1], ev[2]));
        chk(hipEventElapsedTime(&t_sn, ev[2], ev[3]));
        (void)t_l;

        // ---- results
        std::vector<int64_t> h_sn_scan;  // start scan at job boundaries
        std::vector<int64_t> h_u_ptr, h_l_ptr;
        const int64_t* Lp = l_csr ? l_rptr.as<int64_t>() : l_cptr.as<int64_t>();
        const int32_t* Li = l_csr ? l_ridx.as<int32_t>() : l_cidx.as<int32_t>();
        const bool dev_out = (plan.flags & GSOFA_RESULT_ON_DEVICE) != 0;

        std::vector<int64_t> ujb(nj + 1), ljb(nj + 1), sjb(nj + 1);
        {
            // pointer values at job boundaries
            std::vector<int64_t> hu(nrows + 1), hl(nrows + 1), hs;
            chk(hipMemcpyAsync(hu.data(), u_ptr.p, 8 * (nrows + 1), hipMemcpyDeviceToHost, st));
            chk(hipMemcpyAsync(hl.data(), Lp, 8 * (nrows + 1), hipMemcpyDeviceToHost, st));
            if (want_sn && nrows > 0) {
                hs.resize(nrows + 1);
                chk(hipMemcpyAsync(hs.data(), start_scan.p, 8 * (nrows + 1), hipMemcpyDeviceToHost, st));
            }
            chk(hipStreamSynchronize(st));
            for (int32_t j = 0; j <= nj; ++j) {
                const int64_t b = j < nj ? row_base[j] : nrows;
                ujb[j] = hu[b];
                ljb[j] = hl[b];
                sjb[j] = hs.empty() ? 0 : hs[b];
            }
            if (!dev_out) {
                h_u_ptr.swap(hu);
                h_l_ptr.swap(hl);
            }
        }

        std::shared_ptr<std::vector<DBuf>> keep;
        DBuf u_ptr_loc, l_ptr_loc;
        if (dev_out) {
            if (nj > 1) {
                u_ptr_loc = DBuf(8 * (size_t)(nrows + nj));
                l_ptr_loc = DBuf(8 * (size_t)(nrows + nj));
                const unsigned gx = (unsigned)std::min<int64_t>((N + 256) / 256, 64);
                hipLaunchKernelGGL(k_rebase_ptr, dim3(gx, nj), dim3(256), 0, st, nj, d_jrb.as<int64_t>(),
                                   d_jn.as<int32_t>(), u_ptr.as<int64_t>(), u_ptr_loc.as<int64_t>());
                hipLaunchKernelGGL(k_rebase_ptr, dim3(gx, nj), dim3(256), 0, st, nj, d_jrb.as<int64_t>(),
                                   d_jn.as<int32_t>(), Lp, l_ptr_loc.as<int64_t>());
                chk(hipGetLastError());
                chk(hipStreamSynchronize(st));
            }
            keep = std::make_shared<std::vector<DBuf>>();
        }

        for (int32_t j = 0; j < nj; ++j) {
            gsofa_result* r = new_result();
            results[j] = r;
            const int32_t q = jt_of[j];
            r->n = mats[j].n;
            r->flags = plan.flags;
            r->stats.status = jstat[j];
            r->stats.edges_alg = hst[q].edges_alg;
            r->stats.edges_gpu = hst[q].edges_gpu;
            r->stats.iterations = (int32_t)std::min<unsigned long long>(hst[q].iterations, 0x7FFFFFFF);
            r->stats.windows = (int32_t)std::min<unsigned long long>(hst[q].windows, 0x7FFFFFFF);
            r->stats.concurrent_sources = ta.nslots;
            r->stats.peak_device_bytes =
                (uint64_t)(nslots * lay.bytes_per_slot + pool_cap * 4 + nrows * 48 + (nnz_u + 3 * nnz_l) * 4);
            r->stats.t_traverse_ms = t_trav;
            r->stats.t_emit_ms = t_emit;
            r->stats.t_supernode_ms = t_sn;
            if (jstat[j] != GSOFA_OK) continue;
            const int64_t n = mats[j].n, b = row_base[j];
            r->nnz_a = nnz[j];
            r->nnz_u = ujb[j + 1] - ujb[j];
            r->nnz_l = ljb[j + 1] - ljb[j];
            r->fills = r->nnz_u + r->nnz_l - (nnz[j] + n - (int64_t)hst[q].diag);
            r->nsuper = want_sn ? (int32_t)(sjb[j + 1] - sjb[j]) : 0;
            if (!dev_out) {
                r->u_ptr = host_array<int64_t>(r, n + 1);
                r->l_ptr = host_array<int64_t>(r, n + 1);
                for (int64_t i = 0; i <= n; ++i) {
                    r->u_ptr[i] = h_u_ptr[b + i] - ujb[j];
                    r->l_ptr[i] = h_l_ptr[b + i] - ljb[j];
                }
                r->u_idx = host_array<int32_t>(r, r->nnz_u);
                r->l_idx = host_array<int32_t>(r, r->nnz_l);
                if (r->nnz_u)
                    chk(hipMemcpyAsync(r->u_idx, u_idx.as<int32_t>() + ujb[j], 4 * r->nnz_u, hipMemcpyDeviceToHost, st));
                if (r->nnz_l)
                    chk(hipMemcpyAsync(r->l_idx, Li + ljb[j], 4 * r->nnz_l, hipMemcpyDeviceToHost, st));
                if (want_sn) {
                    r->xsup = host_array<int32_t>(r, r->nsuper + 1);
                    r->supno = host_array<int32_t>(r, n);
                    r->xsup[0] = 0;
                    if (n > 0) {
                        chk(hipMemcpyAsync(r->xsup, xsup_all.as<int32_t>() + sjb[j] + j, 4 * (r->nsuper + 1),
                                           hipMemcpyDeviceToHost, st));
                        chk(hipMemcpyAsync(r->supno, supno_all.as<int32_t>() + b, 4 * n, hipMemcpyDeviceToHost, st));
                    }
                }
            } else {
                auto* own = static_cast<ResultOwner*>(r->internal_);
                own->dev = keep;
                if (nj > 1) {
                    r->u_ptr = u_ptr_loc.as<int64_t>() + b + j;
                    r->l_ptr = l_ptr_loc.as<int64_t>() + b + j;
                } else {
                    r->u_ptr = u_ptr.as<int64_t>();
                    r->l_ptr = const_cast<int64_t*>(Lp);
                }
                r->u_idx = u_idx.as<int32_t>() + ujb[j];
                r->l_idx = const_cast<int32_t*>(Li) + ljb[j];
                if (want_sn && n > 0) {
                    r->xsup = xsup_all.as<int32_t>() + sjb[j] + j;
                    r->supno = supno_all.as<int32_t>() + b;
                }
            }
        }
        chk(hipStreamSynchronize(st));
        if (dev_out) {
            for (DBuf* b : {&u_idx, &u_ptr, &l_rptr, &l_ridx, &l_cptr, &l_cidx, &xsup_all, &supno_all,
                            &u_ptr_loc, &l_ptr_loc})
                b->synced = true;
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
    if (own) {
        for (void* p : own->host) std::free(p);
        delete own;
    }
    std::free(r);
}

Plan make_plan(const gsofa_opts* o) {
    Plan p{};
    p.window = 0;
    p.nslots = 0;
    p.max_super = 128;
    p.flags = 0;
    p.budget = 0;
    if (o) {
        p.flags = o->flags;
        p.budget = o->mem_budget_bytes;
        p.nslots = o->concurrent_sources;
        if (o->max_supernode > 0) p.max_super = o->max_supernode;
        else if (o->max_supernode < 0) p.max_super = 0;
        p.window = o->window;
    }
    return p;
}

int check_opts(const gsofa_opts* o) {
    if (!o) return GSOFA_OK;
    if (o->struct_size != 0 && o->struct_size < sizeof(gsofa_opts)) return GSOFA_EINVAL;
    if (o->mem_budget_bytes < 0 || o->window < 0 || o->concurrent_sources < 0) return GSOFA_EINVAL;
    if (o->dev_alloc || o->dev_free) return GSOFA_EINVAL;
    return GSOFA_OK;
}

std::mutex g_api_mu;  // one call at a time per process for the plain entry points

int run_engine(std::vector<MatIn> mats, const gsofa_opts* o, std::vector<gsofa_result*>& outs) {
    Engine eng;
    eng.mats = std::move(mats);
    eng.plan = make_plan(o);
    eng.on_device = o && (o->flags & GSOFA_INPUT_ON_DEVICE);
    eng.st = o ? static_cast<hipStream_t>(o->stream) : nullptr;
    int64_t N = 1;
    for (auto& m : eng.mats) N = std::max<int64_t>(N, m.n);
    if (eng.plan.window <= 0) eng.plan.window = auto_window(N);
    if (eng.plan.flags & GSOFA_LEVEL_ORDER) eng.plan.window = (int32_t)std::min<int64_t>(N, 0x7FFFFFFF);
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
    if (n < 0) return GSOFA_EINVAL;
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
        else if (mats[i].n < 0 || (mats[i].n > 0 && !mats[i].row_ptr)) pre[i] = GSOFA_EINVAL;
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
    return GSOFA_OK;
}

// ------------------------------------------------------------ the server
//
// Continuous batching: max_inflight worker threads, each with its own stream,
// take requests from the arrival queue in order whenever the head request's
// memory estimate fits what is left of the budget. Requests that arrive while
// others run are admitted as soon as a worker and memory are free, and their
// kernels overlap on the device with the running ones. A finished request
// returns its memory to the budget and wakes the waiting workers.

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
};

namespace {

int64_t estimate_request_bytes(int32_t n, int64_t nnz, int32_t nslots) {
    const SlotLayout lay = slot_layout(std::max<int64_t>(n, 1));
    return budget_for(n, nnz, nslots, lay);
}

int32_t serve_slots_for(const gsofa_server* s, int32_t n) {
    if (s->opts.concurrent_sources > 0) return std::min(s->opts.concurrent_sources, std::max(n, 1));
    const int32_t per = std::max(s->slots_total / std::max(1, s->max_inflight / 2), 64);
    return std::min(per, std::max(n, 1));
}

void serve_worker(gsofa_server* s, int sid) {
    (void)hipSetDevice(s->device);
    for (;;) {
        gsofa_server::Req r;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait(lk, [&] {
                if (s->queue.empty()) return s->closing;
                return s->mem_in_use + s->queue.front().est <= s->budget;
            });
            if (s->queue.empty()) return;  // closing and drained
            r = std::move(s->queue.front());
            s->queue.pop_front();
            s->inflight++;
            s->mem_in_use += r.est;
        }
        gsofa_opts o = s->opts;
        o.stream = s->streams[sid];
        o.flags &= ~(uint32_t)GSOFA_INPUT_ON_DEVICE;
        o.mem_budget_bytes = r.est;
        o.concurrent_sources = serve_slots_for(s, r.n);
        std::vector<gsofa_result*> outs;
        const int rc = run_engine({MatIn{r.n, r.rp.data(), r.ci.data()}}, &o, outs);
        gsofa_result* res = (rc == GSOFA_OK && !outs.empty()) ? outs[0] : nullptr;
        if (rc != GSOFA_OK)
            for (auto* x : outs) free_result(x);
        std::lock_guard<std::mutex> g(s->mu);
        s->done[r.ticket] = {rc, res};
        s->inflight--;
        s->mem_in_use -= r.est;
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
        s->slots_total = traverse_resident_slots(di.cus, 3);
        s->budget = s->opts.mem_budget_bytes > 0 ? s->opts.mem_budget_bytes : (int64_t)(di.free_b * 0.85);
        s->streams.assign(s->max_inflight, nullptr);
        for (auto& st : s->streams) chk(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    } catch (...) {
        for (auto st : s->streams)
            if (st) (void)hipStreamDestroy(st);
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
    r.est = estimate_request_bytes(m->n, nnz, serve_slots_for(s, m->n));
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
    delete s;
    return GSOFA_OK;
}
