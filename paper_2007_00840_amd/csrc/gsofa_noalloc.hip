// gsofa_symbolic_noalloc: the one-matrix pipeline of gsofa_symbolic (fill
// detection, row sort, supernodes, L transpose) on device-resident input,
// writing into caller-provided device arrays, with every working buffer carved
// from one fixed scratch array in device memory. Nothing here allocates device
// memory: no hipMalloc, no hipFree, no caller allocator.
//
// Scratch layout of a call (256-byte aligned pieces, in this order):
//   fixed part: job table, counters, per-row arrays (pool offsets and counts,
//     per-source statistics, L row pointers, supernode flags and scan, column
//     counts and cursors), scan scratch, supernode block table;
//   span A: the source slots during fill detection; afterwards (the slots are
//     dead then) the row-wise L and the transpose's staging array;
//   span B: the output pool, then whatever of it the pool did not use.
#include <chrono>
#include <map>
#include <mutex>

#include "gsofa.h"
#include "gsofa_internal.h"

namespace gsofa {
namespace {

constexpr size_t kScratchBytes = GSOFA_NOALLOC_SCRATCH_BYTES;

// The scratch array. In host code this name is only a stand-in for the symbol:
// kernels get the per-device address from hipGetSymbolAddress below.
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_mu;                      // one call at a time per process
std::map<int, uint8_t*> g_scratch;    // device -> that device's copy of the array

// Address of the current device's copy, looked up once per device (set-up;
// the caller holds g_mu and has the device current).
uint8_t* scratch_of(int dev) {
    auto it = g_scratch.find(dev);
    if (it != g_scratch.end()) return it->second;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
        (void)hipGetLastError();
        return nullptr;
    }
    g_scratch[dev] = static_cast<uint8_t*>(p);
    return static_cast<uint8_t*>(p);
}

// Bump carving of one span of the scratch array. A piece that does not fit
// returns nullptr but still advances the offset, so `off` ends as the bytes
// the span would have needed.
struct Span {
    uint8_t* base = nullptr;
    size_t cap = 0, off = 0;
    template <typename T>
    T* take(int64_t count) {
        const size_t o = (off + 255) & ~size_t(255);
        const size_t b = sizeof(T) * (size_t)std::max<int64_t>(count, 1);
        off = o + b;
        return off <= cap ? reinterpret_cast<T*>(base + o) : nullptr;
    }
    size_t need(int64_t bytes) const { return ((off + 255) & ~size_t(255)) + (size_t)bytes; }
};

// Job table entry, pointer bases of the one matrix, and the supernode block
// table (blocks of M rows; M <= 0: one block).
__global__ void k_na_setup(Job* job, Job j, int64_t* jrb, int32_t* jn, int64_t* bfirst, int32_t* blen,
                           int64_t nblocks, int64_t M, int32_t n) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t == 0) {
        *job = j;
        *jrb = 0;
        *jn = n;
    }
    for (int64_t b = t; b < nblocks; b += (int64_t)gridDim.x * blockDim.x) {
        const int64_t f = b * M;
        bfirst[b] = f;
        blen[b] = (int32_t)min<int64_t>(M, (int64_t)n - f);
    }
}

// Pointer arrays of an empty matrix: {0}; xsup of an empty matrix: {0}.
__global__ void k_na_empty(int64_t* u_ptr, int64_t* l_ptr, int32_t* xsup) {
    if (threadIdx.x == 0) {
        u_ptr[0] = 0;
        l_ptr[0] = 0;
        if (xsup) xsup[0] = 0;
    }
}

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

constexpr uint32_t kAllowed = GSOFA_NO_SUPERNODES | GSOFA_L_CSR | GSOFA_NO_LINE95 | GSOFA_LEVEL_ORDER |
                              GSOFA_MAP_WAVE32 | GSOFA_MAP_WAVE32_7 | GSOFA_INPUT_ON_DEVICE |
                              GSOFA_RESULT_ON_DEVICE | GSOFA_EAGER | GSOFA_NO_TUNE;

#define NA_CHK(x)                                  \
    do {                                           \
        if ((x) != hipSuccess) {                   \
            (void)hipGetLastError();               \
            return GSOFA_EDEVICE;                  \
        }                                          \
    } while (0)

int run_noalloc(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, const gsofa_opts* o,
                int64_t* u_ptr, int32_t* u_idx, int64_t u_cap, int64_t* l_ptr, int32_t* l_idx,
                int64_t l_cap, int32_t* xsup, int32_t* supno, gsofa_counts* c) {
    const double t0 = now_ms();
    const uint32_t flags = o ? o->flags : 0u;
    const hipStream_t st = o ? static_cast<hipStream_t>(o->stream) : nullptr;
    const bool want_sn = (flags & GSOFA_NO_SUPERNODES) == 0;
    const bool l_csr = (flags & GSOFA_L_CSR) != 0;
    int64_t M = 128;
    if (o && o->max_supernode > 0) M = o->max_supernode;
    else if (o && o->max_supernode < 0) M = 0;

    int dev = 0;
    NA_CHK(hipGetDevice(&dev));
    uint8_t* base = scratch_of(dev);
    if (!base) return GSOFA_EDEVICE;

    if (n == 0) {
        hipLaunchKernelGGL(k_na_empty, dim3(1), dim3(64), 0, st, u_ptr, l_ptr, want_sn ? xsup : nullptr);
        NA_CHK(hipGetLastError());
        NA_CHK(hipStreamSynchronize(st));
        c->stats.t_total_ms = now_ms() - t0;
        return GSOFA_OK;
    }

    // ---- fixed part of the scratch
    Span sp{base, kScratchBytes, 0};
    const int64_t nblocks = want_sn ? (M > 0 ? ((int64_t)n + M - 1) / M : 1) : 0;
    const int64_t Mb = M > 0 ? M : (int64_t)n;
    Job* d_job = sp.take<Job>(1);
    int64_t* d_jrb = sp.take<int64_t>(1);
    int32_t* d_jn = sp.take<int32_t>(1);
    int32_t* d_bad = sp.take<int32_t>(16);
    unsigned long long* d_cnt = sp.take<unsigned long long>(8);  // [0] work items, [1] pool tail
    JobStats* d_js = sp.take<JobStats>(1);
    int64_t* row_off = sp.take<int64_t>(n);
    int32_t* row_cnt = sp.take<int32_t>(n);
    int32_t* row_lcnt = sp.take<int32_t>(n);
    RowStat* row_stats = sp.take<RowStat>(n);
    int64_t* scan_scr = sp.take<int64_t>(scan_scratch_elems((int64_t)n + 1) + 8);
    int32_t* big_list = sp.take<int32_t>(n);
    int32_t* big_cnt = sp.take<int32_t>(16);
    int64_t* l_rptr = l_csr ? l_ptr : sp.take<int64_t>((int64_t)n + 1);
    int32_t* is_start = want_sn ? sp.take<int32_t>(n) : nullptr;
    int64_t* start_scan = want_sn ? sp.take<int64_t>((int64_t)n + 1) : nullptr;
    int64_t* bfirst = want_sn ? sp.take<int64_t>(nblocks) : nullptr;
    int32_t* blen = want_sn ? sp.take<int32_t>(nblocks) : nullptr;
    int32_t* col_cnt = l_csr ? nullptr : sp.take<int32_t>(n);
    int32_t* cursor = l_csr ? nullptr : sp.take<int32_t>(n);
    const bool fixed_ok = d_job && d_jrb && d_jn && d_bad && d_cnt && d_js && row_off && row_cnt && row_lcnt &&
                          row_stats && scan_scr && big_list && big_cnt && l_rptr &&
                          (!want_sn || (is_start && start_scan && bfirst && blen)) &&
                          (l_csr || (col_cnt && cursor));
    // ---- span A: source slots
    const int mapping = (flags & GSOFA_MAP_WAVE32_7) ? 4 : 0;
    const SlotLayout lay = slot_layout(n);
    int cus = 256;
    NA_CHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (!fixed_ok) {
        c->scratch_bytes = (int64_t)sp.need(lay.bytes_per_slot + 4 * ((int64_t)n + 1024));
        return GSOFA_ECAPACITY;
    }
    // the slots may take up to half of what is left; the output pool gets the rest
    const size_t rest = kScratchBytes - ((sp.off + 255) & ~size_t(255));
    int64_t nslots = (int64_t)(rest / 2) / lay.bytes_per_slot;
    nslots = std::min<int64_t>(nslots, traverse_resident_slots(cus, mapping));
    nslots = std::min<int64_t>(nslots, n);
    if (o && o->concurrent_sources > 0) nslots = std::min<int64_t>(nslots, o->concurrent_sources);
    if (nslots > 4) nslots = nslots / 4 * 4;  // whole blocks of four wavefronts
    if (nslots < 1) {
        c->scratch_bytes = (int64_t)sp.need(lay.bytes_per_slot + 4 * ((int64_t)n + 1024));
        return GSOFA_ECAPACITY;
    }
    Span spA{nullptr, 0, 0};
    {
        const size_t a0 = (sp.off + 255) & ~size_t(255);
        spA.base = base + a0;
        spA.cap = (size_t)nslots * (size_t)lay.bytes_per_slot;
        sp.off = a0 + spA.cap;
    }
    uint8_t* slots = spA.base;
    // ---- span B: output pool
    Span spB{nullptr, 0, 0};
    {
        const size_t b0 = (sp.off + 255) & ~size_t(255);
        spB.base = base + b0;
        spB.cap = b0 < kScratchBytes ? kScratchBytes - b0 : 0;
    }
    const int64_t pool_cap = (int64_t)(spB.cap / 4);
    if (pool_cap < (int64_t)n + 1024) {
        c->scratch_bytes = (int64_t)(sp.off + 4 * ((size_t)n + 1024));
        return GSOFA_ECAPACITY;
    }
    int32_t* pool = reinterpret_cast<int32_t*>(spB.base);

    int32_t window = o && o->window > 0 ? o->window : (n >= 65536 ? 16 : 64);
    if (flags & GSOFA_LEVEL_ORDER) window = n;

    // ---- set-up and input checks (everything that must start at zero is cleared)
    Job j{};
    j.row_ptr = row_ptr;
    j.col_idx = col_idx;
    j.n = n;
    hipLaunchKernelGGL(k_na_setup, dim3((unsigned)std::min<int64_t>((nblocks + 255) / 256 + 1, 1024)), dim3(256), 0,
                       st, d_job, j, d_jrb, d_jn, bfirst, blen, nblocks, Mb, n);
    NA_CHK(hipGetLastError());
    NA_CHK(launch_zero_i32(d_bad, 16, st));
    NA_CHK(launch_zero_i32(reinterpret_cast<int32_t*>(d_cnt), 16, st));
    NA_CHK(launch_zero_i32(reinterpret_cast<int32_t*>(d_js), (int64_t)(sizeof(JobStats) / 4), st));
    NA_CHK(launch_validate(d_job, 1, n, d_bad, st));
    int32_t h_bad = 0;
    int32_t h_last = 0;
    NA_CHK(hipMemcpyAsync(&h_bad, d_bad, 4, hipMemcpyDeviceToHost, st));
    NA_CHK(hipMemcpyAsync(&h_last, row_ptr + n, 4, hipMemcpyDeviceToHost, st));
    NA_CHK(hipStreamSynchronize(st));
    if (h_bad || h_last < 0) return GSOFA_EINVAL;
    c->nnz_a = h_last;

    // ---- fill detection
    const double tt0 = now_ms();
    NA_CHK(launch_init_slots(slots, (int32_t)nslots, lay, st));
    TraverseArgs ta{};
    ta.jobs = d_job;
    ta.njobs = 1;
    ta.nslots = (int32_t)nslots;
    ta.nitems = n;
    ta.item_rows = nullptr;
    ta.row_job = nullptr;
    ta.item_job = nullptr;
    ta.row_stats = row_stats;
    ta.item_counter = d_cnt;
    ta.slots = slots;
    ta.lay = lay;
    ta.row_off = row_off;
    ta.row_cnt = row_cnt;
    ta.row_lcnt = row_lcnt;
    ta.pool = pool;
    ta.pool_tail = d_cnt + 1;
    ta.pool_cap = pool_cap;
    ta.jstats = d_js;
    ta.window = window;
    ta.flags = flags;
    ta.mapping = mapping;
    NA_CHK(launch_traverse(ta, st));
    NA_CHK(launch_job_stats(d_job, 1, n, row_stats, d_js, st));
    JobStats hs{};
    unsigned long long h_tail = 0;
    NA_CHK(hipMemcpyAsync(&hs, d_js, sizeof(JobStats), hipMemcpyDeviceToHost, st));
    NA_CHK(hipMemcpyAsync(&h_tail, d_cnt + 1, 8, hipMemcpyDeviceToHost, st));
    NA_CHK(hipStreamSynchronize(st));
    const double tt1 = now_ms();
    if (hs.err & kErrDuplicate) return GSOFA_EINVAL;
    // the pool tail counts every reservation, also those that did not fit
    c->scratch_bytes = (int64_t)((spB.base - base) + 4 * h_tail);
    if (hs.err & kErrOverflow) return GSOFA_ECAPACITY;

    // ---- counts -> pointers of U (into the caller's u_ptr) and L
    NA_CHK(launch_scan_counts(row_cnt, row_lcnt, n, u_ptr, scan_scr, st));
    NA_CHK(launch_scan_counts(row_lcnt, nullptr, n, l_rptr, scan_scr, st));
    int64_t tot[2] = {0, 0};
    NA_CHK(hipMemcpyAsync(&tot[0], u_ptr + n, 8, hipMemcpyDeviceToHost, st));
    NA_CHK(hipMemcpyAsync(&tot[1], l_rptr + n, 8, hipMemcpyDeviceToHost, st));
    NA_CHK(hipStreamSynchronize(st));
    const int64_t nnz_u = tot[0], nnz_l = tot[1];
    c->nnz_u = nnz_u;
    c->nnz_l = nnz_l;
    c->fills = nnz_u + nnz_l - ((int64_t)h_last + n - (int64_t)hs.diag);
    if (nnz_u > u_cap || nnz_l > l_cap) return GSOFA_ECAPACITY;

    // ---- row-wise L and the transpose's staging: span A (dead slots), then
    // the part of span B the pool left unused
    spB.off = 4 * (size_t)h_tail;
    auto take_late = [&](int64_t count) -> int32_t* {
        if (int32_t* p = spA.take<int32_t>(count)) return p;
        return spB.take<int32_t>(count);
    };
    int32_t* l_ridx = l_csr ? l_idx : take_late(nnz_l);
    int32_t* ctmp = l_csr ? nullptr : take_late(nnz_l);
    if (!l_ridx || (!l_csr && !ctmp)) {
        c->scratch_bytes = (int64_t)((spB.base - base) + 4 * h_tail + 8 * nnz_l + 512);
        return GSOFA_ECAPACITY;
    }

    // ---- sorted rows, supernodes, L by columns
    const RowSpace rs{n, nullptr, nullptr};
    NA_CHK(launch_sort_rows(rs, row_off, row_cnt, row_lcnt, pool, u_ptr, u_idx, l_rptr, l_ridx, big_list,
                            big_cnt, st));
    const double ts0 = now_ms();
    if (want_sn) {
        NA_CHK(launch_supernodes(rs, nblocks, bfirst, blen, u_ptr, l_rptr, l_ridx, is_start, st));
        NA_CHK(launch_scan_counts(is_start, nullptr, n, start_scan, scan_scr, st));
        NA_CHK(launch_supernode_assemble(rs, 1, is_start, start_scan, xsup, supno, st));
        NA_CHK(launch_supernode_terminals(1, d_jrb, d_jn, start_scan, xsup, st));
    }
    if (!l_csr)
        NA_CHK(launch_transpose_l(rs, l_rptr, l_ridx, col_cnt, l_ptr, l_idx, scan_scr, cursor, ctmp, big_list,
                                  big_cnt, st));
    int64_t h_ns = 0;
    if (want_sn) NA_CHK(hipMemcpyAsync(&h_ns, start_scan + n, 8, hipMemcpyDeviceToHost, st));
    NA_CHK(hipStreamSynchronize(st));
    const double t1 = now_ms();

    c->nsuper = (int32_t)h_ns;
    c->stats.concurrent_sources = (int32_t)nslots;
    c->stats.iterations = hs.iterations;
    c->stats.windows = hs.windows;
    c->stats.edges_alg = hs.edges_alg;
    c->stats.edges_gpu = hs.edges_gpu;
    c->stats.peak_device_bytes = (uint64_t)c->scratch_bytes;
    c->stats.t_traverse_ms = tt1 - tt0;
    c->stats.t_emit_ms = ts0 - tt1;
    c->stats.t_supernode_ms = t1 - ts0;
    c->stats.t_total_ms = t1 - t0;
    c->stats.window = window;
    c->stats.mapping = mapping;
    c->stats.launches = 1;
    return GSOFA_OK;
}

}  // namespace
}  // namespace gsofa

using namespace gsofa;

extern "C" GSOFA_API int gsofa_symbolic_noalloc(int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
                                                const gsofa_opts* opts, int64_t* u_ptr, int32_t* u_idx,
                                                int64_t u_cap, int64_t* l_ptr, int32_t* l_idx, int64_t l_cap,
                                                int32_t* xsup, int32_t* supno, gsofa_counts* counts) {
    if (!counts || n < 0 || n > GSOFA_MAX_N || !u_ptr || !l_ptr || u_cap < 0 || l_cap < 0) return GSOFA_EINVAL;
    if (opts) {
        if (opts->struct_size != 0 && opts->struct_size < sizeof(gsofa_opts)) return GSOFA_EINVAL;
        if (opts->flags & ~kAllowed) return GSOFA_EINVAL;
        if (opts->dev_alloc || opts->dev_free || opts->mem_budget_bytes != 0) return GSOFA_EINVAL;
        if (opts->window < 0 || opts->concurrent_sources < 0 || opts->queue_cap < 0) return GSOFA_EINVAL;
    }
    const bool want_sn = !(opts && (opts->flags & GSOFA_NO_SUPERNODES));
    if (n > 0 && (!row_ptr || !col_idx || (want_sn && (!xsup || !supno)))) return GSOFA_EINVAL;
    if (n == 0 && want_sn && !xsup) return GSOFA_EINVAL;
    gsofa_counts c{};
    int rc;
    {
        std::lock_guard<std::mutex> g(g_mu);
        rc = run_noalloc(n, row_ptr, col_idx, opts, u_ptr, u_idx, u_cap, l_ptr, l_idx, l_cap, xsup, supno, &c);
    }
    c.stats.status = rc;
    // the totals found so far help a caller size its buffers on GSOFA_ECAPACITY
    if (rc == GSOFA_OK || rc == GSOFA_ECAPACITY) *counts = c;
    return rc;
}
