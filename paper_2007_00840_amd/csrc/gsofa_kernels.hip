// gfx950 kernels of the symbolic LU factorisation.
//
// Fill detection (Section 4 of the paper): for one source row s, every vertex
// v < s reached from s carries a label, the smallest achievable maximum
// intermediate vertex id over the paths s -> v found so far (the paper's
// maxId). A frontier f passes max(label(f), f) to each neighbour w < s,
// which keeps the atomic minimum; v joins L(s,:) when its label drops below v
// (fill-path theorem, Background); any w > s adjacent to s or to a reached
// vertex joins U(s,:). A vertex whose label improves while it is not yet in
// the structure is expanded again (the paper's revisits).
//
// Schedule (our design; the paper expands breadth-first): a vertex already in
// the structure always passes its own id on, so it is keyed by its id and
// waits in a per-source pending bitmap; a vertex outside the structure is
// keyed by its label. Keys never decrease along an edge, so the traversal runs
// in windows of increasing keys: take the pending vertices with ids in
// [lo, lo + window), relax breadth-first inside the window until no key in it
// changes, then move on. A vertex finished in an earlier window can never
// improve again. With window = n this is the paper's breadth-first order.
//
// One wavefront owns one source slot at a time and pulls sources from a
// global counter (largest ids first: their work grows with the id, Design
// Challenges, challenge 2). Frontier compaction uses wavefront ballots and
// lane prefix counts; per-slot state lives in HBM:
//   lab   : label per vertex, value-range encoded per source so nothing is
//           reset between sources (Section 4, maxId initialisation paragraph);
//           the byte-state kernel keeps one state byte per vertex there
//   P     : pending bitmap of structure vertices waiting for their window
//   qa/qb : current / next worklist (bit 31 of an entry: first visit of the
//           vertex by this source), qs: per-level dedup stamps
//   touch : reached vertices outside the structure (byte-state kernel: reset
//           list)
//   rowb  : the source row's structure, copied to the output pool at the end
#include <atomic>
#include "gsofa_internal.h"
#include "gsofa.h"

namespace gsofa {

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

__device__ __forceinline__ uint32_t lanes_below(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// a value the compiler cannot prove wave-uniform (from a cross-lane operation)
// that is: kept in a scalar register, loops over it stay scalar
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int wave_incl_scan(int v) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int t = __shfl_up(v, (unsigned)d, 64);
        if (lane_id() >= d) v += t;
    }
    return v;
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int d = 32; d; d >>= 1) v = max(v, __shfl_xor(v, d, 64));
    return v;
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int d = 32; d; d >>= 1) v = min(v, __shfl_xor(v, d, 64));
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int d = 32; d; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Slot state is private to the one wavefront (workgroup) that owns the slot
// for the whole launch, so workgroup scope is enough for its loads, atomics
// and fences: they stay in this XCD's L2 instead of going to the memory side.
// Only the work counter, the output pool and the statistics are shared
// across workgroups and use device-scope atomics.
template <typename T>
__device__ __forceinline__ auto ld_coherent(T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T, typename U>
__device__ __forceinline__ auto wg_min(T* p, U v) {
    return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T, typename U>
__device__ __forceinline__ auto wg_or(T* p, U v) {
    return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T, typename U>
__device__ __forceinline__ auto wg_and(T* p, U v) {
    return __hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T, typename U>
__device__ __forceinline__ auto wg_xchg(T* p, U v) {
    return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The host may ask a running launch to give its wave slots up (the request
// server does so when a newly admitted request finds the device full): the flag
// lives in fine-grained host memory and is read with system scope before each
// work item is taken. A launch that sees it takes no further item; the items it
// has taken are finished and the host relaunches from the work counter.
__device__ __forceinline__ bool yield_requested(const TraverseArgs& a) {
    return a.yield != nullptr && __hip_atomic_load(a.yield, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0u;
}

// Order this wavefront's earlier global/LDS accesses before its later ones.
__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void slot_fence() { wave_fence(); }

// Append val for every lane with pred set; count is wave-uniform.
__device__ __forceinline__ void wave_append(bool pred, int32_t val, int32_t* buf, int32_t& count) {
    unsigned long long m = __ballot(pred);
    if (pred) buf[count + (int32_t)lanes_below(m)] = val;
    count += __popcll(m);
}

__global__ void k_zero_i32(int32_t* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

SlotLayout slot_layout(int64_t N) {
    SlotLayout L{};
    if (N < 1) N = 1;
    L.N = N;
    L.nw64 = (N + 63) / 64;
    int64_t o = 0;
    auto take = [&](int64_t bytes) {
        int64_t r = o;
        o += (bytes + 255) & ~int64_t(255);
        return r;
    };
    L.L = N;
    L.qcap = N + 2048;
    L.qcap_d = L.qcap;
    L.rcap_d = N;
    L.off_lab = take(4 * N);
    L.off_p = take(8 * L.nw64);
    L.off_qs = take(4 * N);
    L.off_meta = take(64);
    L.off_ub = 0;
    L.off_qa = take(4 * L.qcap);
    L.off_qb = take(4 * L.qcap);
    L.off_row = take(4 * N);
    L.off_touch = take(4 * N);
    L.bytes_per_slot = o;
    return L;
}

SlotLayout slot_layout_budget(int64_t N, int64_t Lb, int64_t qcap_d) {
    SlotLayout L{};
    if (N < 1) N = 1;
    if (Lb < 1) Lb = 1;
    if (Lb > N) Lb = N;
    L.N = N;
    L.L = Lb;
    L.nw64 = (Lb + 63) / 64;
    int64_t o = 0;
    auto take = [&](int64_t bytes) {
        int64_t r = o;
        o += (bytes + 255) & ~int64_t(255);
        return r;
    };
    // a worklist never holds more than the ids below L plus the level filter's
    // slack; the row buffer at most N entries
    L.qcap = Lb + 2048;
    L.qcap_d = std::max<int64_t>(std::min<int64_t>(qcap_d, L.qcap), 64);
    L.rcap_d = std::max<int64_t>(std::min<int64_t>(qcap_d, N), 64);
    L.off_lab = take(4 * Lb);
    L.off_p = take(8 * L.nw64);
    L.off_qs = take(4 * Lb);
    L.off_meta = take(64);
    L.off_ub = take(4 * ((N + 31) / 32));  // cleared with P, qs and meta (before off_qa)
    L.off_qa = take(4 * L.qcap_d);
    L.off_qb = take(4 * L.qcap_d);
    L.off_row = take(4 * L.rcap_d);
    L.off_touch = 0;
    L.bytes_per_slot = o;
    L.h_q = L.qcap - L.qcap_d;
    L.h_stride = 2 * L.h_q + (N - L.rcap_d);
    return L;
}

// ------------------------------------------------------------ slot init

// lab = all ones, P = qs = meta = 0 (everything before off_qa).
__global__ void k_init_slots(uint8_t* slots, int32_t nslots, SlotLayout lay) {
    const int64_t words_lab = lay.L;
    const int64_t words_rest = (lay.off_qa - lay.off_p) / 4;
    for (int64_t sl = blockIdx.y; sl < nslots; sl += gridDim.y) {
        uint32_t* base = (uint32_t*)(slots + sl * lay.bytes_per_slot);
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words_lab;
             i += (int64_t)gridDim.x * blockDim.x)
            base[i] = kInf;
        uint32_t* rest = (uint32_t*)(slots + sl * lay.bytes_per_slot + lay.off_p);
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words_rest;
             i += (int64_t)gridDim.x * blockDim.x)
            rest[i] = 0u;
    }
}

hipError_t launch_init_slots(uint8_t* slots, int32_t nslots, SlotLayout lay, hipStream_t st) {
    if (nslots <= 0) return hipSuccess;
    int64_t words = lay.L + (lay.off_qa - lay.off_p) / 4;
    int gx = (int)std::min<int64_t>((words + 255) / 256, 64);
    int gy = std::min(nslots, 4096);
    hipLaunchKernelGGL(k_init_slots, dim3(gx, gy), dim3(256), 0, st, slots, nslots, lay);
    return hipGetLastError();
}

// ------------------------------------------------------------ validation

// Input checks for device-resident CSR: row_ptr[0] == 0, non-decreasing,
// columns in [0, n). Rows whose bounds are broken are not read.
__global__ void k_validate(const Job* jobs, int32_t njobs, int64_t max_n, int32_t* bad) {
    const int32_t j = blockIdx.y;
    if (j >= njobs) return;
    const Job J = jobs[j];
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < J.n;
         r += (int64_t)gridDim.x * blockDim.x) {
        int32_t a = J.row_ptr[r], b = J.row_ptr[r + 1];
        bool ok = (a >= 0) && (b >= a) && (r != 0 || a == 0);
        if (ok) {
            for (int32_t e = a; e < b; ++e) {
                int32_t c = J.col_idx[e];
                if (c < 0 || c >= J.n) { ok = false; break; }
            }
        }
        if (!ok) atomicOr(&bad[j], 1);
    }
    (void)max_n;
}

hipError_t launch_validate(const Job* jobs_dev, int32_t njobs, int64_t max_n, int32_t* bad_dev,
                           hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    int gx = (int)std::min<int64_t>((max_n + 255) / 256, 1024);
    if (gx < 1) gx = 1;
    hipLaunchKernelGGL(k_validate, dim3(gx, njobs), dim3(256), 0, st, jobs_dev, njobs, max_n, bad_dev);
    return hipGetLastError();
}

__global__ void k_row_job(const Job* jobs, int32_t njobs, int32_t* row_job, bool by_item) {
    const int32_t j = blockIdx.y;
    if (j >= njobs) return;
    const Job J = jobs[j];
    const int64_t base = by_item ? J.item_base : J.row_base;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < J.n;
         r += (int64_t)gridDim.x * blockDim.x)
        row_job[base + r] = j;
}

hipError_t launch_row_job(const Job* jobs_dev, int32_t njobs, int64_t max_n, int32_t* row_job,
                          hipStream_t st, bool by_item) {
    if (njobs <= 0) return hipSuccess;
    int gx = (int)std::min<int64_t>((max_n + 255) / 256, 1024);
    if (gx < 1) gx = 1;
    hipLaunchKernelGGL(k_row_job, dim3(gx, njobs), dim3(256), 0, st, jobs_dev, njobs, row_job, by_item);
    return hipGetLastError();
}

// -------------------------------------------------------------- traversal

struct WaveTile {
    int32_t scan[64];    // inclusive prefix of frontier degrees
    int32_t start[64];   // first edge of each frontier
    uint32_t outv[64];   // value each frontier passes on: max(label, id)
};
// Edge dealing of the one-wavefront kernel: the chunk's rows with entries, in
// order, as (first edge - degree prefix, lane holding the row), and a bitmap of
// the edges that start a row within a span of kHeadEdges edges.
constexpr int32_t kHeadEdges = 64 * 32;
struct DealTile {
    int2 pk[64];
    unsigned long long heads[kHeadEdges / 64];
};

constexpr int kTravWaves = 4;
constexpr int kIlp = 4;          // edges in flight per lane
constexpr int kHashBits = 8;     // per-wavefront push filter: 256 (level, vertex) entries
// per-wavefront table that keeps one atomic minimum per target vertex and round
// (128 entries; a key holds the vertex id's bits above these 7, a 31-bit value and
// an 8-bit edge slot), used by rounds with at least kDedupMin candidate edges
constexpr int kDedupBits = 7;
constexpr int kDedupMin = 32;

#define GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GLOBAL T* gbl(T* p) {
    return (GLOBAL T*)p;
}

// raw buffer view of a slot's label array (range-checked loads)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t label_rsrc(uint32_t* lab, int64_t n) {
    return __builtin_amdgcn_make_buffer_rsrc(lab, (short)0, (int)(n * 4), 0x00020000);
}

// The label word of a vertex carries all per-source state:
//   stale (older source)          -> not reached yet
//   base + x, x < v               -> v is in the structure (x = 0: original entry)
//   base + x, x > v               -> reached through intermediates up to x, not (yet) a fill
// For w > s the first atomic minimum that finds a stale word marks the U entry.
// The label is read first and the atomic minimum is issued only where it can
// lower it (an atomic on every edge instead measured 4x slower).
// Compiled for W wavefronts per SIMD (register budget 512 / W VGPRs; what spills
// is per-source set-up, outside the level loop; the LDS tables take 15 KB per
// workgroup of four). W = 8 (mapping 0) keeps the most loads in flight: on the
// 64^3 27-point stencil seven and six were 4 % and 7 % slower. W = 7 (mapping 4)
// spills less per source, which pays where sources are many and short: ~4 % on
// the 1000^2 9-point stencil. The tuner picks between them.
//
// B selects the memory-budget variant (mapping 5, GSOFA_BUDGET_MODE; Space
// Optimization section): labels, level stamps and the pending bitmap cover the
// ids below lay.L only (bubble removal: the host runs sources in bands of ids
// below L), U membership is a bitmap over all ids (a vertex above the source is
// never labelled), and the worklists and the row buffer keep lay.qcap_d /
// lay.rcap_d entries in device memory and the rest in pinned host memory
// (external frontier management). With B false every budget branch folds away.
template <int W, bool B>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W, 8))) void k_traverse(TraverseArgs a) {
    __shared__ DealTile tiles[kTravWaves];
    __shared__ unsigned long long pushed[kTravWaves][1 << kHashBits];
    __shared__ unsigned long long rdedup[kTravWaves][1 << kDedupBits];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ln = lane_id();
    const int32_t slot = blockIdx.x * kTravWaves + wv;
    if (slot >= a.nslots) return;
    DealTile& T = tiles[wv];
    unsigned long long* H = pushed[wv];
    unsigned long long* RT = rdedup[wv];

    uint8_t* sb = a.slots + (int64_t)slot * a.lay.bytes_per_slot;
    GLOBAL uint32_t* lab = gbl((uint32_t*)(sb + a.lay.off_lab));
    GLOBAL unsigned long long* P = gbl((unsigned long long*)(sb + a.lay.off_p));
    GLOBAL int32_t* qa = gbl((int32_t*)(sb + a.lay.off_qa));
    GLOBAL int32_t* qb = gbl((int32_t*)(sb + a.lay.off_qb));
    GLOBAL int32_t* rowb = gbl((int32_t*)(sb + a.lay.off_row));
    GLOBAL uint32_t* qs = gbl((uint32_t*)(sb + a.lay.off_qs));
    GLOBAL uint32_t* meta = gbl((uint32_t*)(sb + a.lay.off_meta));
    const __amdgpu_buffer_rsrc_t lab_r = label_rsrc((uint32_t*)(sb + a.lay.off_lab), a.lay.L);
    // budget mode: U membership bits, host parts of the worklists and row buffer
    GLOBAL uint32_t* ub = gbl((uint32_t*)(sb + a.lay.off_ub));
    const int32_t qcd = (int32_t)a.lay.qcap_d;
    const int32_t rcd = (int32_t)a.lay.rcap_d;
    GLOBAL int32_t* hb = B ? gbl(a.host_spill + (int64_t)slot * a.lay.h_stride) : nullptr;
    GLOBAL int32_t* qa_h = hb;
    GLOBAL int32_t* qb_h = B ? hb + a.lay.h_q : nullptr;
    GLOBAL int32_t* rowb_h = B ? hb + 2 * a.lay.h_q : nullptr;
    auto qput = [&](GLOBAL int32_t* d, GLOBAL int32_t* h, int32_t i, int32_t v) {
        if (!B || i < qcd) d[i] = v;
        else h[i - qcd] = v;
    };
    auto qget = [&](GLOBAL int32_t* d, GLOBAL int32_t* h, int32_t i) -> int32_t {
        return (!B || i < qcd) ? ld_coherent(&d[i]) : ld_coherent(&h[i - qcd]);
    };
    auto rput = [&](int32_t i, int32_t v) {
        if (!B || i < rcd) rowb[i] = v;
        else rowb_h[i - rcd] = v;
    };
    auto rget = [&](int32_t i) -> int32_t {
        return (!B || i < rcd) ? ld_coherent(&rowb[i]) : ld_coherent(&rowb_h[i - rcd]);
    };

    const uint32_t R = (uint32_t)a.lay.L;
    const uint32_t emax = 0xFFFFFFFFu / R;
    uint32_t epoch = meta[0];
    uint32_t lvl = meta[1];
    const bool line95 = (a.flags & GSOFA_NO_LINE95) == 0;
    const int32_t D = a.window > 0 ? a.window : 1;
    for (int i = ln; i < (1 << kHashBits); i += 64) H[i] = ~0ull;

    for (;;) {
        unsigned long long k = 0;
        if (ln == 0) k = yield_requested(a) ? ~0ull : atomicAdd(a.item_counter, 1ull);
        k = __shfl(k, 0, 64);
        if (k >= (unsigned long long)a.nitems) break;

        int32_t j, s;
        if (a.item_rows) {
            const int64_t gr = a.item_rows[k];
            j = a.row_job ? a.row_job[gr] : 0;
            s = (int32_t)(gr - a.jobs[j].row_base);
        } else {
            if (a.item_job) {
                j = a.item_job[k];
            } else {
                int32_t lo = 0, hi = a.njobs - 1;
                while (lo < hi) {
                    int32_t mid = (lo + hi + 1) >> 1;
                    if (a.jobs[mid].item_base <= (int64_t)k) lo = mid;
                    else hi = mid - 1;
                }
                j = lo;
            }
            s = a.jobs[j].n - 1 - (int32_t)((int64_t)k - a.jobs[j].item_base);
        }
        j = __builtin_amdgcn_readfirstlane(j);
        s = __builtin_amdgcn_readfirstlane(s);
        const GLOBAL int32_t* rp = gbl(a.jobs[j].row_ptr);
        const GLOBAL int32_t* ci = gbl(a.jobs[j].col_idx);
        const int64_t grow = a.jobs[j].row_base + s;

        // fresh label range for this source (reset once the 32-bit range is used
        // up, or before every source for the ablation of that scheme)
        if (epoch >= emax || (a.flags & GSOFA_RESET_LABELS)) {
            for (int64_t i = ln; i < (int64_t)R; i += 64) lab[i] = kInf;
            epoch = 0;
            slot_fence();
        }
        if (lvl >= 0xF0000000u) {
            for (int i = ln; i < (1 << kHashBits); i += 64) H[i] = ~0ull;
            for (int64_t i = ln; i < (int64_t)R; i += 64) qs[i] = 0u;
            lvl = 0;
            slot_fence();
        }
        ++epoch;
        const uint32_t base = 0xFFFFFFFFu - epoch * R;
        // This source's labels lie in [base, base + R); every older word lies at
        // or above base + R (earlier ranges sit higher, the initial word is the
        // top value). So the relaxation compares encoded words directly:
        // "not reached" is w >= baseR, "value x lowers it" is base + x < w, and
        // "already in the structure" is w < base + v.
        const uint32_t baseR = base + R;

        // a source's first-visit degrees sum to at most nnz < 2^31: 32 bits per lane
        uint32_t e_alg = 0;
        unsigned long long e_gpu = 0;
        int32_t rcount = 0, lcount = 0;
        uint32_t n_iter = 0, n_win = 0;
        unsigned long long n_spill = 0;

        // ---- seed: the source row's own entries (original entries of row s)
        const int32_t rs = rp[s], re = rp[s + 1];
        int32_t ndiag = 0;
        bool dup = false;
        int32_t pmin = 0x7FFFFFFF;
        for (int32_t e0 = rs; e0 < re; e0 += 64) {
            const int32_t e = e0 + ln;
            const bool act = e < re;
            const int32_t w = act ? ci[e] : -1;
            ndiag += __popcll(__ballot(act && w == s));
            bool fresh = false;
            if (act && w != s) {
                if (B && w > s) {
                    const uint32_t bit = 1u << (w & 31);
                    fresh = (wg_or(&ub[w >> 5], bit) & bit) == 0u;
                } else {
                    const uint32_t old = wg_min(&lab[w], base);  // label 0: no intermediate vertex
                    fresh = old != base;  // base is label 0: seeded already (a repeated column)
                }
                dup |= !fresh;
            }
            const bool below = fresh && w < s;
            {
                unsigned long long m = __ballot(fresh);
                if (fresh) rput(rcount + (int32_t)lanes_below(m), w);
                rcount += __popcll(m);
            }
            lcount += __popcll(__ballot(below));
            if (below) {
                wg_or(&P[w >> 6], 1ull << (w & 63));
                e_alg += (uint32_t)(rp[w + 1] - rp[w]);
                pmin = min(pmin, w);
            }
        }
        if (ln == 0) e_alg += (uint32_t)(re - rs);
        e_gpu += (unsigned long long)(re - rs);
        if (__ballot(dup) != 0ull || ndiag > 1) {
            if (ln == 0) atomicOr(&a.jstats[j].err, kErrDuplicate);
        }
        pmin = uni(wave_min(pmin));
        slot_fence();

        // ---- windows of increasing keys
        const int32_t nwp = (s + 63) >> 6;  // pending words covering [0, s)
        int32_t pos = pmin;
        while (pos < s) {
            // lowest pending vertex >= pos
            int32_t found = -1;
            for (int32_t w0 = pos >> 6; w0 < nwp; w0 += 64) {
                const int32_t wi = w0 + ln;
                const unsigned long long word = (wi < nwp) ? ld_coherent(&P[wi]) : 0ull;
                const unsigned long long nz = __ballot(word != 0ull);
                if (nz) {
                    const int jl = __builtin_ctzll(nz);
                    const unsigned long long wd = __shfl(word, jl, 64);
                    found = uni((w0 + jl) * 64 + __builtin_ctzll(wd));
                    break;
                }
            }
            if (found < 0) break;
            const int32_t lo = found;
            const int32_t hi = (int32_t)min((int64_t)lo + D, (int64_t)s);
            ++n_win;

            // extract the pending vertices of [lo, hi) into the worklist
            GLOBAL int32_t* cur = qa;
            GLOBAL int32_t* nxt = qb;
            GLOBAL int32_t* cur_h = qa_h;
            GLOBAL int32_t* nxt_h = qb_h;
            int32_t qn = 0;
            const int32_t wlast = (hi - 1) >> 6;
            for (int32_t w0 = lo >> 6; w0 <= wlast; w0 += 64) {
                const int32_t wi = w0 + ln;
                unsigned long long word = 0ull;
                if (wi <= wlast) {
                    word = ld_coherent(&P[wi]);
                    const int64_t b0 = (int64_t)wi * 64;
                    unsigned long long m = ~0ull;
                    if (b0 < lo) m &= ~0ull << (lo - b0);
                    if (b0 + 64 > hi) m &= (hi - b0 >= 64) ? ~0ull : ((1ull << (hi - b0)) - 1ull);
                    word &= m;
                    if (word) wg_and(&P[wi], ~word);
                }
                const int c = __popcll(word);
                const int incl = wave_incl_scan(c);
                int32_t o = qn + incl - c;
                while (word) {
                    const int b = __builtin_ctzll(word);
                    word &= word - 1ull;
                    qput(cur, cur_h, o++, wi * 64 + b);
                }
                qn += uni(__shfl(incl, 63, 64));
            }
            if (B && qn > qcd) n_spill += (unsigned long long)(qn - qcd);
            wave_fence();

            // breadth-first label correction inside the window
            while (qn > 0) {
                ++lvl;
                ++n_iter;
                int32_t nq = 0;
                // the LDS filter is exact until two vertices of this level collide in
                // it; from then on this level also checks the per-vertex stamps, which
                // bounds the next queue by N + 2 * (1 << kHashBits)
                bool exact = false;
                for (int32_t c0 = 0; c0 < qn; c0 += 64) {
                    const int32_t i = c0 + ln;
                    const bool act = i < qn;
                    // bit 31 of a queue entry: first visit of the vertex by this source
                    const int32_t fr = qget(cur, cur_h, act ? i : 0);
                    const int32_t f = fr & 0x7FFFFFFF;
                    const int32_t fs = rp[f];
                    const int32_t deg = act ? rp[f + 1] - fs : 0;
                    if (fr < 0) e_alg += (uint32_t)deg;
                    // encoded value this row passes on: max(label, f), or the top
                    // word (lowers nothing) if the row holds no label
                    const uint32_t lf = ld_coherent(&lab[f]);
                    const uint32_t ov = lf >= baseR ? kInf : max(lf, base + (uint32_t)f);
                    const int32_t incl = wave_incl_scan(deg);
                    const int32_t total = uni(__shfl(incl, 63, 64));
                    e_gpu += (unsigned long long)total;
                    // one round: kIlp independent edges per lane; every load of the
                    // round is issued before any of its results is used
                    // own[k]: lane holding the row of edge k. A lane's row passes on
                    // ov, or with refresh set the value taken from fraw (its label
                    // re-read); both are taken once the round's loads are in flight.
                    auto round = [&](int32_t (&widx)[kIlp], int32_t (&own)[kIlp], uint32_t fraw, bool refresh,
                                     bool (&act_e)[kIlp]) {
                        int32_t w[kIlp];
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk) w[kk] = ci[widx[kk]];
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk) act_e[kk] = act_e[kk] && w[kk] != s;
                        // slot and key of edge kk in the per-round dedup table (below),
                        // recomputed where used: cheaper than keeping them in registers
                        // across the LDS round trips
                        auto slot = [&](int kk) -> uint32_t {
                            uint32_t wv = (uint32_t)w[kk];
                            asm volatile("" : "+v"(wv));
                            return (wv ^ (wv >> kDedupBits) ^ (wv >> (2 * kDedupBits))) & ((1u << kDedupBits) - 1u);
                        };
                        uint32_t outv[kIlp];
                        uint32_t lv[kIlp];
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk) {
                            if (B && w[kk] > s) {
                                lv[kk] = act_e[kk] ? ld_coherent(&ub[w[kk] >> 5]) : ~0u;
                            } else {
                                const uint32_t off = act_e[kk] ? (uint32_t)w[kk] * 4u : 0xFFFFFFF0u;
                                lv[kk] = __builtin_amdgcn_raw_buffer_load_b32(lab_r, off, 0, 0);
                            }
                        }
                        {
                            const uint32_t ovr = refresh ? (fraw >= baseR ? kInf : max(fraw, base + (uint32_t)f)) : ov;
#pragma unroll
                            for (int kk = 0; kk < kIlp; ++kk) outv[kk] = (uint32_t)__shfl((int)ovr, own[kk], 64);
                        }
                        auto keyof = [&](int kk) -> unsigned long long {
                            uint32_t wv = (uint32_t)w[kk];
                            asm volatile("" : "+v"(wv));
                            return ((unsigned long long)(wv >> kDedupBits) << 40) |
                                   ((unsigned long long)(wv > (uint32_t)s ? 0u : outv[kk]) << 8) |
                                   (unsigned long long)(kk * 64 + ln);
                        };
                        // which edges can change a label: U side unseen, or a smaller value
                        bool cand[kIlp];
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk) {
                            if (B && w[kk] > s) cand[kk] = act_e[kk] && (lv[kk] & (1u << (w[kk] & 31))) == 0u;
                            else if (w[kk] > s) cand[kk] = act_e[kk] && lv[kk] >= baseR;
                            else cand[kk] = act_e[kk] && outv[kk] < lv[kk] && !(line95 && lv[kk] < base + (uint32_t)w[kk]);
                        }
                        // Candidates of one round that share a target all saw the label
                        // as it was before the round; only the one with the smallest value
                        // (ties: the lowest edge slot) needs its atomic minimum: the others
                        // could not lower the label below it, and the one issued returns
                        // the label every decision below needs. Without this, about half
                        // the atomics of a 2D 9-point or 3D 27-point traversal changed
                        // nothing (neighbouring rows of a round share most neighbours).
                        // They meet in a small LDS table: slot from a fold of w, key =
                        // (w's high bits, value, edge slot), so equal keys mean the same
                        // edge and a slot holding another vertex leaves the candidate as
                        // it is. Rounds with few candidates skip it (the LDS round trips
                        // then cost more than the atomics they save).
                        const int32_t ncand = __popcll(__ballot(cand[0])) + __popcll(__ballot(cand[1])) +
                                              __popcll(__ballot(cand[2])) + __popcll(__ballot(cand[3]));
                        if (ncand >= kDedupMin) {
#pragma unroll
                            for (int kk = 0; kk < kIlp; ++kk)
                                if (cand[kk]) RT[slot(kk)] = ~0ull;
                            wave_fence();
#pragma unroll
                            for (int kk = 0; kk < kIlp; ++kk)
                                if (cand[kk])
                                    __hip_atomic_fetch_min(&RT[slot(kk)], keyof(kk), __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_WAVEFRONT);
                            wave_fence();
#pragma unroll
                            for (int kk = 0; kk < kIlp; ++kk) {
                                if (cand[kk]) {
                                    const unsigned long long r = RT[slot(kk)], kq = keyof(kk);
                                    cand[kk] = r == kq || (r >> 40) != (kq >> 40);
                                }
                            }
                        }
                        uint32_t old[kIlp];
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk) {
                            if (B && w[kk] > s)
                                // a set bit reads as "already in U", a clear one as "not reached"
                                old[kk] = cand[kk] ? ((wg_or(&ub[w[kk] >> 5], 1u << (w[kk] & 31)) >> (w[kk] & 31)) & 1u
                                                          ? base : kInf)
                                                   : base;
                            else
                                old[kk] = cand[kk] ? wg_min(&lab[w[kk]], w[kk] > s ? base : outv[kk]) : base;
                        }
                        bool emit[kIlp], isl[kIlp], push[kIlp], first[kIlp];
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk) {
                            const int32_t wk = w[kk];
                            const uint32_t ov = outv[kk];
                            const uint32_t ow = old[kk];
                            const uint32_t bw = base + (uint32_t)wk;
                            emit[kk] = isl[kk] = push[kk] = false;
                            first[kk] = cand[kk] && wk < s && ow >= baseR;
                            if (!cand[kk]) continue;
                            if (wk > s) {
                                emit[kk] = ow >= baseR;
                                continue;
                            }
                            if (ov < ow && ow >= bw) {
                                if (ov < bw) {
                                    // label fell below w: fill (s, w)
                                    emit[kk] = true;
                                    isl[kk] = true;
                                    if (wk < hi) push[kk] = true;
                                    else wg_or(&P[wk >> 6], 1ull << (wk & 63));
                                } else {
                                    push[kk] = true;
                                }
                            }
                        }
                        // drop repeated pushes of a vertex within one level
                        bool evict = false;
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk) {
                            if (push[kk]) {
                                const unsigned long long key = ((unsigned long long)lvl << 32) | (uint32_t)w[kk];
                                const uint32_t h = ((uint32_t)w[kk] * 2654435761u) >> (32 - kHashBits);
                                const unsigned long long prev = __hip_atomic_exchange(
                                    &H[h], key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                                push[kk] = prev != key;
                                evict |= push[kk] && (uint32_t)(prev >> 32) == lvl;
                            }
                        }
                        if (exact) {
#pragma unroll
                            for (int kk = 0; kk < kIlp; ++kk)
                                if (push[kk]) push[kk] = wg_xchg(&qs[w[kk]], lvl) != lvl;
                        }
                        exact = exact || __ballot(evict) != 0ull;
                        // a vertex reached for the first time contributes its degree
                        // once: a pushed one carries the first-visit flag to its
                        // expansion, where the degree is loaded anyway; the rest (in
                        // the structure beyond the window) load it here
                        bool any = false;
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk) {
                            if (first[kk] && !push[kk]) e_alg += (uint32_t)(rp[w[kk] + 1] - rp[w[kk]]);
                            any |= emit[kk] | push[kk];
                        }
                        if (__ballot(any) == 0ull) return;
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk) {
                            unsigned long long m = __ballot(emit[kk]);
                            if (emit[kk]) rput(rcount + (int32_t)lanes_below(m), w[kk]);
                            rcount += __popcll(m);
                            lcount += __popcll(__ballot(isl[kk]));
                            m = __ballot(push[kk]);
                            if (push[kk])
                                qput(nxt, nxt_h, nq + (int32_t)lanes_below(m),
                                     (int32_t)((uint32_t)w[kk] | (first[kk] ? 0x80000000u : 0u)));
                            nq += __popcll(m);
                        }
                    };
                    // The chunk's edges, concatenated, are dealt so that consecutive
                    // lanes take consecutive edges (edge r0 + 64 k + l goes to lane l in
                    // slot k of a round). One column-index load instruction then reads
                    // 256 contiguous bytes, and a row's neighbours (sorted ids) share
                    // label cache lines inside one instruction. The owner of an edge is
                    // found without a search: rows with entries are packed in LDS, a
                    // bitmap marks the edges that start a row, and the owner of lane l's
                    // edge in a block of 64 is the owner of the block's first edge (a
                    // ballot over the rows' first edges) plus the rows starting among
                    // the block's edges 1..l.
                    // From the second round on, each row re-reads its own label (one
                    // load per row, handed to its edges by a lane shuffle): a row that an
                    // earlier round of this chunk lowered passes on the lower value at
                    // once instead of a stale one that later levels have to correct
                    // (17 % fewer edges scanned on a 2D 9-point grid, 11 % on a 3D
                    // 27-point one).
                    const bool has = deg > 0;
                    const int32_t excl = incl - deg;
                    {
                        const unsigned long long hm = __ballot(has);
                        if (has) T.pk[lanes_below(hm)] = make_int2(fs - excl, ln);
                    }
                    const int32_t nr = (total + 64 * kIlp - 1) / (64 * kIlp);
                    for (int32_t rr = 0; rr < nr; ++rr) {
                        const int32_t r0 = rr * (64 * kIlp);
                        // only rows with edges in this round re-read their label:
                        // finished rows pass nothing on, later rows re-read theirs when
                        // their round comes. Issued first, used only once the round's
                        // loads are in flight; sc0 (aux 1) as for a coherent load, an
                        // out-of-range offset (no refresh) returns 0 without an access.
                        const bool refresh = rr > 0 && has && incl > r0 && excl < r0 + 64 * kIlp;
                        const uint32_t fraw = __builtin_amdgcn_raw_buffer_load_b32(
                            lab_r, refresh ? (uint32_t)f * 4u : 0xFFFFFFF0u, 0, 1);
                        const int32_t W0 = r0 & ~(kHeadEdges - 1);
                        if (r0 == W0) {
                            // row starts among edges [W0, W0 + kHeadEdges)
                            wave_fence();
                            if (ln < kHeadEdges / 64) T.heads[ln] = 0ull;
                            wave_fence();
                            if (has && excl >= W0 && excl < W0 + kHeadEdges)
                                __hip_atomic_fetch_or(&T.heads[(excl - W0) >> 6], 1ull << (excl & 63),
                                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                            wave_fence();
                        }
                        int32_t widx[kIlp], own[kIlp];
                        bool act_e[kIlp];
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk) {
                            const int32_t b = r0 + kk * 64;
                            const int32_t ei = b + ln;
                            act_e[kk] = ei < total;
                            const unsigned long long hd = T.heads[(b - W0) >> 6];
                            const int32_t o = __popcll(__ballot(has && excl <= b)) - 1 +
                                              __popcll(hd & ((2ull << ln) - 1ull) & ~1ull);
                            const int2 q = T.pk[o];
                            widx[kk] = act_e[kk] ? q.x + ei : 0;
                            own[kk] = q.y;
                        }
                        round(widx, own, fraw, refresh, act_e);
                    }
                    wave_fence();
                }
                GLOBAL int32_t* t = cur;
                cur = nxt;
                nxt = t;
                t = cur_h;
                cur_h = nxt_h;
                nxt_h = t;
                qn = nq;
                if (B && qn > qcd) n_spill += (unsigned long long)(qn - qcd);
                wave_fence();
            }
            pos = hi;
        }

        // ---- finish the row: diagonal, copy to the pool
        if (ln == 0) rput(rcount, s);
        rcount += 1;
        if (B && rcount > rcd) n_spill += (unsigned long long)(rcount - rcd);
        slot_fence();
        unsigned long long off = 0;
        if (ln == 0) off = atomicAdd(a.pool_tail, (unsigned long long)rcount);
        off = __shfl(off, 0, 64);
        const bool fits = (int64_t)(off + rcount) <= a.pool_cap;
        GLOBAL int32_t* pool = gbl(a.pool);
        if (fits || B)
            for (int32_t i = ln; i < rcount; i += 64) {
                const int32_t v = rget(i);
                if (fits) pool[off + i] = v;
                // every set bit of a U word belongs to this source: clear the word
                if (B && v > s) ub[v >> 5] = 0u;
            }
        if (B && n_spill && ln == 0) atomicAdd(&a.jstats[j].spilled, n_spill);
        if (ln == 0) {
            a.row_off[grow] = fits ? (int64_t)off : -1;
            a.row_cnt[grow] = rcount;
            a.row_lcnt[grow] = lcount;
            if (!fits) atomicOr(&a.jstats[j].err, kErrOverflow);
        }

        const unsigned long long e_alg_s = wave_sum_u64((unsigned long long)e_alg);
        if (ln == 0 && a.row_stats)
            a.row_stats[grow] = RowStat{e_alg_s, e_gpu, n_iter, (n_win & 0x7FFFFFFFu) | (ndiag > 0 ? 0x80000000u : 0u)};
        slot_fence();
    }
    if (ln == 0) {
        meta[0] = epoch;
        meta[1] = lvl;
    }
}

// ------------------------------------------------- byte-state variant
//
// Inside a window a label only ever takes values in [lo, hi), and once the
// window is over a vertex is final: in the structure or not. So one byte per
// vertex is enough for windows of up to 253 ids:
//   0        in the structure (passes its own id on)
//   1 .. D   reached in the current window, label lo + byte - 1
//   0xFE     reached in an earlier window, not in the structure (final)
//   0xFF     not reached by this source
// A quarter of the 32-bit label footprint keeps more of each source's state in
// L2. Bytes change by compare-and-swap on their 32-bit word. Reached vertices
// are listed and their bytes reset to 0xFF when the source is done.
constexpr uint32_t kStStruct = 0u, kStSettled = 0xFEu, kStNone = 0xFFu;

__global__ __launch_bounds__(256) void k_traverse8(TraverseArgs a) {
    __shared__ WaveTile tiles[kTravWaves];
    __shared__ unsigned long long pushed[kTravWaves][1 << kHashBits];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ln = lane_id();
    const int32_t slot = blockIdx.x * kTravWaves + wv;
    if (slot >= a.nslots) return;
    WaveTile& T = tiles[wv];
    unsigned long long* H = pushed[wv];

    uint8_t* sb = a.slots + (int64_t)slot * a.lay.bytes_per_slot;
    GLOBAL uint8_t* st8 = gbl((uint8_t*)(sb + a.lay.off_lab));
    GLOBAL uint32_t* stw = gbl((uint32_t*)(sb + a.lay.off_lab));
    GLOBAL unsigned long long* P = gbl((unsigned long long*)(sb + a.lay.off_p));
    GLOBAL int32_t* qa = gbl((int32_t*)(sb + a.lay.off_qa));
    GLOBAL int32_t* qb = gbl((int32_t*)(sb + a.lay.off_qb));
    GLOBAL int32_t* rowb = gbl((int32_t*)(sb + a.lay.off_row));
    GLOBAL int32_t* touch = gbl((int32_t*)(sb + a.lay.off_touch));
    GLOBAL uint32_t* qs = gbl((uint32_t*)(sb + a.lay.off_qs));
    GLOBAL uint32_t* meta = gbl((uint32_t*)(sb + a.lay.off_meta));
    const __amdgpu_buffer_rsrc_t st_r =
        __builtin_amdgcn_make_buffer_rsrc((uint8_t*)(sb + a.lay.off_lab), (short)0, (int)a.lay.N, 0x00020000);

    const uint32_t R = (uint32_t)a.lay.N;
    uint32_t lvl = meta[1];
    const int32_t D = a.window;  // 1 .. 253
    for (int i = ln; i < (1 << kHashBits); i += 64) H[i] = ~0ull;


    for (;;) {
        unsigned long long k = 0;
        if (ln == 0) k = yield_requested(a) ? ~0ull : atomicAdd(a.item_counter, 1ull);
        k = __shfl(k, 0, 64);
        if (k >= (unsigned long long)a.nitems) break;

        int32_t j, s;
        if (a.item_rows) {
            const int64_t gr = a.item_rows[k];
            j = a.row_job ? a.row_job[gr] : 0;
            s = (int32_t)(gr - a.jobs[j].row_base);
        } else {
            if (a.item_job) {
                j = a.item_job[k];
            } else {
                int32_t lo = 0, hi = a.njobs - 1;
                while (lo < hi) {
                    int32_t mid = (lo + hi + 1) >> 1;
                    if (a.jobs[mid].item_base <= (int64_t)k) lo = mid;
                    else hi = mid - 1;
                }
                j = lo;
            }
            s = a.jobs[j].n - 1 - (int32_t)((int64_t)k - a.jobs[j].item_base);
        }
        j = __builtin_amdgcn_readfirstlane(j);
        s = __builtin_amdgcn_readfirstlane(s);
        const GLOBAL int32_t* rp = gbl(a.jobs[j].row_ptr);
        const GLOBAL int32_t* ci = gbl(a.jobs[j].col_idx);
        const int64_t grow = a.jobs[j].row_base + s;
        if (lvl >= 0xF0000000u) {
            for (int i = ln; i < (1 << kHashBits); i += 64) H[i] = ~0ull;
            for (int64_t i = ln; i < (int64_t)R; i += 64) qs[i] = 0u;
            lvl = 0;
            slot_fence();
        }

        unsigned long long e_alg = 0, e_gpu = 0;
        int32_t rcount = 0, lcount = 0, tcount = 0;
        uint32_t n_iter = 0, n_win = 0;

        // ---- seed: original entries of row s enter the structure
        const int32_t rs = rp[s], re = rp[s + 1];
        int32_t ndiag = 0;
        bool dup = false;
        int32_t pmin = 0x7FFFFFFF;
        for (int32_t e0 = rs; e0 < re; e0 += 64) {
            const int32_t e = e0 + ln;
            const bool act = e < re;
            const int32_t w = act ? ci[e] : -1;
            ndiag += __popcll(__ballot(act && w == s));
            bool fresh = false;
            if (act && w != s) {
                const uint32_t sh = (uint32_t)(w & 3) * 8u;
                const uint32_t old = wg_and(&stw[w >> 2], ~(0xFFu << sh));  // byte -> 0
                fresh = ((old >> sh) & 0xFFu) == kStNone;
                dup |= !fresh;
            }
            const bool below = fresh && w < s;
            {
                unsigned long long m = __ballot(fresh);
                if (fresh) rowb[rcount + (int32_t)lanes_below(m)] = w;
                rcount += __popcll(m);
            }
            lcount += __popcll(__ballot(below));
            if (below) {
                wg_or(&P[w >> 6], 1ull << (w & 63));
                e_alg += (unsigned long long)(rp[w + 1] - rp[w]);
                pmin = min(pmin, w);
            }
        }
        if (ln == 0) {
            e_alg += (unsigned long long)(re - rs);
            e_gpu += (unsigned long long)(re - rs);
        }
        if (__ballot(dup) != 0ull || ndiag > 1) {
            if (ln == 0) atomicOr(&a.jstats[j].err, kErrDuplicate);
        }
        pmin = wave_min(pmin);
        slot_fence();

        // ---- windows of increasing keys
        const int32_t nwp = (s + 63) >> 6;
        int32_t pos = pmin;
        while (pos < s) {
            int32_t found = -1;
            for (int32_t w0 = pos >> 6; w0 < nwp; w0 += 64) {
                const int32_t wi = w0 + ln;
                const unsigned long long word = (wi < nwp) ? ld_coherent(&P[wi]) : 0ull;
                const unsigned long long nz = __ballot(word != 0ull);
                if (nz) {
                    const int jl = __builtin_ctzll(nz);
                    const unsigned long long wd = __shfl(word, jl, 64);
                    found = (w0 + jl) * 64 + __builtin_ctzll(wd);
                    break;
                }
            }
            if (found < 0) break;
            const int32_t lo = found;
            const int32_t hi = (int32_t)min((int64_t)lo + D, (int64_t)s);
            ++n_win;

            GLOBAL int32_t* cur = qa;
            GLOBAL int32_t* nxt = qb;
            int32_t qn = 0;
            const int32_t wlast = (hi - 1) >> 6;
            for (int32_t w0 = lo >> 6; w0 <= wlast; w0 += 64) {
                const int32_t wi = w0 + ln;
                unsigned long long word = 0ull;
                if (wi <= wlast) {
                    word = ld_coherent(&P[wi]);
                    const int64_t b0 = (int64_t)wi * 64;
                    unsigned long long m = ~0ull;
                    if (b0 < lo) m &= ~0ull << (lo - b0);
                    if (b0 + 64 > hi) m &= (hi - b0 >= 64) ? ~0ull : ((1ull << (hi - b0)) - 1ull);
                    word &= m;
                    if (word) wg_and(&P[wi], ~word);
                }
                const int c = __popcll(word);
                const int incl = wave_incl_scan(c);
                int32_t o = qn + incl - c;
                while (word) {
                    const int b = __builtin_ctzll(word);
                    word &= word - 1ull;
                    cur[o++] = wi * 64 + b;
                }
                qn += __shfl(incl, 63, 64);
            }
            const int32_t tmark = tcount;
            wave_fence();

            while (qn > 0) {
                ++lvl;
                ++n_iter;
                int32_t nq = 0;
                bool exact = false;
                for (int32_t c0 = 0; c0 < qn; c0 += 64) {
                    const int32_t i = c0 + ln;
                    const bool act = i < qn;
                    // bit 31 of a queue entry: first visit of the vertex by this source
                    const int32_t fr = ld_coherent(&cur[act ? i : 0]);
                    const int32_t f = fr & 0x7FFFFFFF;
                    const int32_t fs = rp[f];
                    const int32_t deg = act ? rp[f + 1] - fs : 0;
                    if (fr < 0) e_alg += (unsigned long long)deg;
                    const uint32_t fb = (ld_coherent(&stw[f >> 2]) >> ((f & 3) * 8)) & 0xFFu;
                    // a frontier is in the structure (passes its id) or reached in this window
                    const uint32_t ov = fb == kStStruct ? (uint32_t)f
                                                        : (fb >= 1u && fb <= (uint32_t)D) ? (uint32_t)lo + fb - 1u : kInf;
                    e_gpu += (unsigned long long)deg;
                    const int32_t incl = wave_incl_scan(deg);
                    const int32_t total = __shfl(incl, 63, 64);
                    auto round = [&](int32_t (&widx)[kIlp], uint32_t (&outv)[kIlp], bool (&act_e)[kIlp]) {
                        int32_t w[kIlp];
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk) w[kk] = ci[widx[kk]];
                        uint32_t sb8[kIlp];
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk) {
                            act_e[kk] = act_e[kk] && w[kk] != s && outv[kk] != kInf;
                            const uint32_t off = act_e[kk] ? (uint32_t)w[kk] : 0xFFFFFFF0u;
                            sb8[kk] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(st_r, off, 0, 0);
                        }
                        // candidates: an unseen U vertex, or a label the edge lowers
                        bool cand[kIlp];
                        uint32_t nb[kIlp];
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk) {
                            const uint32_t b = sb8[kk];
                            const uint32_t olab = b == kStNone ? kInf
                                                  : (b == kStStruct || b == kStSettled) ? 0u : (uint32_t)lo + b - 1u;
                            if (w[kk] > s) {
                                cand[kk] = act_e[kk] && b == kStNone;
                                nb[kk] = kStStruct;
                            } else {
                                cand[kk] = act_e[kk] && b != kStStruct && b != kStSettled && outv[kk] < olab;
                                nb[kk] = outv[kk] < (uint32_t)w[kk] ? kStStruct : outv[kk] - (uint32_t)lo + 1u;
                            }
                        }
                        // byte updates: compare-and-swap on the containing word
                        uint32_t ob[kIlp];
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk) {
                            ob[kk] = 0x100u;  // no change
                            if (!cand[kk]) continue;
                            const int32_t wk = w[kk];
                            GLOBAL uint32_t* word = &stw[wk >> 2];
                            const uint32_t sh = (uint32_t)(wk & 3) * 8u;
                            uint32_t cw = *word;
                            for (;;) {
                                const uint32_t b = (cw >> sh) & 0xFFu;
                                bool improves;
                                if (wk > s) improves = b == kStNone;
                                else {
                                    const uint32_t olab = b == kStNone ? kInf
                                                          : (b == kStStruct || b == kStSettled) ? 0u
                                                                                                : (uint32_t)lo + b - 1u;
                                    improves = b != kStStruct && b != kStSettled && outv[kk] < olab;
                                }
                                if (!improves) break;
                                const uint32_t nw = (cw & ~(0xFFu << sh)) | (nb[kk] << sh);
                                if (__hip_atomic_compare_exchange_strong(word, &cw, nw, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                                         __HIP_MEMORY_SCOPE_WORKGROUP)) {
                                    ob[kk] = b;
                                    break;
                                }
                            }
                        }
                        bool emit[kIlp], isl[kIlp], push[kIlp], first[kIlp], tch[kIlp];
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk) {
                            const int32_t wk = w[kk];
                            const bool chg = ob[kk] != 0x100u;
                            emit[kk] = isl[kk] = push[kk] = tch[kk] = false;
                            first[kk] = chg && wk < s && ob[kk] == kStNone;
                            if (!chg) continue;
                            if (wk > s) {
                                emit[kk] = true;
                                continue;
                            }
                            if (nb[kk] == kStStruct) {
                                // label fell below w: fill (s, w)
                                emit[kk] = true;
                                isl[kk] = true;
                                if (wk < hi) push[kk] = true;
                                else wg_or(&P[wk >> 6], 1ull << (wk & 63));
                            } else {
                                push[kk] = true;
                                tch[kk] = ob[kk] == kStNone;
                            }
                        }
                        bool evict = false;
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk) {
                            if (push[kk]) {
                                const unsigned long long key = ((unsigned long long)lvl << 32) | (uint32_t)w[kk];
                                const uint32_t h = ((uint32_t)w[kk] * 2654435761u) >> (32 - kHashBits);
                                const unsigned long long prev = __hip_atomic_exchange(
                                    &H[h], key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                                push[kk] = prev != key;
                                evict |= push[kk] && (uint32_t)(prev >> 32) == lvl;
                            }
                        }
                        if (exact) {
#pragma unroll
                            for (int kk = 0; kk < kIlp; ++kk)
                                if (push[kk]) push[kk] = wg_xchg(&qs[w[kk]], lvl) != lvl;
                        }
                        exact = exact || __ballot(evict) != 0ull;
                        // first visits: degree counted at expansion (flagged push) or here
                        bool any = false;
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk) {
                            if (first[kk] && !push[kk]) e_alg += (unsigned long long)(rp[w[kk] + 1] - rp[w[kk]]);
                            any |= emit[kk] | push[kk] | tch[kk];
                        }
                        if (__ballot(any) == 0ull) return;
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk) {
                            unsigned long long m = __ballot(emit[kk]);
                            if (emit[kk]) rowb[rcount + (int32_t)lanes_below(m)] = w[kk];
                            rcount += __popcll(m);
                            lcount += __popcll(__ballot(isl[kk]));
                            m = __ballot(push[kk]);
                            if (push[kk])
                                nxt[nq + (int32_t)lanes_below(m)] =
                                    (int32_t)((uint32_t)w[kk] | (first[kk] ? 0x80000000u : 0u));
                            nq += __popcll(m);
                            m = __ballot(tch[kk]);
                            if (tch[kk]) touch[tcount + (int32_t)lanes_below(m)] = w[kk];
                            tcount += __popcll(m);
                        }
                    };
                    const int32_t maxdeg = wave_max(deg);
                    if (maxdeg <= 64) {
                        for (int32_t t0 = 0; t0 < maxdeg; t0 += kIlp) {
                            int32_t widx[kIlp];
                            uint32_t outv[kIlp];
                            bool act_e[kIlp];
#pragma unroll
                            for (int kk = 0; kk < kIlp; ++kk) {
                                act_e[kk] = t0 + kk < deg;
                                widx[kk] = act_e[kk] ? fs + t0 + kk : 0;
                                outv[kk] = ov;
                            }
                            round(widx, outv, act_e);
                        }
                    } else {
                        T.scan[ln] = incl;
                        T.start[ln] = fs;
                        T.outv[ln] = ov;
                        wave_fence();
                        for (int32_t r0 = 0; r0 < total; r0 += 64 * kIlp) {
                            int32_t widx[kIlp];
                            uint32_t outv[kIlp];
                            bool act_e[kIlp];
#pragma unroll
                            for (int kk = 0; kk < kIlp; ++kk) {
                                const int32_t ei = r0 + kk * 64 + ln;
                                int32_t jl = 0, jh = 63;
                                while (jl < jh) {
                                    const int32_t mid = (jl + jh) >> 1;
                                    if (T.scan[mid] > ei) jh = mid;
                                    else jl = mid + 1;
                                }
                                const int32_t excl = jl ? T.scan[jl - 1] : 0;
                                act_e[kk] = ei < total;
                                widx[kk] = act_e[kk] ? T.start[jl] + (ei - excl) : 0;
                                outv[kk] = T.outv[jl];
                            }
                            round(widx, outv, act_e);
                        }
                    }
                    wave_fence();
                }
                GLOBAL int32_t* t = cur;
                cur = nxt;
                nxt = t;
                qn = nq;
                wave_fence();
            }
            // the window is over: everything it reached outside the structure is final
            for (int32_t i = tmark + ln; i < tcount; i += 64) {
                const int32_t v = ld_coherent(&touch[i]);
                const uint32_t sh = (uint32_t)(v & 3) * 8u;
                uint32_t cw = ld_coherent(&stw[v >> 2]);
                for (;;) {
                    const uint32_t b = (cw >> sh) & 0xFFu;
                    if (b == kStStruct || b == kStSettled) break;
                    const uint32_t nw = (cw & ~(0xFFu << sh)) | (kStSettled << sh);
                    if (__hip_atomic_compare_exchange_strong(&stw[v >> 2], &cw, nw, __ATOMIC_RELAXED,
                                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
                        break;
                }
            }
            wave_fence();
            pos = hi;
        }

        // ---- finish the row: diagonal, copy to the pool, reset the state bytes
        if (ln == 0) rowb[rcount] = s;
        rcount += 1;
        slot_fence();
        unsigned long long off = 0;
        if (ln == 0) off = atomicAdd(a.pool_tail, (unsigned long long)rcount);
        off = __shfl(off, 0, 64);
        const bool fits = (int64_t)(off + rcount) <= a.pool_cap;
        GLOBAL int32_t* pool = gbl(a.pool);
        if (fits)
            for (int32_t i = ln; i < rcount; i += 64) pool[off + i] = ld_coherent(&rowb[i]);
        if (ln == 0) {
            a.row_off[grow] = fits ? (int64_t)off : -1;
            a.row_cnt[grow] = rcount;
            a.row_lcnt[grow] = lcount;
            if (!fits) atomicOr(&a.jstats[j].err, kErrOverflow);
        }
        for (int32_t i = ln; i < rcount - 1; i += 64) {
            const int32_t v = ld_coherent(&rowb[i]);
            wg_or(&stw[v >> 2], 0xFFu << ((v & 3) * 8));
        }
        for (int32_t i = ln; i < tcount; i += 64) {
            const int32_t v = ld_coherent(&touch[i]);
            wg_or(&stw[v >> 2], 0xFFu << ((v & 3) * 8));
        }

        e_alg = wave_sum_u64(e_alg);
        e_gpu = wave_sum_u64(e_gpu);
        if (ln == 0 && a.row_stats)
            a.row_stats[grow] = RowStat{e_alg, e_gpu, n_iter, (n_win & 0x7FFFFFFFu) | (ndiag > 0 ? 0x80000000u : 0u)};
        slot_fence();
    }
    if (ln == 0) meta[1] = lvl;
}

// --------------------------------------------- workgroup-per-source variant
//
// The same traversal with NW wavefronts cooperating on one source: fewer
// sources are in flight at once, so each source's labels keep a larger share
// of its XCD's L2. Frontier chunks of 64 vertices are dealt to the
// wavefronts; queue and row appends go through LDS counters; levels end at a
// workgroup barrier.

struct WgCtl {
    int32_t job, src, found, pmin;
    int32_t cnt[3];        // next-queue counters, one per level modulo 3
    int32_t exact[3];      // per-level exact-dedup flags, same indexing
    int32_t rcount, lcount, dup, ndiag;
    unsigned long long e_alg, e_gpu;
};

template <int NW>
__global__ __launch_bounds__(64 * NW) void k_traverse_wg(TraverseArgs a) {
    constexpr int kWgHashBits = 11;
    __shared__ WaveTile tiles[NW];
    __shared__ unsigned long long H[1 << kWgHashBits];
    __shared__ WgCtl C;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ln = lane_id();
    const int tid = threadIdx.x;
    const int32_t slot = blockIdx.x;
    if (slot >= a.nslots) return;
    WaveTile& T = tiles[wv];

    uint8_t* sb = a.slots + (int64_t)slot * a.lay.bytes_per_slot;
    GLOBAL uint32_t* lab = gbl((uint32_t*)(sb + a.lay.off_lab));
    GLOBAL unsigned long long* P = gbl((unsigned long long*)(sb + a.lay.off_p));
    GLOBAL int32_t* qa = gbl((int32_t*)(sb + a.lay.off_qa));
    GLOBAL int32_t* qb = gbl((int32_t*)(sb + a.lay.off_qb));
    GLOBAL int32_t* rowb = gbl((int32_t*)(sb + a.lay.off_row));
    GLOBAL uint32_t* qs = gbl((uint32_t*)(sb + a.lay.off_qs));
    GLOBAL uint32_t* meta = gbl((uint32_t*)(sb + a.lay.off_meta));
    const __amdgpu_buffer_rsrc_t lab_r = label_rsrc((uint32_t*)(sb + a.lay.off_lab), a.lay.N);

    const uint32_t R = (uint32_t)a.lay.N;
    const uint32_t emax = 0xFFFFFFFFu / R;
    uint32_t epoch = meta[0];
    uint32_t lvl = meta[1];
    const bool line95 = (a.flags & GSOFA_NO_LINE95) == 0;
    const int32_t D = a.window > 0 ? a.window : 1;
    for (int i = tid; i < (1 << kWgHashBits); i += 64 * NW) H[i] = ~0ull;

    // wave-level append of val where pred holds, to buf at an LDS-reserved offset
    auto append = [&](bool pred, int32_t val, GLOBAL int32_t* buf, int32_t* counter) {
        const unsigned long long m = __ballot(pred);
        if (m == 0ull) return;
        int32_t b = 0;
        if (ln == 0) b = atomicAdd(counter, (int32_t)__popcll(m));
        b = __shfl(b, 0, 64);
        if (pred) buf[b + (int32_t)lanes_below(m)] = val;
    };

    for (;;) {
        if (tid == 0) {
            const unsigned long long k = yield_requested(a) ? ~0ull : atomicAdd(a.item_counter, 1ull);
            int32_t j = -1, s = 0;
            if (k < (unsigned long long)a.nitems) {
                if (a.item_rows) {
                    const int64_t gr = a.item_rows[k];
                    j = a.row_job ? a.row_job[gr] : 0;
                    s = (int32_t)(gr - a.jobs[j].row_base);
                } else {
                    if (a.item_job) {
                        j = a.item_job[k];
                    } else {
                        int32_t lo = 0, hi = a.njobs - 1;
                        while (lo < hi) {
                            int32_t mid = (lo + hi + 1) >> 1;
                            if (a.jobs[mid].item_base <= (int64_t)k) lo = mid;
                            else hi = mid - 1;
                        }
                        j = lo;
                    }
                    s = a.jobs[j].n - 1 - (int32_t)((int64_t)k - a.jobs[j].item_base);
                }
            }
            C.job = j;
            C.src = s;
            C.rcount = C.lcount = C.dup = C.ndiag = 0;
            C.pmin = 0x7FFFFFFF;
            C.e_alg = C.e_gpu = 0ull;
        }
        __syncthreads();
        const int32_t j = __builtin_amdgcn_readfirstlane(C.job);
        const int32_t s = __builtin_amdgcn_readfirstlane(C.src);
        if (j < 0) break;
        const GLOBAL int32_t* rp = gbl(a.jobs[j].row_ptr);
        const GLOBAL int32_t* ci = gbl(a.jobs[j].col_idx);
        const int64_t grow = a.jobs[j].row_base + s;

        if (epoch >= emax || (a.flags & GSOFA_RESET_LABELS)) {
            for (int64_t i = tid; i < (int64_t)R; i += 64 * NW) lab[i] = kInf;
            epoch = 0;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __syncthreads();
        }
        if (lvl >= 0xF0000000u) {
            for (int i = tid; i < (1 << kWgHashBits); i += 64 * NW) H[i] = ~0ull;
            for (int64_t i = tid; i < (int64_t)R; i += 64 * NW) qs[i] = 0u;
            lvl = 0;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __syncthreads();
        }
        ++epoch;
        const uint32_t base = 0xFFFFFFFFu - epoch * R;
        auto dec = [&](uint32_t v) -> uint32_t {
            return (v >= base && v - base < R) ? v - base : kInf;
        };
        unsigned long long e_alg = 0, e_gpu = 0;
        uint32_t n_iter = 0, n_win = 0;

        // ---- seed
        const int32_t rs = rp[s], re = rp[s + 1];
        {
            int32_t pmin = 0x7FFFFFFF;
            for (int32_t e0 = rs; e0 < re; e0 += 64 * NW) {
                const int32_t e = e0 + tid;
                const bool act = e < re;
                const int32_t w = act ? ci[e] : -1;
                const int32_t nd = __popcll(__ballot(act && w == s));
                if (ln == 0 && nd) atomicAdd(&C.ndiag, nd);
                bool fresh = false;
                if (act && w != s) {
                    const uint32_t old = wg_min(&lab[w], base);
                    fresh = dec(old) != 0u;
                    if (!fresh) C.dup = 1;
                }
                const bool below = fresh && w < s;
                append(fresh, w, rowb, &C.rcount);
                const int32_t nl = __popcll(__ballot(below));
                if (ln == 0 && nl) atomicAdd(&C.lcount, nl);
                if (below) {
                    wg_or(&P[w >> 6], 1ull << (w & 63));
                    e_alg += (unsigned long long)(rp[w + 1] - rp[w]);
                    pmin = min(pmin, w);
                }
            }
            pmin = wave_min(pmin);
            if (ln == 0 && pmin != 0x7FFFFFFF) atomicMin(&C.pmin, pmin);
        }
        if (tid == 0) {
            e_alg += (unsigned long long)(re - rs);
            e_gpu += (unsigned long long)(re - rs);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __syncthreads();
        if (tid == 0 && (C.dup || C.ndiag > 1)) atomicOr(&a.jstats[j].err, kErrDuplicate);

        // ---- windows
        const int32_t nwp = (s + 63) >> 6;
        int32_t pos = __builtin_amdgcn_readfirstlane(C.pmin);
        GLOBAL int32_t* cur = qa;
        GLOBAL int32_t* nxt = qb;
        while (pos < s) {
            if (tid == 0) C.found = 0x7FFFFFFF;
            __syncthreads();
            for (int32_t w0 = pos >> 6; w0 < nwp; w0 += 64 * NW) {
                const int32_t wi = w0 + tid;
                const unsigned long long word = (wi < nwp) ? ld_coherent(&P[wi]) : 0ull;
                if (word) atomicMin(&C.found, wi * 64 + __builtin_ctzll(word));
                __syncthreads();
                const int32_t got = C.found;
                __syncthreads();  // every thread has read C.found before any may change it
                if (got != 0x7FFFFFFF) break;
            }
            const int32_t found = __builtin_amdgcn_readfirstlane(C.found);
            if (found == 0x7FFFFFFF) break;
            const int32_t lo = found;
            const int32_t hi = (int32_t)min((int64_t)lo + D, (int64_t)s);
            ++n_win;
            // extract [lo, hi) into cur
            if (tid == 0) {
                C.cnt[lvl % 3] = 0;
                C.cnt[(lvl + 1) % 3] = 0;
                C.exact[(lvl + 1) % 3] = 0;
            }
            __syncthreads();
            const int32_t wlast = (hi - 1) >> 6;
            for (int32_t w0 = lo >> 6; w0 <= wlast; w0 += 64 * NW) {
                const int32_t wi = w0 + tid;
                unsigned long long word = 0ull;
                if (wi <= wlast) {
                    word = ld_coherent(&P[wi]);
                    const int64_t b0 = (int64_t)wi * 64;
                    unsigned long long m = ~0ull;
                    if (b0 < lo) m &= ~0ull << (lo - b0);
                    if (b0 + 64 > hi) m &= (hi - b0 >= 64) ? ~0ull : ((1ull << (hi - b0)) - 1ull);
                    word &= m;
                    if (word) wg_and(&P[wi], ~word);
                }
                const int c = __popcll(word);
                int32_t o = 0;
                if (c) o = atomicAdd(&C.cnt[lvl % 3], c);
                while (word) {
                    const int b = __builtin_ctzll(word);
                    word &= word - 1ull;
                    cur[o++] = wi * 64 + b;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __syncthreads();
            int32_t qn = __builtin_amdgcn_readfirstlane(C.cnt[lvl % 3]);

            while (qn > 0) {
                ++lvl;
                ++n_iter;
                // level lvl appends to counter lvl % 3; the one for lvl + 1 was last
                // used two levels ago and is cleared now
                if (tid == 0) {
                    C.cnt[(lvl + 1) % 3] = 0;
                    C.exact[(lvl + 1) % 3] = 0;
                }
                int32_t* nqc = &C.cnt[lvl % 3];
                int32_t* exf = &C.exact[lvl % 3];
                for (int32_t c0 = wv * 64; c0 < qn; c0 += 64 * NW) {
                    const int32_t i = c0 + ln;
                    const bool act = i < qn;
                    const int32_t f = ld_coherent(&cur[act ? i : 0]);
                    const int32_t fs = rp[f];
                    const int32_t deg = act ? rp[f + 1] - fs : 0;
                    const uint32_t dl = dec(ld_coherent(&lab[f]));
                    const uint32_t ov = (dl == kInf) ? kInf : max(dl, (uint32_t)f);
                    e_gpu += (unsigned long long)deg;
                    const int32_t incl = wave_incl_scan(deg);
                    const int32_t total = __shfl(incl, 63, 64);
                    auto round = [&](int32_t (&widx)[kIlp], uint32_t (&outv)[kIlp], bool (&act_e)[kIlp]) {
                        int32_t w[kIlp];
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk) w[kk] = ci[widx[kk]];
                        uint32_t lv[kIlp];
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk) {
                            act_e[kk] = act_e[kk] && w[kk] != s;
                            const uint32_t off = act_e[kk] ? (uint32_t)w[kk] * 4u : 0xFFFFFFF0u;
                            lv[kk] = __builtin_amdgcn_raw_buffer_load_b32(lab_r, off, 0, 0);
                        }
                        bool cand[kIlp];
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk) {
                            const uint32_t d = dec(lv[kk]);
                            if (w[kk] > s) cand[kk] = act_e[kk] && d == kInf;
                            else cand[kk] = act_e[kk] && outv[kk] < d && !(line95 && d < (uint32_t)w[kk]);
                        }
                        uint32_t old[kIlp];
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk)
                            old[kk] = cand[kk] ? wg_min(&lab[w[kk]], base + (w[kk] > s ? 0u : outv[kk])) : base;
                        bool emit[kIlp], isl[kIlp], push[kIlp], first[kIlp];
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk) {
                            const int32_t wk = w[kk];
                            const uint32_t o2 = outv[kk];
                            const uint32_t dold = dec(old[kk]);
                            emit[kk] = isl[kk] = push[kk] = false;
                            first[kk] = cand[kk] && wk < s && dold == kInf;
                            if (!cand[kk]) continue;
                            if (wk > s) {
                                emit[kk] = dold == kInf;
                                continue;
                            }
                            if (o2 < dold && dold >= (uint32_t)wk) {
                                if (o2 < (uint32_t)wk) {
                                    emit[kk] = true;
                                    isl[kk] = true;
                                    if (wk < hi) push[kk] = true;
                                    else wg_or(&P[wk >> 6], 1ull << (wk & 63));
                                } else {
                                    push[kk] = true;
                                }
                            }
                        }
                        int32_t fdeg[kIlp];
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk)
                            fdeg[kk] = first[kk] ? rp[w[kk] + 1] - rp[w[kk]] : 0;
                        bool evict = false;
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk) {
                            if (push[kk]) {
                                const unsigned long long key = ((unsigned long long)lvl << 32) | (uint32_t)w[kk];
                                const uint32_t h = ((uint32_t)w[kk] * 2654435761u) >> (32 - kWgHashBits);
                                const unsigned long long prev = __hip_atomic_exchange(
                                    &H[h], key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                                push[kk] = prev != key;
                                evict |= push[kk] && (uint32_t)(prev >> 32) == lvl;
                            }
                        }
                        if (*exf) {
#pragma unroll
                            for (int kk = 0; kk < kIlp; ++kk)
                                if (push[kk]) push[kk] = wg_xchg(&qs[w[kk]], lvl) != lvl;
                        }
                        if (__ballot(evict) != 0ull && ln == 0) *exf = 1;
                        bool any = false;
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk) {
                            e_alg += (unsigned long long)fdeg[kk];
                            any |= emit[kk] | push[kk];
                        }
                        if (__ballot(any) == 0ull) return;
#pragma unroll
                        for (int kk = 0; kk < kIlp; ++kk) {
                            append(emit[kk], w[kk], rowb, &C.rcount);
                            const int32_t nl = __popcll(__ballot(isl[kk]));
                            if (ln == 0 && nl) atomicAdd(&C.lcount, nl);
                            append(push[kk], w[kk], nxt, nqc);
                        }
                    };
                    const int32_t maxdeg = wave_max(deg);
                    if (maxdeg <= 64) {
                        for (int32_t t0 = 0; t0 < maxdeg; t0 += kIlp) {
                            int32_t widx[kIlp];
                            uint32_t outv[kIlp];
                            bool act_e[kIlp];
#pragma unroll
                            for (int kk = 0; kk < kIlp; ++kk) {
                                act_e[kk] = t0 + kk < deg;
                                widx[kk] = act_e[kk] ? fs + t0 + kk : 0;
                                outv[kk] = ov;
                            }
                            round(widx, outv, act_e);
                        }
                    } else {
                        T.scan[ln] = incl;
                        T.start[ln] = fs;
                        T.outv[ln] = ov;
                        wave_fence();
                        for (int32_t r0 = 0; r0 < total; r0 += 64 * kIlp) {
                            int32_t widx[kIlp];
                            uint32_t outv[kIlp];
                            bool act_e[kIlp];
#pragma unroll
                            for (int kk = 0; kk < kIlp; ++kk) {
                                const int32_t ei = r0 + kk * 64 + ln;
                                int32_t jl = 0, jh = 63;
                                while (jl < jh) {
                                    const int32_t mid = (jl + jh) >> 1;
                                    if (T.scan[mid] > ei) jh = mid;
                                    else jl = mid + 1;
                                }
                                const int32_t excl = jl ? T.scan[jl - 1] : 0;
                                act_e[kk] = ei < total;
                                widx[kk] = act_e[kk] ? T.start[jl] + (ei - excl) : 0;
                                outv[kk] = T.outv[jl];
                            }
                            round(widx, outv, act_e);
                        }
                        wave_fence();
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
                __syncthreads();
                qn = __builtin_amdgcn_readfirstlane(*nqc);
                GLOBAL int32_t* t = cur;
                cur = nxt;
                nxt = t;
            }
            pos = hi;
        }

        // ---- finish the row
        if (e_alg) atomicAdd(&C.e_alg, e_alg);
        if (e_gpu) atomicAdd(&C.e_gpu, e_gpu);
        __syncthreads();
        const int32_t rc = __builtin_amdgcn_readfirstlane(C.rcount) + 1;
        __shared__ unsigned long long s_off;
        if (tid == 0) {
            rowb[rc - 1] = s;
            s_off = atomicAdd(a.pool_tail, (unsigned long long)rc);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __syncthreads();
        const unsigned long long off = s_off;
        const bool fits = (int64_t)(off + rc) <= a.pool_cap;
        GLOBAL int32_t* pool = gbl(a.pool);
        if (fits)
            for (int32_t i = tid; i < rc; i += 64 * NW) pool[off + i] = ld_coherent(&rowb[i]);
        if (tid == 0) {
            a.row_off[grow] = fits ? (int64_t)off : -1;
            a.row_cnt[grow] = rc;
            a.row_lcnt[grow] = C.lcount;
            if (!fits) atomicOr(&a.jstats[j].err, kErrOverflow);
            if (a.row_stats)
                a.row_stats[grow] = RowStat{C.e_alg, C.e_gpu, n_iter,
                                            (n_win & 0x7FFFFFFFu) | (C.ndiag > 0 ? 0x80000000u : 0u)};
        }
        __syncthreads();
    }
    if (tid == 0) {
        meta[0] = epoch;
        meta[1] = lvl;
    }
}

// ------------------------------------------- one thread per source (fill2)
//
// The comparison baseline of the Evaluation section's fill2 study: the fill2
// threshold search run with one GPU thread per source row and no parallelism
// inside a source. Thresholds (vertices of the structure below the source) are
// taken in increasing order from a per-thread binary min-heap; from each, a
// depth-first search walks the unvisited vertices below it; an unvisited
// vertex above the threshold reached that way is in the structure (every
// intermediate of its path is at most the threshold, which is below both ends)
// and, if below the source, becomes a later threshold. Every vertex is visited
// at most once per source, so the edges scanned are exactly the algorithmic
// ones. Per-thread state uses the slot layout: visit stamps in the label array,
// the heap in the first worklist, the search stack in the second, the row
// buffer as in k_traverse.
__global__ __launch_bounds__(256) void k_fill2_thread(TraverseArgs a) {
    const int32_t slot = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (slot >= a.nslots) return;
    uint8_t* sb = a.slots + (int64_t)slot * a.lay.bytes_per_slot;
    uint32_t* stamp = (uint32_t*)(sb + a.lay.off_lab);
    int32_t* heap = (int32_t*)(sb + a.lay.off_qa);
    int32_t* stk = (int32_t*)(sb + a.lay.off_qb);
    int32_t* rowb = (int32_t*)(sb + a.lay.off_row);
    uint32_t* meta = (uint32_t*)(sb + a.lay.off_meta);
    uint32_t epoch = meta[0];
    const int64_t N = a.lay.N;

    for (;;) {
        const unsigned long long k = yield_requested(a) ? ~0ull : atomicAdd(a.item_counter, 1ull);
        if (k >= (unsigned long long)a.nitems) break;
        int32_t j, s;
        if (a.item_rows) {
            const int64_t gr = a.item_rows[k];
            j = a.row_job ? a.row_job[gr] : 0;
            s = (int32_t)(gr - a.jobs[j].row_base);
        } else {
            if (a.item_job) {
                j = a.item_job[k];
            } else {
                int32_t lo = 0, hi = a.njobs - 1;
                while (lo < hi) {
                    const int32_t mid = (lo + hi + 1) >> 1;
                    if (a.jobs[mid].item_base <= (int64_t)k) lo = mid;
                    else hi = mid - 1;
                }
                j = lo;
            }
            s = a.jobs[j].n - 1 - (int32_t)((int64_t)k - a.jobs[j].item_base);
        }
        const int32_t* rp = a.jobs[j].row_ptr;
        const int32_t* ci = a.jobs[j].col_idx;
        const int64_t grow = a.jobs[j].row_base + s;
        // stamps start at kInf (never an epoch); restart the count long before
        if (epoch >= 0xFFFFFFF0u) {
            for (int64_t i = 0; i < N; ++i) stamp[i] = 0u;
            epoch = 0;
        }
        ++epoch;
        stamp[s] = epoch;
        int32_t rcount = 0, lcount = 0, ndiag = 0;
        int64_t hn = 0;
        bool dup = false;
        unsigned long long e_alg = (unsigned long long)(rp[s + 1] - rp[s]);
        uint32_t n_thr = 0;
        auto heap_push = [&](int32_t x) {
            int64_t i = hn++;
            while (i > 0) {
                const int64_t p = (i - 1) >> 1;
                if (heap[p] <= x) break;
                heap[i] = heap[p];
                i = p;
            }
            heap[i] = x;
        };
        auto heap_pop = [&]() -> int32_t {
            const int32_t top = heap[0];
            const int32_t x = heap[--hn];
            int64_t i = 0;
            for (;;) {
                int64_t c = 2 * i + 1;
                if (c >= hn) break;
                if (c + 1 < hn && heap[c + 1] < heap[c]) ++c;
                if (heap[c] >= x) break;
                heap[i] = heap[c];
                i = c;
            }
            if (hn > 0) heap[i] = x;
            return top;
        };
        // the source row's own entries
        for (int32_t e = rp[s]; e < rp[s + 1]; ++e) {
            const int32_t w = ci[e];
            if (w == s) {
                ++ndiag;
                continue;
            }
            if (stamp[w] == epoch) {
                dup = true;
                continue;
            }
            stamp[w] = epoch;
            rowb[rcount++] = w;
            if (w < s) {
                heap_push(w);
                ++lcount;
            }
        }
        // thresholds in increasing order
        while (hn > 0) {
            const int32_t t = heap_pop();
            ++n_thr;
            int64_t sp = 0;
            stk[sp++] = t;
            while (sp > 0) {
                const int32_t x = stk[--sp];
                const int32_t xs = rp[x], xe = rp[x + 1];
                e_alg += (unsigned long long)(xe - xs);
                for (int32_t e = xs; e < xe; ++e) {
                    const int32_t w = ci[e];
                    if (stamp[w] == epoch) continue;
                    stamp[w] = epoch;
                    if (w > t) {
                        rowb[rcount++] = w;
                        if (w < s) {
                            heap_push(w);
                            ++lcount;
                        }
                    } else {
                        stk[sp++] = w;
                    }
                }
            }
        }
        rowb[rcount++] = s;
        const unsigned long long off = atomicAdd(a.pool_tail, (unsigned long long)rcount);
        const bool fits = (int64_t)(off + rcount) <= a.pool_cap;
        if (fits)
            for (int32_t i = 0; i < rcount; ++i) a.pool[off + i] = rowb[i];
        a.row_off[grow] = fits ? (int64_t)off : -1;
        a.row_cnt[grow] = rcount;
        a.row_lcnt[grow] = lcount;
        if (!fits) atomicOr(&a.jstats[j].err, kErrOverflow);
        if (dup || ndiag > 1) atomicOr(&a.jstats[j].err, kErrDuplicate);
        if (a.row_stats)
            a.row_stats[grow] = RowStat{e_alg, e_alg, n_thr, ndiag > 0 ? 0x80000000u : 0u};
    }
    meta[0] = epoch;
}

int32_t traverse_resident_slots(int cus, int mapping) {
    // resident blocks per CU, queried once per mapping
    static std::atomic<int> known[6] = {{-1}, {-1}, {-1}, {-1}, {-1}, {-1}};
    const bool wave_map = mapping == 0 || mapping == 3 || mapping == 4 || mapping == 5;
    if (mapping >= 0 && mapping < 6) {
        const int b = known[mapping].load();
        if (b > 0) return b * (wave_map ? kTravWaves : 1) * cus;
    }
    int blocks = 0;
    hipError_t e;
    if (mapping == 6) {
        // one thread per source: resident threads
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_fill2_thread, 256, 0);
        if (e != hipSuccess || blocks <= 0) {
            (void)hipGetLastError();
            blocks = 1;
        }
        return blocks * 256 * cus;
    }
    if (mapping == 3) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_traverse8, 64 * kTravWaves, 0);
    else if (mapping == 1) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_traverse_wg<16>, 64 * 16, 0);
    else if (mapping == 2) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_traverse_wg<8>, 64 * 8, 0);
    else if (mapping == 4) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_traverse<7, false>, 64 * kTravWaves, 0);
    else if (mapping == 5) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_traverse<6, true>, 64 * kTravWaves, 0);
    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_traverse<8, false>, 64 * kTravWaves, 0);
    if (e != hipSuccess || blocks <= 0) {
        (void)hipGetLastError();
        blocks = 1;
    } else if (mapping >= 0 && mapping < 6) {
        known[mapping].store(blocks);
    }
    return blocks * (wave_map ? kTravWaves : 1) * cus;
}

hipError_t launch_traverse(const TraverseArgs& a, hipStream_t st) {
    if (a.nslots <= 0 || a.nitems <= 0) return hipSuccess;
    if (a.mapping == 6) {
        hipLaunchKernelGGL(k_fill2_thread, dim3((unsigned)((a.nslots + 255) / 256)), dim3(256), 0, st, a);
    } else if (a.mapping == 1) {
        hipLaunchKernelGGL(k_traverse_wg<16>, dim3(a.nslots), dim3(64 * 16), 0, st, a);
    } else if (a.mapping == 2) {
        hipLaunchKernelGGL(k_traverse_wg<8>, dim3(a.nslots), dim3(64 * 8), 0, st, a);
    } else if (a.mapping == 3) {
        const int blocks = (a.nslots + kTravWaves - 1) / kTravWaves;
        hipLaunchKernelGGL(k_traverse8, dim3(blocks), dim3(64 * kTravWaves), 0, st, a);
    } else if (a.mapping == 4) {
        const int blocks = (a.nslots + kTravWaves - 1) / kTravWaves;
        hipLaunchKernelGGL((k_traverse<7, false>), dim3(blocks), dim3(64 * kTravWaves), 0, st, a);
    } else if (a.mapping == 5) {
        const int blocks = (a.nslots + kTravWaves - 1) / kTravWaves;
        hipLaunchKernelGGL((k_traverse<6, true>), dim3(blocks), dim3(64 * kTravWaves), 0, st, a);
    } else {
        const int blocks = (a.nslots + kTravWaves - 1) / kTravWaves;
        hipLaunchKernelGGL((k_traverse<8, false>), dim3(blocks), dim3(64 * kTravWaves), 0, st, a);
    }
    return hipGetLastError();
}

// Per-job sums of the per-source statistics: blocks of 256 rows of one job
// each add their partial sums (jstats starts zeroed; err is left as it is).
__global__ __launch_bounds__(256) void k_job_stats(const Job* jobs, int32_t njobs, const RowStat* rs,
                                                   JobStats* js) {
    __shared__ unsigned long long part[5][4];
    const int32_t j = blockIdx.y;
    if (j >= njobs) return;
    const Job J = jobs[j];
    unsigned long long ea = 0, eg = 0, it = 0, wn = 0, dg = 0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < J.n; r += (int64_t)gridDim.x * blockDim.x) {
        const RowStat x = rs[J.row_base + r];
        ea += x.edges_alg;
        eg += x.edges_gpu;
        it += x.iterations;
        wn += x.windows & 0x7FFFFFFFu;
        dg += x.windows >> 31;
    }
    ea = wave_sum_u64(ea);
    eg = wave_sum_u64(eg);
    it = wave_sum_u64(it);
    wn = wave_sum_u64(wn);
    dg = wave_sum_u64(dg);
    const int wv = threadIdx.x >> 6;
    if (lane_id() == 0) {
        part[0][wv] = ea;
        part[1][wv] = eg;
        part[2][wv] = it;
        part[3][wv] = wn;
        part[4][wv] = dg;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        const unsigned long long v = part[threadIdx.x][0] + part[threadIdx.x][1] + part[threadIdx.x][2] +
                                     part[threadIdx.x][3];
        if (v) {
            unsigned long long* f = threadIdx.x == 0 ? &js[j].edges_alg
                                    : threadIdx.x == 1 ? &js[j].edges_gpu
                                    : threadIdx.x == 2 ? &js[j].iterations
                                    : threadIdx.x == 3 ? &js[j].windows
                                                       : &js[j].diag;
            atomicAdd(f, v);
        }
    }
}

hipError_t launch_job_stats(const Job* jobs_dev, int32_t njobs, int64_t max_n, const RowStat* row_stats,
                            JobStats* jstats, hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>((max_n + 4095) / 4096, 256));
    hipLaunchKernelGGL(k_job_stats, dim3(gx, njobs), dim3(256), 0, st, jobs_dev, njobs, row_stats, jstats);
    return hipGetLastError();
}

// Small device-to-host transfers (statistics, counters, totals) as a kernel
// that writes pinned host memory directly. A copy packet queued behind a
// long-running kernel waits in a copy engine's queue, where it holds up the
// copies of every other stream (a request's input upload waited for another
// request's whole traversal); a kernel waits in its own stream only.
__global__ void k_copy_to_host(const uint32_t* src, uint32_t* dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        __hip_atomic_store(&dst[i], src[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __threadfence_system();
}

// The other direction: pinned host memory (written by the host before the
// launch) into device memory, read with system scope so that no cached copy of
// an earlier use of the staging block is seen.
__global__ void k_copy_from_host(const uint32_t* src, uint32_t* dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = __hip_atomic_load(&src[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

hipError_t launch_copy_from_host(void* dst, const void* src, size_t bytes, hipStream_t st) {
    if (bytes == 0) return hipSuccess;
    if (bytes % 4 != 0) return hipErrorInvalidValue;
    const int64_t n = (int64_t)(bytes / 4);
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_copy_from_host, dim3(blocks), dim3(256), 0, st, static_cast<const uint32_t*>(src),
                       static_cast<uint32_t*>(dst), n);
    return hipGetLastError();
}

// Device-to-device copy (output-pool growth) in 256-thread workgroups.
__global__ void k_copy_device(const uint32_t* src, uint32_t* dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

hipError_t launch_copy_device(void* dst, const void* src, size_t bytes, hipStream_t st) {
    if (bytes == 0) return hipSuccess;
    if (bytes % 4 != 0) return hipErrorInvalidValue;
    const int64_t n = (int64_t)(bytes / 4);
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_copy_device, dim3(blocks), dim3(256), 0, st, static_cast<const uint32_t*>(src),
                       static_cast<uint32_t*>(dst), n);
    return hipGetLastError();
}

hipError_t launch_copy_to_host(void* dst, const void* src, size_t bytes, hipStream_t st) {
    if (bytes == 0) return hipSuccess;
    if (bytes % 4 != 0) return hipErrorInvalidValue;
    const int64_t n = (int64_t)(bytes / 4);
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_copy_to_host, dim3(blocks), dim3(256), 0, st, static_cast<const uint32_t*>(src),
                       static_cast<uint32_t*>(dst), n);
    return hipGetLastError();
}

// ------------------------------------------------------------------ scan

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

int64_t scan_scratch_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t* sh, int64_t& total) {
    // sh: kScanThreads/64 entries
    const int ln = lane_id(), wv = threadIdx.x >> 6;
    int64_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int64_t t = __shfl_up(x, (unsigned)d, 64);
        if (ln >= d) x += t;
    }
    if (ln == 63) sh[wv] = x;
    __syncthreads();
    int64_t pre = 0, tot = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) {
        if (w < wv) pre += sh[w];
        tot += sh[w];
    }
    __syncthreads();
    total = tot;
    return pre + x - v;
}

__device__ __forceinline__ int64_t scan_val(const int32_t* a, const int32_t* b, int64_t i, int64_t n) {
    if (i >= n) return 0;
    return (int64_t)a[i] - (b ? (int64_t)b[i] : 0);
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int32_t* a, const int32_t* b,
                                                              int64_t n, int64_t* partial) {
    __shared__ int64_t sh[kScanThreads / 64];
    const int64_t t0 = (int64_t)blockIdx.x * kScanTile;
    int64_t sum = 0;
    for (int k = 0; k < kScanItems; ++k) sum += scan_val(a, b, t0 + (int64_t)k * kScanThreads + threadIdx.x, n);
    int64_t total;
    block_excl_scan(sum, sh, total);
    if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_partials(int64_t* partial, int64_t nb) {
    __shared__ int64_t sh[kScanThreads / 64];
    int64_t carry = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += kScanThreads) {
        const int64_t i = c0 + threadIdx.x;
        const int64_t v = i < nb ? partial[i] : 0;
        int64_t total;
        const int64_t ex = block_excl_scan(v, sh, total);
        if (i < nb) partial[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) partial[nb] = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const int32_t* a, const int32_t* b, int64_t n,
                                                             int64_t nb, const int64_t* partial, int64_t* out) {
    __shared__ int64_t sh[kScanThreads / 64];
    const int64_t t0 = (int64_t)blockIdx.x * kScanTile;
    // each thread owns kScanItems consecutive elements
    int64_t v[kScanItems];
    int64_t sum = 0;
    const int64_t my0 = t0 + (int64_t)threadIdx.x * kScanItems;
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = scan_val(a, b, my0 + k, n);
        sum += v[k];
    }
    int64_t total;
    int64_t run = (blockIdx.x < nb ? partial[blockIdx.x] : 0) + block_excl_scan(sum, sh, total);
    for (int k = 0; k < kScanItems; ++k) {
        if (my0 + k < n) out[my0 + k] = run;
        run += v[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = partial[nb];
}

hipError_t launch_scan_counts(const int32_t* a, const int32_t* b, int64_t n, int64_t* out,
                              int64_t* scratch, hipStream_t st) {
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 0) {
        hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanThreads), 0, st, scratch, (int64_t)0);
        hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(kScanThreads), 0, st, a, b, (int64_t)0, (int64_t)0,
                           scratch, out);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, st, a, b, n, scratch);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanThreads), 0, st, scratch, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, st, a, b, n, nb, scratch, out);
    return hipGetLastError();
}

// ------------------------------------------------------- segment sorting
//
// A segment holds distinct int32 values. Sorted ascending, its first `split`
// values go to outA and the rest to outB.

// Segment sorts. Every segment holds distinct non-negative ids, so where its
// values span few ids it is ranked in an LDS bitmap (set a bit per value, count
// bits per word, prefix-sum, emit in order): work ~ span/32 + cnt instead of a
// bitonic network's cnt log^2 cnt. One wavefront takes a segment whose span
// fits its 8192-bit bitmap, or a wide one of at most 256 values (bitonic);
// the rest go to a block that ranks them in 16 KB bitmap chunks.
constexpr int kSmallSeg = 256;                 // wavefront bitonic limit
constexpr int kWaveBmWords = kSmallSeg;        // wavefront bitmap: the same LDS, 8192 bits
// Block bitmap chunk: 16 KB of LDS, so eight 256-thread blocks share a CU and
// 2,048 of them sort rows at once (one row per block at a time, latency-bound);
// wider spans take several chunks. With 64 KB chunks (two blocks per CU) the rows
// of the 64^3 27-point stencil took 10.7 ms to sort instead of 5.1.
constexpr int kBitmapBits = 1 << 17;
constexpr unsigned kBigSortBlocks = 2048;

__device__ __forceinline__ void write_split(int32_t idx, int32_t v, int32_t split, int32_t* outA,
                                            int32_t* outB) {
    if (idx < split) outA[idx] = v;
    else outB[idx - split] = v;
}

// wavefront bitonic sort of up to 256 values in LDS buffer buf[256]
__device__ void wave_bitonic_segment(const int32_t* in, int32_t cnt, int32_t split, int32_t* outA,
                                     int32_t* outB, int32_t* buf) {
    const int ln = lane_id();
    int32_t m = 1;
    while (m < cnt) m <<= 1;
    for (int i = ln; i < m; i += 64) buf[i] = i < cnt ? in[i] : 0x7FFFFFFF;
    wave_fence();
    for (int32_t k = 2; k <= m; k <<= 1) {
        for (int32_t jj = k >> 1; jj > 0; jj >>= 1) {
            for (int32_t i = ln; i < m; i += 64) {
                const int32_t ixj = i ^ jj;
                if (ixj > i) {
                    const int32_t x = buf[i], y = buf[ixj];
                    const bool up = (i & k) == 0;
                    if ((x > y) == up) {
                        buf[i] = y;
                        buf[ixj] = x;
                    }
                }
            }
            wave_fence();
        }
    }
    for (int i = ln; i < cnt; i += 64) write_split(i, buf[i], split, outA, outB);
    wave_fence();
}

// wavefront bitmap ranking of a segment with values in [lo, lo + 32 * words)
__device__ void wave_bitmap_segment(const int32_t* in, int32_t cnt, int32_t lo, int32_t words, int32_t split,
                                    int32_t* outA, int32_t* outB, uint32_t* bm) {
    const int ln = lane_id();
    for (int i = ln; i < words; i += 64) bm[i] = 0u;
    wave_fence();
    for (int i = ln; i < cnt; i += 64) {
        const int32_t d = in[i] - lo;
        atomicOr(&bm[d >> 5], 1u << (d & 31));
    }
    wave_fence();
    // lane ln owns words [ln * per, ln * per + per)
    const int per = (words + 63) >> 6;
    int32_t mine = 0;
    for (int q = 0; q < per; ++q) {
        const int i = ln * per + q;
        if (i < words) mine += __popc(bm[i]);
    }
    int32_t r = wave_incl_scan(mine) - mine;
    for (int q = 0; q < per; ++q) {
        const int i = ln * per + q;
        uint32_t word = i < words ? bm[i] : 0u;
        while (word) {
            const int b = __builtin_ctz(word);
            word &= word - 1u;
            write_split(r++, lo + i * 32 + b, split, outA, outB);
        }
    }
    wave_fence();
}

// One wavefront sorts the segment if it can (bitmap for a narrow span,
// bitonic for at most 256 values); returns false if the segment needs a block.
__device__ bool wave_sort_segment(const int32_t* in, int32_t cnt, int32_t split, int32_t* outA, int32_t* outB,
                                  int32_t* buf) {
    if (cnt <= 0) return true;
    int32_t vmin = 0x7FFFFFFF, vmax = -1;
    for (int i = lane_id(); i < cnt; i += 64) {
        const int32_t v = in[i];
        vmin = min(vmin, v);
        vmax = max(vmax, v);
    }
    vmin = wave_min(vmin);
    vmax = wave_max(vmax);
    const int64_t span = (int64_t)vmax - vmin + 1;
    if (span <= 32 * kWaveBmWords) {
        wave_bitmap_segment(in, cnt, vmin, (int32_t)((span + 31) >> 5), split, outA, outB, (uint32_t*)buf);
        return true;
    }
    if (cnt <= kSmallSeg) {
        wave_bitonic_segment(in, cnt, split, outA, outB, buf);
        return true;
    }
    return false;
}

// block bitmap ranking over value chunks of at most kBitmapBits
__device__ void block_sort_segment(const int32_t* in, int32_t cnt, int32_t split, int32_t* outA,
                                   int32_t* outB, uint32_t* bm /* kBitmapBits / 32 words */) {
    __shared__ int32_t red[2];
    __shared__ int32_t wsum[16];
    const int tid = threadIdx.x, nt = blockDim.x;
    int32_t vmin = 0x7FFFFFFF, vmax = -1;
    for (int i = tid; i < cnt; i += nt) {
        const int32_t v = in[i];
        vmin = min(vmin, v);
        vmax = max(vmax, v);
    }
    if (tid == 0) {
        red[0] = 0x7FFFFFFF;
        red[1] = -1;
    }
    __syncthreads();
    atomicMin(&red[0], vmin);
    atomicMax(&red[1], vmax);
    __syncthreads();
    vmin = red[0];
    vmax = red[1];
    __syncthreads();
    int32_t rank_base = 0;
    for (int64_t c0 = vmin; c0 <= vmax; c0 += kBitmapBits) {
        const int64_t bits = std::min<int64_t>((int64_t)vmax - c0 + 1, kBitmapBits);
        const int nwords = (int)((bits + 31) >> 5);
        const int per_t = (nwords + nt - 1) / nt;  // words per thread
        for (int i = tid; i < nwords; i += nt) bm[i] = 0u;
        __syncthreads();
        for (int i = tid; i < cnt; i += nt) {
            const int64_t d = (int64_t)in[i] - c0;
            if (d >= 0 && d < bits) atomicOr(&bm[d >> 5], 1u << (d & 31));
        }
        __syncthreads();
        // each thread owns per_t consecutive words: count, block scan, emit
        int32_t mine = 0;
        for (int q = 0; q < per_t; ++q) {
            const int i = tid * per_t + q;
            if (i < nwords) mine += __popc(bm[i]);
        }
        const int32_t x = wave_incl_scan(mine);
        if (lane_id() == 63) wsum[tid >> 6] = x;
        __syncthreads();
        int32_t pre = 0, tot = 0;
        for (int w = 0; w < nt / 64; ++w) {
            if (w < (tid >> 6)) pre += wsum[w];
            tot += wsum[w];
        }
        int32_t r = rank_base + pre + x - mine;
        for (int q = 0; q < per_t; ++q) {
            const int i = tid * per_t + q;
            uint32_t word = i < nwords ? bm[i] : 0u;
            while (word) {
                const int b = __builtin_ctz(word);
                word &= word - 1u;
                write_split(r++, (int32_t)(c0 + (int64_t)i * 32 + b), split, outA, outB);
            }
        }
        rank_base += tot;
        __syncthreads();
    }
}

// rows: pool segment -> L (entries < row) and U (entries >= row)
__global__ __launch_bounds__(256) void k_sort_rows_small(int64_t nrows, const int64_t* row_off,
                                                         const int32_t* row_cnt, const int32_t* row_lcnt,
                                                         const int32_t* pool, const int64_t* u_ptr,
                                                         int32_t* u_idx, const int64_t* l_ptr,
                                                         int32_t* l_idx, int32_t* big_list,
                                                         int32_t* big_count) {
    __shared__ int32_t buf[4][kSmallSeg];
    const int wv = threadIdx.x >> 6;
    const int64_t r = (int64_t)blockIdx.x * 4 + wv;
    if (r >= nrows) return;
    if (!wave_sort_segment(pool + row_off[r], row_cnt[r], row_lcnt[r], l_idx + l_ptr[r], u_idx + u_ptr[r],
                           buf[wv]))
        if (lane_id() == 0) big_list[atomicAdd(big_count, 1)] = (int32_t)r;
}

__global__ __launch_bounds__(256) void k_sort_rows_big(const int64_t* row_off, const int32_t* row_cnt,
                                                       const int32_t* row_lcnt, const int32_t* pool,
                                                       const int64_t* u_ptr, int32_t* u_idx,
                                                       const int64_t* l_ptr, int32_t* l_idx,
                                                       const int32_t* big_list, const int32_t* big_count) {
    __shared__ uint32_t bm[kBitmapBits / 32];
    const int32_t nb = *big_count;
    for (int32_t q = blockIdx.x; q < nb; q += gridDim.x) {
        const int32_t r = big_list[q];
        block_sort_segment(pool + row_off[r], row_cnt[r], row_lcnt[r], l_idx + l_ptr[r],
                           u_idx + u_ptr[r], bm);
    }
}

hipError_t launch_sort_rows(RowSpace rs, const int64_t* row_off, const int32_t* row_cnt,
                            const int32_t* row_lcnt, const int32_t* pool, const int64_t* u_ptr,
                            int32_t* u_idx, const int64_t* l_ptr, int32_t* l_idx, int32_t* big_list,
                            int32_t* big_count, hipStream_t st) {
    if (rs.nrows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, big_count, (int64_t)1);
    hipLaunchKernelGGL(k_sort_rows_small, dim3((unsigned)((rs.nrows + 3) / 4)), dim3(256), 0, st,
                       rs.nrows, row_off, row_cnt, row_lcnt, pool, u_ptr, u_idx, l_ptr, l_idx,
                       big_list, big_count);
    hipLaunchKernelGGL(k_sort_rows_big, dim3(kBigSortBlocks), dim3(256), 0, st, row_off, row_cnt, row_lcnt, pool,
                       u_ptr, u_idx, l_ptr, l_idx, big_list, big_count);
    return hipGetLastError();
}

// ------------------------------------------------------------ L transpose

__device__ __forceinline__ int64_t job_base_of(const RowSpace& rs, int64_t r) {
    return rs.row_job ? rs.job_row_base[rs.row_job[r]] : 0;
}

// column counts of L (global column = job base + local column)
__global__ __launch_bounds__(256) void k_col_hist(RowSpace rs, const int64_t* l_rptr,
                                                  const int32_t* l_ridx, int32_t* col_cnt) {
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= rs.nrows) return;
    const int64_t b = job_base_of(rs, r);
    for (int64_t e = l_rptr[r] + lane_id(); e < l_rptr[r + 1]; e += 64) atomicAdd(&col_cnt[b + l_ridx[e]], 1);
}

__global__ __launch_bounds__(256) void k_col_scatter(RowSpace rs, const int64_t* l_rptr,
                                                     const int32_t* l_ridx, const int64_t* l_cptr,
                                                     int32_t* cursor, int32_t* tmp) {
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= rs.nrows) return;
    const int64_t b = job_base_of(rs, r);
    const int32_t local = (int32_t)(r - b);
    for (int64_t e = l_rptr[r] + lane_id(); e < l_rptr[r + 1]; e += 64) {
        const int64_t c = b + l_ridx[e];
        tmp[l_cptr[c] + atomicAdd(&cursor[c], 1)] = local;
    }
}

__global__ __launch_bounds__(256) void k_sort_cols_small(int64_t ncols, const int64_t* cptr,
                                                         const int32_t* tmp, int32_t* out,
                                                         int32_t* big_list, int32_t* big_count) {
    __shared__ int32_t buf[4][kSmallSeg];
    const int wv = threadIdx.x >> 6;
    const int64_t c = (int64_t)blockIdx.x * 4 + wv;
    if (c >= ncols) return;
    const int32_t cnt = (int32_t)(cptr[c + 1] - cptr[c]);
    if (!wave_sort_segment(tmp + cptr[c], cnt, cnt, out + cptr[c], nullptr, buf[wv]))
        if (lane_id() == 0) big_list[atomicAdd(big_count, 1)] = (int32_t)c;
}

__global__ __launch_bounds__(256) void k_sort_cols_big(const int64_t* cptr, const int32_t* tmp,
                                                       int32_t* out, const int32_t* big_list,
                                                       const int32_t* big_count) {
    __shared__ uint32_t bm[kBitmapBits / 32];
    const int32_t nb = *big_count;
    for (int32_t q = blockIdx.x; q < nb; q += gridDim.x) {
        const int32_t c = big_list[q];
        const int32_t cnt = (int32_t)(cptr[c + 1] - cptr[c]);
        block_sort_segment(tmp + cptr[c], cnt, cnt, out + cptr[c], nullptr, bm);
    }
}

hipError_t launch_zero_i32(int32_t* p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_zero_i32, dim3(g), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_transpose_l(RowSpace rs, const int64_t* l_rptr, const int32_t* l_ridx,
                              int32_t* col_cnt, int64_t* l_cptr, int32_t* l_cidx,
                              int64_t* scan_scratch, int32_t* cursor, int32_t* tmp,
                              int32_t* big_list, int32_t* big_count, hipStream_t st) {
    const int64_t n = rs.nrows;
    if (n <= 0) return launch_scan_counts(col_cnt, nullptr, 0, l_cptr, scan_scratch, st);
    const unsigned zb = (unsigned)std::min<int64_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_zero_i32, dim3(zb), dim3(256), 0, st, col_cnt, n);
    hipLaunchKernelGGL(k_zero_i32, dim3(zb), dim3(256), 0, st, cursor, n);
    const unsigned rb = (unsigned)((n + 3) / 4);
    hipLaunchKernelGGL(k_col_hist, dim3(rb), dim3(256), 0, st, rs, l_rptr, l_ridx, col_cnt);
    hipError_t e = launch_scan_counts(col_cnt, nullptr, n, l_cptr, scan_scratch, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_col_scatter, dim3(rb), dim3(256), 0, st, rs, l_rptr, l_ridx, l_cptr, cursor, tmp);
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, big_count, (int64_t)1);
    hipLaunchKernelGGL(k_sort_cols_small, dim3(rb), dim3(256), 0, st, n, l_cptr, tmp, l_cidx, big_list, big_count);
    hipLaunchKernelGGL(k_sort_cols_big, dim3(kBigSortBlocks), dim3(256), 0, st, l_cptr, tmp, l_cidx, big_list, big_count);
    return hipGetLastError();
}

// --------------------------------------------------------- supernodes
//
// Definition T3 inside independent blocks of rows (Section 5). Phase I: a row
// s > block start with nnz(U(s,:)) == nnz(U(s-1,:)) - 1 may extend the
// supernode above it; every other row leads one. Phase II: each leader walks
// the rows after it while phase I allows, checking L(s, r) != 0 for the
// current supernode start r; where it fails, s starts a new supernode.

__device__ __forceinline__ int64_t ucount(const int64_t* u_ptr, int64_t r) { return u_ptr[r + 1] - u_ptr[r]; }

__device__ __forceinline__ bool l_has(const int64_t* l_rptr, const int32_t* l_ridx, int64_t s, int32_t col) {
    int64_t lo = l_rptr[s], hi = l_rptr[s + 1];
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (l_ridx[mid] < col) lo = mid + 1;
        else hi = mid;
    }
    return lo < l_rptr[s + 1] && l_ridx[lo] == col;
}

__global__ __launch_bounds__(256) void k_supernodes(RowSpace rs, int64_t nblocks, const int64_t* first,
                                                    const int32_t* len, const int64_t* u_ptr,
                                                    const int64_t* l_rptr, const int32_t* l_ridx,
                                                    int32_t* is_start) {
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= nblocks) return;
    const int64_t f0 = first[b];
    const int64_t end = f0 + len[b];
    const int64_t jb = job_base_of(rs, f0);
    for (int64_t s = f0 + lane_id(); s < end; s += 64) {
        const bool follower = s > f0 && ucount(u_ptr, s) == ucount(u_ptr, s - 1) - 1;
        is_start[s] = follower ? 0 : 1;
    }
    wave_fence();
    for (int64_t r0 = f0 + lane_id(); r0 < end; r0 += 64) {
        const bool leader = !(r0 > f0 && ucount(u_ptr, r0) == ucount(u_ptr, r0 - 1) - 1);
        if (!leader) continue;
        int64_t r = r0;
        for (int64_t s = r0 + 1; s < end; ++s) {
            if (ucount(u_ptr, s) != ucount(u_ptr, s - 1) - 1) break;  // next phase-I leader
            if (!l_has(l_rptr, l_ridx, s, (int32_t)(r - jb))) {
                is_start[s] = 1;
                r = s;
            }
        }
    }
}

hipError_t launch_supernodes(RowSpace rs, int64_t nblocks, const int64_t* block_first_row,
                             const int32_t* block_len, const int64_t* u_ptr, const int64_t* l_rptr,
                             const int32_t* l_ridx, int32_t* is_start, hipStream_t st) {
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_supernodes, dim3((unsigned)((nblocks + 3) / 4)), dim3(256), 0, st, rs, nblocks,
                       block_first_row, block_len, u_ptr, l_rptr, l_ridx, is_start);
    return hipGetLastError();
}

__global__ void k_sn_assemble(RowSpace rs, const int32_t* is_start, const int64_t* scan, int32_t* xsup,
                              int32_t* supno) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < rs.nrows;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = rs.row_job ? rs.row_job[r] : 0;
        const int64_t b = rs.row_job ? rs.job_row_base[j] : 0;
        const int64_t k = scan[r];  // supernode starts before r, all jobs
        if (is_start[r]) xsup[k + j] = (int32_t)(r - b);
        supno[r] = (int32_t)(k + is_start[r] - 1 - scan[b]);
    }
}

__global__ void k_sn_terminal(int32_t njobs, const int64_t* job_row_base, const int32_t* job_n,
                              const int64_t* scan, int32_t* xsup) {
    for (int32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < njobs; j += gridDim.x * blockDim.x)
        xsup[scan[job_row_base[j] + job_n[j]] + j] = job_n[j];
}

hipError_t launch_supernode_assemble(RowSpace rs, int32_t njobs, const int32_t* is_start,
                                     const int64_t* start_scan, int32_t* xsup_all, int32_t* supno_all,
                                     hipStream_t st) {
    (void)njobs;
    if (rs.nrows <= 0) return hipSuccess;
    const unsigned g = (unsigned)std::min<int64_t>((rs.nrows + 255) / 256, 4096);
    hipLaunchKernelGGL(k_sn_assemble, dim3(g), dim3(256), 0, st, rs, is_start, start_scan, xsup_all, supno_all);
    return hipGetLastError();
}

hipError_t launch_supernode_terminals(int32_t njobs, const int64_t* job_row_base, const int32_t* job_n,
                                      const int64_t* start_scan, int32_t* xsup_all, hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    const unsigned g = (unsigned)std::min<int64_t>((njobs + 255) / 256, 1024);
    hipLaunchKernelGGL(k_sn_terminal, dim3(g), dim3(256), 0, st, njobs, job_row_base, job_n, start_scan, xsup_all);
    return hipGetLastError();
}

}  // namespace gsofa
