// Internal interface between the host runtime and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gsofa {

constexpr int kWave = 64;
constexpr uint32_t kInf = 0xFFFFFFFFu;

// One matrix of a launch. Rows of all jobs of a launch live in one global row
// space: job j owns global rows [row_base, row_base + n) and work items
// [item_base, item_base + n).
struct Job {
    const int32_t* row_ptr;   // device, n+1
    const int32_t* col_idx;   // device
    int32_t n;
    int32_t pad;
    int64_t row_base;
    int64_t item_base;
};

// Per-job counters written by the kernels.
struct JobStats {
    unsigned long long edges_alg;
    unsigned long long edges_gpu;
    unsigned long long iterations;
    unsigned long long windows;
    unsigned long long diag;  // rows with a stored diagonal entry
    unsigned long long spilled;  // worklist / row-buffer entries written to host memory
    int32_t err;              // bit 0: repeated column in a row; bit 1: pool overflow
    int32_t pad;
};

// Per-source statistics, stored once per source without atomics and summed
// per matrix afterwards (k_job_stats).
struct RowStat {
    unsigned long long edges_alg;
    unsigned long long edges_gpu;
    uint32_t iterations;
    uint32_t windows;  // bit 31: the row stores its own diagonal entry
};

constexpr int32_t kErrDuplicate = 1;
constexpr int32_t kErrOverflow = 2;

// Working state of one source slot (one wavefront). N = largest n of the launch.
// Labels, level stamps and the pending bitmap cover ids below L (L = N, or in
// memory-budget mode the largest source id of the band plus one: no vertex at
// or above the source is ever labelled). Worklists and the row buffer hold
// qcap_d / rcap_d entries in device memory; in memory-budget mode the rest of
// their worst case (h_q entries per worklist, N - rcap_d for the row buffer)
// lies in pinned host memory, h_stride entries per slot.
struct SlotLayout {
    int64_t N;
    int64_t L;
    int64_t nw64;             // 64-bit words of the pending bitmap
    int64_t qcap;             // worklist capacity (device and host parts together)
    int64_t qcap_d, rcap_d;   // device entries per worklist / row buffer
    int64_t h_q, h_stride;    // host entries per worklist / per slot (budget mode)
    int64_t off_lab, off_p, off_qs, off_qa, off_qb, off_row, off_touch, off_meta, off_ub;
    int64_t bytes_per_slot;
};

SlotLayout slot_layout(int64_t N);
// Memory-budget layout: labels for ids below L, a U-membership bitmap over N
// ids, qcap_d device entries per worklist and row buffer.
SlotLayout slot_layout_budget(int64_t N, int64_t L, int64_t qcap_d);

struct TraverseArgs {
    const Job* jobs;
    int32_t njobs;
    int32_t nslots;
    int64_t nitems;                   // work items (sources) in total
    const int32_t* item_rows;         // optional explicit list of global rows (re-runs)
    const int32_t* row_job;           // global row -> job (only read with item_rows)
    const int32_t* item_job;          // work item -> job (nullptr: one job)
    RowStat* row_stats;               // per global row (nullptr: not recorded)
    unsigned long long* item_counter; // dynamic work distribution
    uint8_t* slots;                   // nslots * bytes_per_slot
    SlotLayout lay;
    int64_t* row_off;                 // per global row: offset in pool (-1 on overflow)
    int32_t* row_cnt;                 // per global row: |struct(row)| incl. diagonal
    int32_t* row_lcnt;                // per global row: |L(row,:)|
    int32_t* pool;
    unsigned long long* pool_tail;
    int64_t pool_cap;
    JobStats* jstats;
    int32_t window;                   // threshold-window span in vertex ids
    uint32_t flags;
    int32_t mapping;                  // 0: one wavefront per source (32-bit labels); 1: 16, 2: 8
                                      // wavefronts per source; 3: one wavefront, byte states;
                                      // 4: as 0, compiled for seven wavefronts per SIMD;
                                      // 5: memory-budget kernel; 6: one thread per source (fill2)
    int32_t* host_spill;              // budget mode: pinned host memory, lay.h_stride entries per slot
    const uint32_t* yield;            // optional flag in fine-grained host memory: when the host
                                      // sets it, the launch stops taking work items (the ones taken
                                      // are finished); item_counter then tells where to resume
};

// Row-space description shared by the assembly kernels. With one job,
// row_job == nullptr and every base is 0.
struct RowSpace {
    int64_t nrows;
    const int32_t* row_job;       // global row -> job
    const int64_t* job_row_base;  // job -> first global row
};

hipError_t launch_validate(const Job* jobs_dev, int32_t njobs, int64_t max_n,
                           int32_t* bad_dev, hipStream_t st);
hipError_t launch_init_slots(uint8_t* slots, int32_t nslots, SlotLayout lay, hipStream_t st);
hipError_t launch_traverse(const TraverseArgs& a, hipStream_t st);
// bytes (a multiple of 4) from device memory to pinned host memory, by a kernel
// on the stream (no copy-engine packet that would wait behind earlier kernels)
hipError_t launch_copy_to_host(void* dst, const void* src, size_t bytes, hipStream_t st);
// bytes (a multiple of 4) from device memory to device memory, by a kernel
hipError_t launch_copy_device(void* dst, const void* src, size_t bytes, hipStream_t st);
// bytes (a multiple of 4) from pinned host memory to device memory, by a kernel
hipError_t launch_copy_from_host(void* dst, const void* src, size_t bytes, hipStream_t st);
// source slots that fit on the device at once (occupancy of the traversal kernel)
int32_t traverse_resident_slots(int cus, int mapping);
// out[base_j + i] = j for i < n_j, base = row_base (by_item false) or item_base
hipError_t launch_row_job(const Job* jobs_dev, int32_t njobs, int64_t max_n, int32_t* row_job,
                          hipStream_t st, bool by_item = false);
// jstats[j] += sums of row_stats over the rows of job j (err is left as it is);
// jstats must be zero beforehand
hipError_t launch_job_stats(const Job* jobs_dev, int32_t njobs, int64_t max_n, const RowStat* row_stats,
                            JobStats* jstats, hipStream_t st);
// out[0..n] = exclusive scan of (a[i] - (b ? b[i] : 0)); scratch >= scan_scratch_elems(n)
int64_t scan_scratch_elems(int64_t n);
hipError_t launch_scan_counts(const int32_t* a, const int32_t* b, int64_t n, int64_t* out,
                              int64_t* scratch, hipStream_t st);
// Sort every row's pool segment; write the entries < row into L (CSR) and the
// rest into U (CSR). big_list needs nrows entries, big_count one int.
hipError_t launch_sort_rows(RowSpace rs, const int64_t* row_off, const int32_t* row_cnt,
                            const int32_t* row_lcnt, const int32_t* pool,
                            const int64_t* u_ptr, int32_t* u_idx,
                            const int64_t* l_ptr, int32_t* l_idx,
                            int32_t* big_list, int32_t* big_count, hipStream_t st);
// L given row-wise (local column ids) -> column-wise (local row ids).
// col_cnt and cursor hold nrows ints, tmp nnz(L) ints.
hipError_t launch_transpose_l(RowSpace rs, const int64_t* l_rptr, const int32_t* l_ridx,
                              int32_t* col_cnt, int64_t* l_cptr, int32_t* l_cidx,
                              int64_t* scan_scratch, int32_t* cursor, int32_t* tmp,
                              int32_t* big_list, int32_t* big_count, hipStream_t st);
hipError_t launch_zero_i32(int32_t* p, int64_t n, hipStream_t st);
// Supernode starts (Definition T3) per block of rows.
hipError_t launch_supernodes(RowSpace rs, int64_t nblocks, const int64_t* block_first_row,
                             const int32_t* block_len, const int64_t* u_ptr,
                             const int64_t* l_rptr, const int32_t* l_ridx,
                             int32_t* is_start, hipStream_t st);
// xsup/supno from the start flags and their exclusive scan.
hipError_t launch_supernode_assemble(RowSpace rs, int32_t njobs, const int32_t* is_start,
                                     const int64_t* start_scan, int32_t* xsup_all,
                                     int32_t* supno_all, hipStream_t st);
hipError_t launch_supernode_terminals(int32_t njobs, const int64_t* job_row_base,
                                      const int32_t* job_n, const int64_t* start_scan,
                                      int32_t* xsup_all, hipStream_t st);

}  // namespace gsofa
