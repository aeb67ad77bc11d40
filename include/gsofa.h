/*
 * gsofa.h -- C ABI of the MI355X (gfx950) sparse symbolic LU factorisation
 * library (method of Gaihre, Li, Liu, "gSoFa: Scalable Sparse Symbolic LU
 * Factorization on GPUs", 2020).
 *
 * Problem (Introduction; Background, symbolic factorisation): given the
 * nonzero pattern of a square sparse matrix A, already permuted for
 * stability and fill reduction and stored as CSR, compute the nonzero
 * structure of its LU factors (no pivoting, no numerical cancellation) and
 * the supernode partition of the rows. By the fill-path theorem (Background)
 * (i, j) is in L+U iff i == j or a directed path i -> ... -> j exists in the
 * graph of A whose intermediate vertices are all smaller than both i and j.
 * Graph model (Introduction): row i is vertex i; every stored off-diagonal
 * (i, j) is an edge i -> j; diagonal entries add nothing.
 *
 * Conventions shared by every entry point:
 *   - indices are int32, output offsets int64; 0-based.
 *   - L is strictly lower (unit diagonal implied); U holds the diagonal
 *     (always, even where A has no diagonal entry).
 *   - default output layout: L as CSC (l_ptr[n+1], row indices ascending
 *     within each column), U as CSR (u_ptr[n+1], column indices ascending).
 *     GSOFA_L_CSR gives L as CSR (columns ascending within each row).
 *   - supernodes follow Definition T3 (Background, supernodes): row s joins
 *     the supernode running from r through s-1 iff
 *     nnz(U(s,:)) == nnz(U(s-1,:)) - 1 and L(s, r) != 0. Detection runs on
 *     independent blocks of max_supernode consecutive rows (the paper's
 *     chunk size equals the maximum supernode size, Section 5), so no
 *     supernode crosses a multiple of max_supernode and the first row of each
 *     block starts one. xsup[k] is the first row of supernode k
 *     (xsup[nsuper] = n); supno[i] is the supernode of row i.
 *   - inputs are caller-owned and read-only; nothing is retained after a call
 *     returns (serve_submit copies its input).
 *   - results are library-owned; release them with gsofa_result_free.
 *     Host result arrays of 1 MiB or more together are in page-locked memory
 *     where the system has it (pageable memory otherwise, and for smaller
 *     results); released blocks are kept for later results up to 8 GiB, and a
 *     release beyond that frees memory, which waits for the work running on
 *     the device.
 *   - no C++ exception crosses this boundary; every entry point returns a
 *     gsofa_status and leaves its output arguments untouched on error.
 *   - one library instance drives the current HIP device of the calling
 *     thread; calls from several threads on one device are serialised.
 */
#ifndef GSOFA_H
#define GSOFA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define GSOFA_API __attribute__((visibility("default")))
#else
#define GSOFA_API
#endif

typedef enum {
    GSOFA_OK = 0,
    GSOFA_EINVAL = 1,     /* malformed input or argument                        */
    GSOFA_ENOMEM = 2,     /* device budget below one source's working state      */
    GSOFA_EDEVICE = 3,    /* a HIP runtime call failed                           */
    GSOFA_EAGAIN = 4,     /* serve: request not finished yet                     */
    GSOFA_ECAPACITY = 5,  /* serve: request larger than the admission budget     */
    GSOFA_ENOTFOUND = 6   /* serve: unknown or already collected ticket          */
} gsofa_status;

/* Largest supported matrix order. Per-source label arrays are addressed with
 * 32-bit byte offsets (4 bytes per vertex), so n must stay below 2^30; a larger
 * n is rejected with GSOFA_EINVAL by every entry point. */
#define GSOFA_MAX_N 1073741823

/* option flags */
#define GSOFA_NO_SUPERNODES     0x1u  /* skip supernode detection (nsuper = 0)        */
#define GSOFA_L_CSR             0x2u  /* return L row-wise (skip the transpose)       */
#define GSOFA_RESULT_ON_DEVICE  0x4u  /* result arrays stay in device memory          */
#define GSOFA_INPUT_ON_DEVICE   0x8u  /* row_ptr / col_idx are device pointers        */
#define GSOFA_NO_LINE95         0x10u /* ablation: relax labels of vertices already in
                                         the structure (the paper's optional check,
                                         Section 4, access-order paragraph, switched
                                         off); results are unchanged                  */
#define GSOFA_LEVEL_ORDER       0x20u /* ablation: the paper's breadth-first frontier
                                         order instead of windowed order; results are
                                         unchanged, work grows                        */
/* traversal mapping (tuning knob, results unchanged); none set -> the
 * autotuner's choice, by default one wavefront per source row with 32-bit labels */
#define GSOFA_MAP_WAVE32        0x40u  /* one wavefront per source row, 32-bit labels  */
#define GSOFA_MAP_WG8           0x80u  /* eight wavefronts per source row              */
#define GSOFA_MAP_WG16          0x100u /* sixteen wavefronts per source row            */
#define GSOFA_MAP_BYTE          0x800u /* one wavefront per source row, one state byte
                                          per vertex (windows up to 253 ids)          */
#define GSOFA_MAP_WAVE32_7      0x1000u /* as GSOFA_MAP_WAVE32, the kernel compiled for
                                          seven instead of eight wavefronts per SIMD
                                          (fewer sources in flight, less spilled per
                                          source)                                      */
/* By default the device work of a call between two host synchronisations
 * (traversal; pointer scans; row sort; supernodes; L transpose and result
 * pointers) is captured into HIP graphs and each phase is one graph launch;
 * executable graphs are cached per phase and updated in place for the next
 * call. GSOFA_EAGER launches every kernel on the stream instead, and so does
 * a call on one matrix of at most 65,536 rows, whose phases are too short for
 * capture to pay; results are identical. */
#define GSOFA_EAGER             0x200u
/* With window = 0, concurrent_sources = 0 and no mapping or ablation flag, the
 * window span, the mapping and the sources in flight are autotuned: for each
 * size class (device, log2 of the largest n, mean row length, batch size) the
 * first call with at least 65,536 source rows times every candidate on one
 * stratified sample of its rows and keeps the fastest for later calls; smaller
 * calls of an untuned class use window 16 with 32-bit labels. GSOFA_TUNE_NOW
 * times the candidates in this call whatever its size, and re-tunes its class.
 * Results are identical for every choice. */
#define GSOFA_TUNE_NOW          0x400u
/* Never time tuner trials in this call (latency-sensitive callers): use the size
 * class's cached choice, else the defaults. The server sets it for every request. */
#define GSOFA_NO_TUNE           0x2000u
/* Memory-budget mode (Space Optimization section): the traversal keeps for each
 * source only what its id needs on the device and puts frontier overflow in host
 * memory, so that more sources fit a small mem_budget_bytes.
 *   - bubble removal: labels, level stamps and the pending bitmap of a source
 *     cover the vertices below it only; sources run in bands of decreasing ids,
 *     each band a launch whose slots are sized for its largest id, so lower
 *     bands fit more sources in flight (dynamic space allocation);
 *   - U-side membership is a bitmap over all n vertices;
 *   - external frontier management: the two worklists and the row buffer of a
 *     source hold opts->queue_cap entries in device memory; entries beyond that
 *     are written to pinned host memory and read back from there by the next
 *     level (or, for the row buffer, by the copy to the output pool);
 *   - sources in flight are then cut until the slots fit the budget.
 * Results are identical to the default mode; stats report spilled entries and
 * launches. */
#define GSOFA_BUDGET_MODE       0x4000u
/* Comparison baseline (Evaluation, fill2 comparison): the fill2 threshold search
 * with one GPU thread per source row, no intra-source parallelism. Results are
 * identical; it exists to be timed against the default kernel. */
#define GSOFA_MAP_THREAD        0x8000u
/* Ablation of the maxId re-initialisation optimisation (Section 4, maxId
 * initialisation paragraph): reset the whole label array of a slot before every
 * source (O(n) per source) instead of moving to a fresh value range. Results
 * are unchanged. */
#define GSOFA_RESET_LABELS      0x10000u
/* Server: work-item admission. A large request's traversal (more than 65,536
 * rows) gives its wave slots up when a request is admitted onto a full device:
 * it takes no further source, finishes the ones it holds, and resumes from
 * where it stopped once the new request's traversal is on the device (at most
 * once per 20 ms). Results are unchanged. Off by default: the server already
 * keeps a reserve of wave slots that large traversals never take, and a yield
 * idles the large traversal until its slowest current source is done. Ignored
 * outside the server. */
#define GSOFA_SERVE_YIELD       0x20000u

/* A CSR pattern: n rows, row_ptr[n+1], col_idx[row_ptr[n]]; host pointers
 * unless GSOFA_INPUT_ON_DEVICE is set. */
typedef struct {
    int32_t n;
    const int32_t* row_ptr;
    const int32_t* col_idx;
} gsofa_csr;

typedef struct {
    int32_t status;             /* per-matrix status (batch, serve)                       */
    int32_t concurrent_sources; /* sources in flight at once (#C)                         */
    uint64_t iterations;        /* frontier-expansion steps, summed over sources          */
    uint64_t windows;           /* threshold windows, summed over sources                 */
    uint64_t edges_alg;         /* algorithmic edges: for each source row, deg(src) plus
                                   deg(v) of every v < src reachable from src through
                                   vertices < src (each counted once per source)          */
    uint64_t edges_gpu;         /* edges actually scanned, revisits included              */
    uint64_t peak_device_bytes; /* device working memory of this call                     */
    double t_traverse_ms;       /* fill-detection kernel time: the per-source seed (the
                                   source row's own entries) runs inside the traversal
                                   kernel, so seed and traversal are timed together       */
    double t_emit_ms;           /* pointer scans and per-row sort into CSR                */
    double t_supernode_ms;
    double t_total_ms;          /* whole call, host copies included                       */
    int32_t window;             /* threshold-window span used                             */
    int32_t mapping;            /* traversal mapping used: 0 one wavefront per source with
                                   32-bit labels, 4 the same compiled for seven wavefronts
                                   per SIMD, 3 one wavefront with byte states, 2 / 1 eight
                                   / sixteen wavefronts per source, 5 the memory-budget
                                   kernel (GSOFA_BUDGET_MODE), 6 one thread per source
                                   (GSOFA_MAP_THREAD, comparison baseline)                */
    double t_tune_ms;           /* autotuner trial time spent in this call (0 if none)    */
    uint64_t spilled_entries;   /* worklist and row-buffer entries written to host memory
                                   (GSOFA_BUDGET_MODE; 0 otherwise)                       */
    int32_t launches;           /* traversal launches (source-id bands in budget mode,
                                   relaunches of a served request after it yielded,
                                   pool-regrowth re-runs)                                 */
    int32_t pad_;
} gsofa_stats;

typedef void* (*gsofa_alloc_fn)(size_t bytes, void* ctx);
typedef void (*gsofa_free_fn)(void* ptr, void* ctx);

typedef struct {
    uint32_t struct_size;       /* sizeof(gsofa_opts); 0 or a zeroed struct = defaults   */
    int32_t max_supernode;      /* block size for supernodes; 0 -> 128; <0 -> unbounded  */
    int64_t mem_budget_bytes;   /* device working-memory cap; 0 -> 90 % of free memory    */
    uint32_t flags;             /* GSOFA_* flags above                                    */
    int32_t window;             /* threshold-window span (vertex ids); 0 -> autotuned    */
    int32_t concurrent_sources; /* sources in flight; 0 -> planned from memory and CUs    */
    void* stream;               /* hipStream_t to run on; NULL -> the null stream         */
    gsofa_alloc_fn dev_alloc;   /* optional caller-side device allocator (for example a
                                   tensor framework's caching allocator). With dev_alloc
                                   and dev_free both set, every device buffer of the call
                                   comes from dev_alloc(bytes, alloc_ctx), called on the
                                   calling thread (worker threads for the server) with the
                                   call's device current: source-slot state, output pool,
                                   scratch and GSOFA_RESULT_ON_DEVICE results. It returns
                                   memory aligned to at least 256 bytes, or NULL (the call
                                   then fails with GSOFA_ENOMEM). The library's own device
                                   cache is neither used nor filled by such a call.
                                   Working buffers go back through dev_free(ptr, alloc_ctx)
                                   only once the call's device work has completed; result
                                   buffers when gsofa_result_free releases the last result
                                   of the call. Setting only one of the two: GSOFA_EINVAL. */
    gsofa_free_fn dev_free;
    void* alloc_ctx;            /* passed unchanged to dev_alloc and dev_free              */
    int32_t queue_cap;          /* GSOFA_BUDGET_MODE: device entries per source worklist
                                   and row buffer before the overflow goes to host memory;
                                   0 -> 8192                                               */
    int32_t pad_;
} gsofa_opts;

typedef struct {
    int32_t n;
    int64_t nnz_a;              /* stored entries of A                                    */
    int64_t nnz_l, nnz_u;       /* strict L; U with diagonal                              */
    int64_t fills;              /* nnz(L) + nnz(U) - nnz(pattern(A) with diagonal)        */
    int64_t* l_ptr;             /* [n+1]: CSC column pointers (CSR row pointers with
                                   GSOFA_L_CSR)                                           */
    int32_t* l_idx;             /* [nnz_l]                                                */
    int64_t* u_ptr;             /* [n+1]: CSR row pointers of U                           */
    int32_t* u_idx;             /* [nnz_u]                                                */
    int32_t nsuper;
    int32_t* xsup;              /* [nsuper+1]                                             */
    int32_t* supno;             /* [n]                                                    */
    uint32_t flags;             /* flags the result was produced with                     */
    gsofa_stats stats;
    void* internal_;            /* library bookkeeping; do not touch                      */
} gsofa_result;

typedef struct gsofa_server gsofa_server;

/*
 * Symbolic factorisation of one matrix: fill detection for every source row
 * (Section 4: per-source traversal of the graph of A carrying, for every
 * reached vertex, the smallest achievable maximum intermediate id, relaxed
 * with atomic minimum, and the fill-path test), many sources concurrently
 * (Section 4, multi-source paragraph), then supernodes (Section 5).
 *   n >= 0; row_ptr[n+1] with row_ptr[0] == 0 and non-decreasing;
 *   col_idx[row_ptr[n]] in [0, n), no repeated column within a row
 *   (column order within a row is free; a missing diagonal is allowed).
 * Errors: GSOFA_EINVAL for a malformed CSR or bad opts; GSOFA_ENOMEM when
 * mem_budget_bytes cannot hold one source's state; GSOFA_EDEVICE on HIP
 * failure. On success *out receives a new result.
 */
GSOFA_API int gsofa_symbolic(int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
                   const gsofa_opts* opts, gsofa_result** out);

/*
 * Many independent matrices in one pass: every (matrix, source row) pair is
 * a work item of one persistent traversal launch; sorting, assembly and
 * supernodes run once over the whole batch. outs[count] receives one result
 * per matrix (each freed separately). Returns GSOFA_OK, or the first failing
 * per-matrix status (every outs[i] is still set, with stats.status telling
 * which ones failed and no arrays on those).
 */
GSOFA_API int gsofa_batch(int32_t count, const gsofa_csr* mats, const gsofa_opts* opts,
                gsofa_result** outs);

/*
 * Request server with continuous batching: a free worker (at most
 * max_inflight are busy) admits the oldest queued request whose estimated
 * device memory fits what is left of the budget (opts->mem_budget_bytes,
 * default: free device memory plus what the library holds idle); a request
 * waiting for memory is passed by later ones at most 32 times, then admitted
 * before any other once its memory is free. A worker that
 * admits a request of at most 65,536 rows also takes the later queued small
 * requests that fit (up to 64 and 2^20 rows together) and runs them as one
 * persistent launch, as gsofa_batch does. Admitted work runs concurrently on
 * the device and finished requests release their memory, which admits the
 * next. A request's traversal takes a share of the resident wavefronts less
 * a reserve of 256 that kernels of requests admitted meanwhile run in; a
 * request admitted with nothing else running or queued takes every resident
 * wavefront but the reserve, and a large request (over 65,536 rows) admitted
 * while its traversal runs starts its own traversal when that one ends; with
 * GSOFA_SERVE_YIELD running large traversals also give their wave slots up to
 * a request admitted onto a full device. Requests never time tuner trials
 * (cached choices or defaults).
 *   serve_submit copies the CSR (host pointers) and returns a ticket.
 *     GSOFA_ECAPACITY if the request alone can never fit the budget.
 *   serve_poll waits up to timeout_us microseconds (0 = just test,
 *     <0 = wait forever) for the ticket; GSOFA_EAGAIN if not done,
 *     GSOFA_ENOTFOUND for an unknown or collected ticket; otherwise the
 *     request's own status, with *out set on GSOFA_OK.
 *   serve_close drops requests that were not admitted yet, waits for the
 *     running ones and frees the server (with every uncollected result).
 */
GSOFA_API int gsofa_serve_open(const gsofa_opts* opts, int32_t max_inflight, gsofa_server** srv);
GSOFA_API int gsofa_serve_submit(gsofa_server* srv, const gsofa_csr* m, uint64_t* ticket);
GSOFA_API int gsofa_serve_poll(gsofa_server* srv, uint64_t ticket, int32_t timeout_us,
                     gsofa_result** out);
GSOFA_API int gsofa_serve_close(gsofa_server* srv);

/* Frees a result (host or device arrays). NULL is ignored. */
GSOFA_API void gsofa_result_free(gsofa_result* r);

/* Static text for a status code. */
GSOFA_API const char* gsofa_strerror(int status);

/* Releases cached device memory held between calls on the current device. */
GSOFA_API int gsofa_release_cache(void);

/* Process-wide HIP graph counters since load: out[0] executable graphs
 * instantiated, out[1] executable graphs updated in place for a later call,
 * out[2] graph launches. out must hold 3 entries; GSOFA_EINVAL if NULL. */
GSOFA_API int gsofa_graph_counters(uint64_t* out);

/*
 * For callers that cannot allocate device memory (code between the nodes of a
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * gsofa_symbolic on device-resident input into caller-provided device output
 * arrays, with no device allocation at all. Every working buffer is carved
 * from one fixed scratch array of GSOFA_NOALLOC_SCRATCH_BYTES that the library
 * holds in device memory on every GPU it runs on, from the first call on that
 * GPU until the process ends; it calls no hipMalloc, hipFree or other
 * allocating routine, and no caller allocator.
 *   row_ptr[n+1], col_idx[row_ptr[n]]: device pointers, as for
 *     GSOFA_INPUT_ON_DEVICE (checked on the device; GSOFA_EINVAL if malformed).
 *   u_ptr[n+1] (int64), u_idx[u_cap]: U in CSR; l_ptr[n+1] (int64),
 *     l_idx[l_cap]: L in CSC (CSR with GSOFA_L_CSR); xsup[n+1], supno[n]:
 *     supernodes (may be NULL with GSOFA_NO_SUPERNODES). All device pointers,
 *     caller-owned; n >= 0 and u_ptr, l_ptr non-NULL even for n = 0.
 *   counts (host, caller-owned): nnz and fill totals, nsuper, statistics, and
 *     scratch_bytes, the scratch the call needed (or would have needed).
 *   opts: stream, window, concurrent_sources, max_supernode and the flags
 *     GSOFA_NO_SUPERNODES, GSOFA_L_CSR, GSOFA_NO_LINE95, GSOFA_LEVEL_ORDER,
 *     GSOFA_MAP_WAVE32, GSOFA_MAP_WAVE32_7, GSOFA_INPUT_ON_DEVICE,
 *     GSOFA_RESULT_ON_DEVICE, GSOFA_EAGER, GSOFA_NO_TUNE; any other flag, a
 *     caller allocator or a memory budget -> GSOFA_EINVAL.
 * GSOFA_ECAPACITY (with counts->scratch_bytes and, once known, the nnz totals
 * set) when the matrix needs more than the scratch array holds -- its per-row
 * arrays and at least one source's state up front, the output structure after
 * fill detection -- or when u_cap / l_cap are below nnz(U) / nnz(L); the
 * output arrays then hold no result (their contents are unspecified).
 * Otherwise the result equals gsofa_symbolic's.
 * Calls share the one scratch array of their GPU, which keeps the previous
 * call's contents (every call clears what it needs cleared): the entry point
 * holds a process-wide lock and returns only after its device work on
 * opts->stream has completed, so calls from one process never overlap; calls
 * that bypassed this (none can through this ABI) would race on it.
 */
#define GSOFA_NOALLOC_SCRATCH_BYTES (128ull << 20)

typedef struct {
    int64_t nnz_a, nnz_l, nnz_u, fills;
    int32_t nsuper;
    int32_t pad_;
    int64_t scratch_bytes;      /* scratch needed by this call (what it would need on
                                   GSOFA_ECAPACITY)                                       */
    gsofa_stats stats;
} gsofa_counts;

GSOFA_API int gsofa_symbolic_noalloc(int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
                                     const gsofa_opts* opts, int64_t* u_ptr, int32_t* u_idx,
                                     int64_t u_cap, int64_t* l_ptr, int32_t* l_idx, int64_t l_cap,
                                     int32_t* xsup, int32_t* supno, gsofa_counts* counts);

/* Process-wide device-memory counters since load, for the current device and
 * all others together: out[0] bytes the library currently holds from its own
 * hipMalloc calls (in use and cached idle), out[1] hipMalloc calls made by the
 * library, out[2] bytes obtained through caller allocators (dev_alloc),
 * out[3] dev_alloc calls, out[4] dev_free calls. out must hold 5 entries;
 * GSOFA_EINVAL if NULL. */
GSOFA_API int gsofa_memory_counters(uint64_t* out);

#ifdef __cplusplus
}
#endif

#endif /* GSOFA_H */
