/*
 * CPU ORACLE -- test infrastructure only.
 *
 * Plain, slow-but-exact reference for sparse symbolic LU factorisation
 * (gSoFa, Gaihre/Li/Liu 2020). Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this code; the product library
 * never does. It shares no code with the GPU path.
 *
 * Graph model (Introduction): vertex = row; every stored off-diagonal
 * (i, j) is a directed edge i -> j; self edges are ignored.
 *
 * Result definition (Background, fill-path theorem): (i, j) is in the filled
 * pattern of L+U iff i == j, or a directed path i -> ... -> j exists whose
 * intermediate vertices are all smaller than both i and j. L(i,:) holds the
 * j < i, U(i,:) the j >= i (the diagonal is always in U).
 *
 * O1 below is the Rose-Tarjan fill2 search the paper starts from
 * (Background, fill2 description): for one source row, thresholds are
 * taken strictly in increasing order; from each threshold t a depth-first
 * search walks unvisited vertices smaller than t; an unvisited vertex w > t
 * reached this way is in the row's structure (every intermediate on the path
 * is <= t < w, and t < src), and if w < src it becomes a later threshold.
 * Every vertex is visited at most once per row. Rows are independent
 * (Design Challenges, challenge 1), so rows run in parallel over threads,
 * never inside a row.
 *
 * S1 is Definition T3 (Background, supernodes): row s joins the supernode
 * that starts at r and extends through s-1 iff
 *     nnz(U(s,:)) == nnz(U(s-1,:)) - 1   and   L(s, r) != 0,
 * evaluated independently inside consecutive blocks of max_supernode rows
 * (the chunk size equals the maximum supernode size, scheduling paragraph of
 * the supernode section), each block's first row starting a supernode.
 */
#define _GNU_SOURCE
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- small growable int32 vector ------------------------------------- */
typedef struct { int32_t *a; int64_t n, cap; } ivec;

static int iv_push(ivec *v, int32_t x)
{
    if (v->n == v->cap) {
        int64_t nc = v->cap ? v->cap * 2 : 1024;
        int32_t *na = (int32_t *)realloc(v->a, sizeof(int32_t) * nc);
        if (!na) return -1;
        v->a = na;
        v->cap = nc;
    }
    v->a[v->n++] = x;
    return 0;
}

/* ---- binary min-heap of vertex ids ------------------------------------ */
static void heap_push(int32_t *h, int64_t *hn, int32_t x)
{
    int64_t i = (*hn)++;
    h[i] = x;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h[p] <= h[i]) break;
        int32_t t = h[p]; h[p] = h[i]; h[i] = t;
        i = p;
    }
}

static int32_t heap_pop(int32_t *h, int64_t *hn)
{
    int32_t top = h[0];
    int64_t n = --(*hn);
    h[0] = h[n];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < n && h[l] < h[m]) m = l;
        if (r < n && h[r] < h[m]) m = r;
        if (m == i) break;
        int32_t t = h[m]; h[m] = h[i]; h[i] = t;
        i = m;
    }
    return top;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/*
 * O1 for one row. `visited` is an n-array where visited[v] == src marks v as
 * seen in this row (rows are distinct, so no reset is needed between rows as
 * long as it starts at -1). `heap` and `stack` have room for n entries.
 * Appends the row's structure, sorted ascending, to `out`; returns the
 * algorithmic edge count deg(src) + sum of deg(v) over the visited v < src.
 */
static int64_t fill2_row(int32_t n, const int32_t *rp, const int32_t *ci,
                         int32_t src, int32_t *visited, int32_t *heap,
                         int32_t *stack, ivec *out, int64_t *lcount)
{
    int64_t start = out->n;
    int64_t hn = 0;
    int64_t edges = (int64_t)rp[src + 1] - rp[src];
    visited[src] = src;
    iv_push(out, src);
    for (int64_t e = rp[src]; e < rp[src + 1]; ++e) {
        int32_t w = ci[e];
        if (visited[w] == src) continue;
        visited[w] = src;
        iv_push(out, w);
        if (w < src) heap_push(heap, &hn, w);
    }
    while (hn > 0) {
        int32_t t = heap_pop(heap, &hn);
        int64_t sp = 0;
        stack[sp++] = t;
        while (sp > 0) {
            int32_t x = stack[--sp];
            edges += (int64_t)rp[x + 1] - rp[x];
            for (int64_t e = rp[x]; e < rp[x + 1]; ++e) {
                int32_t w = ci[e];
                if (visited[w] == src) continue;
                visited[w] = src;
                if (w > t) {
                    iv_push(out, w);          /* max intermediate is t < w */
                    if (w < src) heap_push(heap, &hn, w);
                } else {
                    stack[sp++] = w;          /* w < t: passable under t */
                }
            }
        }
    }
    (void)n;
    qsort(out->a + start, (size_t)(out->n - start), sizeof(int32_t), cmp_i32);
    int64_t lc = 0;
    for (int64_t k = start; k < out->n && out->a[k] < src; ++k) ++lc;
    *lcount = lc;
    return edges;
}

typedef struct {
    int32_t n;
    const int32_t *rp, *ci;
    const int32_t *rows;   /* the rows to compute, in the caller's order */
    int32_t nrows;
    int64_t *cnt, *lcnt, *edges;
    volatile int64_t next; /* work counter over positions, largest rows first */
    const int32_t *order;  /* positions sorted by descending row id */
    int failed;
} job_t;

typedef struct {
    job_t *job;
    ivec out;       /* concatenated rows computed by this thread */
    ivec pos;       /* which positions, in the order computed */
} worker_t;

static void *worker_main(void *arg)
{
    worker_t *w = (worker_t *)arg;
    job_t *j = w->job;
    int32_t *visited = (int32_t *)malloc(sizeof(int32_t) * (size_t)(j->n > 0 ? j->n : 1));
    int32_t *heap = (int32_t *)malloc(sizeof(int32_t) * (size_t)(j->n > 0 ? j->n : 1));
    int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * (size_t)(j->n > 0 ? j->n : 1));
    if (!visited || !heap || !stack) { j->failed = 1; goto done; }
    for (int32_t i = 0; i < j->n; ++i) visited[i] = -1;
    for (;;) {
        int64_t k = __atomic_fetch_add(&j->next, 1, __ATOMIC_RELAXED);
        if (k >= j->nrows) break;
        int32_t p = j->order[k];
        int32_t src = j->rows[p];
        int64_t before = w->out.n, lc = 0;
        j->edges[p] = fill2_row(j->n, j->rp, j->ci, src, visited, heap, stack, &w->out, &lc);
        j->cnt[p] = w->out.n - before;
        j->lcnt[p] = lc;
        if (iv_push(&w->pos, p) != 0) { j->failed = 1; break; }
    }
done:
    free(visited); free(heap); free(stack);
    return NULL;
}

static const int32_t *g_sort_rows;
static int cmp_pos_desc(const void *a, const void *b)
{
    int32_t x = g_sort_rows[*(const int32_t *)a], y = g_sort_rows[*(const int32_t *)b];
    return (x < y) - (x > y);
}

/*
 * Structure of the requested rows (all rows if rows == NULL).
 *   cnt[k]   = |struct(rows[k])| (L and U entries, diagonal included)
 *   lcnt[k]  = |L(rows[k],:)|
 *   edges[k] = algorithmic edges of that row's search
 * *entries receives a malloc'd array with the rows' sorted structures
 * concatenated in the order of `rows` (free with oracle_free).
 * Returns 0, or -1 on allocation failure.
 */
int oracle_rows(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                const int32_t *rows, int32_t nrows, int nthreads,
                int64_t *cnt, int64_t *lcnt, int64_t *edges, int32_t **entries)
{
    int32_t *all = NULL;
    if (!rows) {
        all = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        if (!all) return -1;
        for (int32_t i = 0; i < n; ++i) all[i] = i;
        rows = all;
        nrows = n;
    }
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nrows > 0 ? nrows : 1));
    for (int32_t k = 0; k < nrows; ++k) order[k] = k;
    g_sort_rows = rows;
    qsort(order, (size_t)nrows, sizeof(int32_t), cmp_pos_desc);
    if (nthreads < 1) nthreads = 1;
    job_t job = {n, row_ptr, col_idx, rows, nrows, cnt, lcnt, edges, 0, order, 0};
    worker_t *ws = (worker_t *)calloc((size_t)nthreads, sizeof(worker_t));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    for (int t = 0; t < nthreads; ++t) {
        ws[t].job = &job;
        pthread_create(&th[t], NULL, worker_main, &ws[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    int rc = job.failed ? -1 : 0;
    /* gather into caller order */
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * ((size_t)nrows + 1));
    off[0] = 0;
    for (int32_t k = 0; k < nrows; ++k) off[k + 1] = off[k] + cnt[k];
    int32_t *res = (int32_t *)malloc(sizeof(int32_t) * (size_t)(off[nrows] > 0 ? off[nrows] : 1));
    if (!res) rc = -1;
    for (int t = 0; t < nthreads && rc == 0; ++t) {
        int64_t src_off = 0;
        for (int64_t q = 0; q < ws[t].pos.n; ++q) {
            int32_t p = ws[t].pos.a[q];
            memcpy(res + off[p], ws[t].out.a + src_off, sizeof(int32_t) * (size_t)cnt[p]);
            src_off += cnt[p];
        }
    }
    for (int t = 0; t < nthreads; ++t) { free(ws[t].out.a); free(ws[t].pos.a); }
    free(ws); free(th); free(off); free(order); free(all);
    if (rc != 0) { free(res); return rc; }
    *entries = res;
    return 0;
}

void oracle_free(void *p) { free(p); }

static int l_contains(const int64_t *l_ptr, const int32_t *l_idx, int32_t s, int32_t r)
{
    int64_t lo = l_ptr[s], hi = l_ptr[s + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (l_idx[mid] < r) lo = mid + 1;
        else hi = mid;
    }
    return lo < l_ptr[s + 1] && l_idx[lo] == r;
}

/*
 * S1: supernode partition by Definition T3, block by block.
 *   u_cnt[s] = nnz(U(s,:)) (diagonal included)
 *   L given row-wise (l_ptr[n+1], l_idx sorted within rows)
 *   max_supernode = block size M (0 = one block over all rows)
 * Writes xsup[0..nsuper] (supernode starts followed by n) and supno[n].
 * Returns nsuper.
 */
int32_t oracle_supernodes(int32_t n, const int64_t *u_cnt, const int64_t *l_ptr,
                          const int32_t *l_idx, int32_t max_supernode,
                          int32_t *xsup, int32_t *supno)
{
    int64_t M = max_supernode > 0 ? max_supernode : (n > 0 ? n : 1);
    int32_t ns = 0;
    for (int64_t b = 0; b < n; b += M) {
        int64_t end = b + M < n ? b + M : n;
        int32_t r = (int32_t)b;
        xsup[ns] = r;
        supno[r] = ns;
        ++ns;
        for (int64_t s = b + 1; s < end; ++s) {
            if (u_cnt[s] == u_cnt[s - 1] - 1 && l_contains(l_ptr, l_idx, (int32_t)s, r)) {
                supno[s] = ns - 1;       /* s joins [r .. s-1] */
                continue;
            }
            r = (int32_t)s;              /* s starts a new supernode */
            xsup[ns] = r;
            supno[s] = ns;
            ++ns;
        }
    }
    xsup[ns] = n;
    return ns;
}

/* ---- transpose of a CSR pattern (test helper, no arithmetic of the method)
 * out_ptr[c+1] - out_ptr[c] = entries in column c; rows are visited in
 * increasing order, so each column's row indices come out ascending. This
 * turns the row-wise L of O1 into the column-wise layout the library returns. */
int oracle_transpose(int32_t n, const int64_t *ptr, const int32_t *idx,
                     int64_t *out_ptr, int32_t *out_idx)
{
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!cur) return -1;
    memset(out_ptr, 0, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t e = 0; e < ptr[n]; ++e) out_ptr[idx[e] + 1] += 1;
    for (int32_t c = 0; c < n; ++c) out_ptr[c + 1] += out_ptr[c];
    for (int32_t c = 0; c < n; ++c) cur[c] = out_ptr[c];
    for (int32_t r = 0; r < n; ++r)
        for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e) out_idx[cur[idx[e]]++] = r;
    free(cur);
    return 0;
}
