/*
 * CPU comparison baseline: the Gilbert-Peierls symbolic factorisation
 * (Background section, where the paper describes it as the column-by-column
 * form of fill1 that sequential CPU codes use). Not the oracle and not the
 * product: it is timed beside the GPU path, and its tests check it against
 * the oracle.
 *
 * Column k of the factors: starting from the row indices of A(:, k), a
 * depth-first search in the graph of the already computed columns of L
 * (edge j -> i for every L(i, j) != 0, j < k) reaches exactly the rows of
 * column k of L+U. Rows above k (and k itself, always present) form U(:, k),
 * rows below k form L(:, k), which then serves the later columns. Columns
 * depend on earlier ones, so the method is sequential.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t *a;
    int64_t n, cap;
} gvec;

static int gv_push(gvec *v, int32_t x)
{
    if (v->n == v->cap) {
        int64_t c = v->cap ? 2 * v->cap : 4096;
        int32_t *p = (int32_t *)realloc(v->a, sizeof(int32_t) * (size_t)c);
        if (!p) return -1;
        v->a = p;
        v->cap = c;
    }
    v->a[v->n++] = x;
    return 0;
}

static int cmp_i32(const void *x, const void *y)
{
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

/*
 * A given by columns (col_ptr[n+1], row_idx). Outputs, malloc'ed here and
 * released with gp_free: L by columns (*l_ptr[n+1], *l_idx, rows ascending)
 * and U by columns (*u_ptr[n+1], *u_idx, rows ascending, diagonal included).
 * *edges = L entries scanned by the searches. ncols_done: columns computed
 * (all n unless time_limit_s > 0 stopped it early; the limit is checked
 * between columns with the supplied clock callback, NULL for none).
 */
int gp_symbolic(int32_t n, const int32_t *col_ptr, const int32_t *row_idx, int64_t **l_ptr,
                int32_t **l_idx, int64_t **u_ptr, int32_t **u_idx, int64_t *edges,
                double (*clock)(void), double time_limit_s, int32_t *ncols_done)
{
    int64_t *lp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *up = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *mark = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *reach = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    gvec L = {0}, U = {0};
    int64_t scanned = 0;
    int rc = -1;
    int32_t k = 0;
    if (!lp || !up || !mark || !stack || !reach) goto out;
    for (int32_t i = 0; i < n; ++i) mark[i] = -1;
    const double t0 = clock ? clock() : 0.0;
    for (k = 0; k < n; ++k) {
        if (clock && time_limit_s > 0 && k > 0 && (k & 255) == 0 && clock() - t0 > time_limit_s) break;
        int32_t nr = 0;
        mark[k] = k;
        reach[nr++] = k;
        for (int32_t e = col_ptr[k]; e < col_ptr[k + 1]; ++e) {
            const int32_t r0 = row_idx[e];
            if (mark[r0] == k) continue;
            mark[r0] = k;
            reach[nr++] = r0;
            int32_t sp = 0;
            stack[sp++] = r0;
            while (sp > 0) {
                const int32_t v = stack[--sp];
                if (v >= k) continue; /* column v of L is not known yet */
                scanned += lp[v + 1] - lp[v];
                for (int64_t f = lp[v]; f < lp[v + 1]; ++f) {
                    const int32_t w = L.a[f];
                    if (mark[w] == k) continue;
                    mark[w] = k;
                    reach[nr++] = w;
                    stack[sp++] = w;
                }
            }
        }
        qsort(reach, (size_t)nr, sizeof(int32_t), cmp_i32);
        for (int32_t t = 0; t < nr; ++t) {
            if (reach[t] <= k) {
                if (gv_push(&U, reach[t])) goto out;
            } else {
                if (gv_push(&L, reach[t])) goto out;
            }
        }
        lp[k + 1] = L.n;
        up[k + 1] = U.n;
    }
    for (int32_t c = k; c < n; ++c) {
        lp[c + 1] = L.n;
        up[c + 1] = U.n;
    }
    *l_ptr = lp;
    *u_ptr = up;
    *l_idx = L.a ? L.a : (int32_t *)malloc(sizeof(int32_t));
    *u_idx = U.a ? U.a : (int32_t *)malloc(sizeof(int32_t));
    *edges = scanned;
    *ncols_done = k;
    lp = up = NULL;
    L.a = U.a = NULL;
    rc = 0;
out:
    free(lp);
    free(up);
    free(mark);
    free(stack);
    free(reach);
    free(L.a);
    free(U.a);
    return rc;
}

void gp_free(void *p) { free(p); }
