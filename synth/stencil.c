/*
 * Seeded synthetic sparse-matrix generator (input side only).
 *
 * Produces the stencil matrices that stand in for the paper's SuiteSparse
 * inputs (evaluation section, dataset table): 2D 5/9-point and 3D 7/27-point
 * grid stencils, in natural or geometric nested-dissection order, with each
 * off-diagonal entry dropped independently (keyed by the original grid
 * coordinates of its row and column cell, so the pattern is nonsymmetric),
 * the diagonal always kept, and optional extra entries inside a band.
 *
 * This file holds no part of the symbolic factorisation itself. It is shared
 * by the CPU oracle tests and the GPU path only as a source of inputs.
 *
 * All randomness comes from one counter-based hash, SplitMix64's output
 * function (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014): sm64(x) mixes x + 0x9E3779B97F4A7C15.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

uint64_t synth_sm64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* ---- geometric nested dissection ------------------------------------- */

typedef struct {
    int32_t nx, ny, nz;
    int32_t *rank;   /* natural id -> new id */
    int64_t next;
} nd_ctx;

static void number_box_lex(nd_ctx *c, int lo[3], int hi[3])
{
    for (int z = lo[2]; z < hi[2]; ++z)
        for (int y = lo[1]; y < hi[1]; ++y)
            for (int x = lo[0]; x < hi[0]; ++x) {
                int64_t id = (int64_t)x + (int64_t)c->nx * ((int64_t)y + (int64_t)c->ny * z);
                c->rank[id] = (int32_t)c->next++;
            }
}

/* Recursive bisection: cut the longest axis (ties broken x, then y, then z)
 * at lo + extent/2; number the lower part, then the upper part, then the
 * one-cell-thick separator (lexicographically, x fastest). Boxes whose
 * longest extent is at most 2 are numbered lexicographically. */
static void nd_rec(nd_ctx *c, int lo[3], int hi[3])
{
    int ext[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
    if (ext[0] <= 0 || ext[1] <= 0 || ext[2] <= 0) return;
    int longest = ext[0];
    if (ext[1] > longest) longest = ext[1];
    if (ext[2] > longest) longest = ext[2];
    if (longest <= 2) { number_box_lex(c, lo, hi); return; }
    int ax = (ext[0] == longest) ? 0 : (ext[1] == longest) ? 1 : 2;
    int cut = lo[ax] + ext[ax] / 2;
    int l_hi[3] = {hi[0], hi[1], hi[2]};
    l_hi[ax] = cut;
    nd_rec(c, lo, l_hi);
    int u_lo[3] = {lo[0], lo[1], lo[2]};
    u_lo[ax] = cut + 1;
    nd_rec(c, u_lo, hi);
    int s_lo[3] = {lo[0], lo[1], lo[2]}, s_hi[3] = {hi[0], hi[1], hi[2]};
    s_lo[ax] = cut;
    s_hi[ax] = cut + 1;
    number_box_lex(c, s_lo, s_hi);
}

/* rank[natural id] for an nx*ny*nz grid; order 0 = natural, 1 = ND. */
int synth_order(int32_t nx, int32_t ny, int32_t nz, int order, int32_t *rank)
{
    if (nx <= 0 || ny <= 0 || nz <= 0) return -1;
    int64_t n = (int64_t)nx * ny * nz;
    if (order == 0) {
        for (int64_t i = 0; i < n; ++i) rank[i] = (int32_t)i;
        return 0;
    }
    nd_ctx c = {nx, ny, nz, rank, 0};
    int lo[3] = {0, 0, 0}, hi[3] = {nx, ny, nz};
    nd_rec(&c, lo, hi);
    return c.next == n ? 0 : -2;
}

/* ---- stencil CSR --------------------------------------------------------- */

static int stencil_offsets(int kind, int off[27][3])
{
    int k = 0;
    switch (kind) {
    case 5: /* 2D 5-point */
        off[k][0] = -1; off[k][1] = 0; off[k++][2] = 0;
        off[k][0] = 1;  off[k][1] = 0; off[k++][2] = 0;
        off[k][0] = 0;  off[k][1] = -1; off[k++][2] = 0;
        off[k][0] = 0;  off[k][1] = 1; off[k++][2] = 0;
        break;
    case 9: /* 2D 9-point */
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx)
                if (dx || dy) { off[k][0] = dx; off[k][1] = dy; off[k++][2] = 0; }
        break;
    case 7: /* 3D 7-point */
        for (int a = 0; a < 3; ++a)
            for (int s = -1; s <= 1; s += 2) {
                off[k][0] = off[k][1] = off[k][2] = 0;
                off[k++][a] = s;
            }
        break;
    case 27: /* 3D 27-point */
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx)
                    if (dx || dy || dz) { off[k][0] = dx; off[k][1] = dy; off[k++][2] = dz; }
        break;
    default:
        return -1;
    }
    return k;
}

static int drop_entry(uint64_t seed, int64_t i_nat, int64_t j_nat, uint32_t thresh)
{
    uint64_t h = synth_sm64(synth_sm64(seed ^ (uint64_t)i_nat) ^ (uint64_t)j_nat);
    return (uint32_t)(h >> 32) < thresh;
}

static void sort_small(int32_t *a, int64_t len)
{
    for (int64_t i = 1; i < len; ++i) {
        int32_t v = a[i];
        int64_t j = i - 1;
        while (j >= 0 && a[j] > v) { a[j + 1] = a[j]; --j; }
        a[j + 1] = v;
    }
}

/*
 * Build the CSR of a stencil matrix in the chosen order.
 *   kind: 5, 9 (2D, nz must be 1), 7, 27 (3D)
 *   drop_thresh: an off-diagonal (i,j) is dropped iff
 *       sm64(sm64(seed ^ i_nat) ^ j_nat) >> 32 < drop_thresh
 *     (0 keeps everything; floor(0.2 * 2^32) = 858993459 drops ~20 %)
 *   row_ptr: n+1 entries; col: capacity n*(points) entries.
 * Returns nnz, or a negative value on bad arguments.
 */
int64_t synth_stencil(int kind, int32_t nx, int32_t ny, int32_t nz, int order,
                      uint64_t seed, uint32_t drop_thresh,
                      int32_t *row_ptr, int32_t *col)
{
    int off[27][3];
    int npts = stencil_offsets(kind, off);
    if (npts < 0) return -1;
    if ((kind == 5 || kind == 9) && nz != 1) return -1;
    int64_t n = (int64_t)nx * ny * nz;
    if (n <= 0 || n > 0x7FFFFFFF) return -1;
    int32_t *rank = (int32_t *)malloc(sizeof(int32_t) * n);
    int32_t *inv = (int32_t *)malloc(sizeof(int32_t) * n);
    if (!rank || !inv) { free(rank); free(inv); return -3; }
    if (synth_order(nx, ny, nz, order, rank) != 0) { free(rank); free(inv); return -2; }
    for (int64_t i = 0; i < n; ++i) inv[rank[i]] = (int32_t)i;
    int64_t nnz = 0;
    row_ptr[0] = 0;
    for (int64_t p = 0; p < n; ++p) {
        int64_t i = inv[p];
        int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((int64_t)nx * ny));
        int64_t start = nnz;
        col[nnz++] = (int32_t)p; /* diagonal always kept */
        for (int k = 0; k < npts; ++k) {
            int xx = x + off[k][0], yy = y + off[k][1], zz = z + off[k][2];
            if (xx < 0 || yy < 0 || zz < 0 || xx >= nx || yy >= ny || zz >= nz) continue;
            int64_t j = (int64_t)xx + (int64_t)nx * ((int64_t)yy + (int64_t)ny * zz);
            if (drop_entry(seed, i, j, drop_thresh)) continue;
            col[nnz++] = rank[j];
        }
        sort_small(col + start, nnz - start);
        if (nnz > 0x7FFFFFFF) { free(rank); free(inv); return -4; }
        row_ptr[p + 1] = (int32_t)nnz;
    }
    free(rank);
    free(inv);
    return nnz;
}

/*
 * Add extra off-diagonal entries inside a band, in the final ordering:
 * `draws` draws t = 0..draws-1 with h = sm64(key + t), where
 * key = sm64(seed ^ 0x5851F42D4C957F2D); row i = (h >> 32) mod n,
 * distance d = 1 + ((h >> 8) mod bw), column j = i + d if (h & 1) else i - d.
 * Draws that fall outside [0, n) or hit an existing entry are skipped.
 * Input rows must be sorted. Output capacity: nnz + draws.
 * Returns the new nnz.
 */
int64_t synth_band_extras(int32_t n, const int32_t *row_ptr, const int32_t *col,
                          int64_t draws, uint64_t seed, int32_t bw,
                          int32_t *out_row_ptr, int32_t *out_col)
{
    if (n <= 0 || bw <= 0) return -1;
    uint64_t key = synth_sm64(seed ^ 0x5851F42D4C957F2Dull);
    int64_t nnz = row_ptr[n];
    /* per-row lists of added columns, kept as a flat array sorted afterwards */
    int32_t *er = (int32_t *)malloc(sizeof(int32_t) * (draws > 0 ? draws : 1));
    int32_t *ec = (int32_t *)malloc(sizeof(int32_t) * (draws > 0 ? draws : 1));
    int64_t ne = 0;
    for (int64_t t = 0; t < draws; ++t) {
        uint64_t h = synth_sm64(key + (uint64_t)t);
        int64_t i = (int64_t)((h >> 32) % (uint64_t)n);
        int64_t d = 1 + (int64_t)((h >> 8) % (uint64_t)bw);
        int64_t j = (h & 1) ? i + d : i - d;
        if (j < 0 || j >= n) continue;
        er[ne] = (int32_t)i;
        ec[ne] = (int32_t)j;
        ++ne;
    }
    /* bucket the extras by row */
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t e = 0; e < ne; ++e) cnt[er[e] + 1]++;
    for (int32_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    int32_t *bucket = (int32_t *)malloc(sizeof(int32_t) * (ne > 0 ? ne : 1));
    int64_t *fillp = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    memcpy(fillp, cnt, sizeof(int64_t) * ((size_t)n + 1));
    for (int64_t e = 0; e < ne; ++e) bucket[fillp[er[e]]++] = ec[e];
    int64_t o = 0;
    out_row_ptr[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        int64_t b0 = cnt[i], b1 = cnt[i + 1];
        sort_small(bucket + b0, b1 - b0);
        int64_t a = row_ptr[i], a1 = row_ptr[i + 1];
        int64_t b = b0;
        int32_t last = -1;
        while (a < a1 || b < b1) {
            int32_t v;
            if (b >= b1 || (a < a1 && col[a] <= bucket[b])) v = col[a++];
            else v = bucket[b++];
            if (v == last) continue; /* collision with an existing or repeated entry */
            out_col[o++] = v;
            last = v;
        }
        out_row_ptr[i + 1] = (int32_t)o;
    }
    (void)nnz;
    free(er); free(ec); free(cnt); free(bucket); free(fillp);
    return o;
}
