/*
 * Dexel offset oracle: plain, slow, obviously correct CPU reference.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code
 * with the GPU library and must never be called on the product path.
 *
 * What it computes (Chen, Panozzo, Dumas, "Half-Space Power Diagrams and
 * Discrete Surface Offsets"):
 *
 *  - Dilation (Sec. 3.1, "Dilation" equation): the set of points within
 *    distance r of the shape.  For a dexel grid with unit spacing this is,
 *    per output column c, the union over every input column c' with lateral
 *    squared distance d2 = dx^2 + dy^2 <= r^2 and every interval [a, b] of c'
 *    of the capsule chord [a - h, b + h], h = sqrt(r^2 - d2).  This is the
 *    brute-force dilation the paper uses as its correctness baseline
 *    (Sec. 4, "Baseline Comparison"): every segment emits its dilated
 *    segments in the disk of radius r around it and all of them are merged.
 *  - Erosion (Sec. 3.1, "Erosion"): complement, dilate, complement.  Gaps
 *    of a column are taken as closed intervals with -inf/+inf ends; only
 *    in-grid columns are complemented (columns outside the grid impose no
 *    constraint); the final complement keeps intervals of positive length.
 *
 * Two precisions:
 *  - ORACLE_F64: h = sqrt(r^2 - d2) in double, chord ends a - h, b + h in
 *    double, union in double.  This is the reference result.
 *  - ORACLE_F32_MODEL: h is the double square root rounded once to float,
 *    each chord end is the exact difference/sum rounded once to float, and
 *    the union is taken over these float values.  This models a float32
 *    evaluation of the same definition.
 *
 * Union rule: sort chords by (start, end); a chord whose start is <= the
 * running end of the current group joins it (closed intervals, so touching
 * intervals merge).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_F64 0
#define ORACLE_F32_MODEL 1
#define ORACLE_DILATE 0
#define ORACLE_ERODE 1

typedef struct {
    double lo, hi;
} ivl;

typedef struct {
    int dx, dy;
    double h;
} stencil_pt;

static int cmp_ivl(const void* pa, const void* pb) {
    const ivl* a = (const ivl*)pa;
    const ivl* b = (const ivl*)pb;
    if (a->lo < b->lo) return -1;
    if (a->lo > b->lo) return 1;
    if (a->hi < b->hi) return -1;
    if (a->hi > b->hi) return 1;
    return 0;
}

/* All integer offsets with dx^2 + dy^2 <= r^2, with their chord half-width.
 * r^2 is formed in double from the float radius, which is exact. */
static stencil_pt* make_stencil(double r, int mode, int* count) {
    double r2 = r * r;
    int R = (int)floor(r);
    int cap = (2 * R + 1) * (2 * R + 1);
    stencil_pt* s = (stencil_pt*)malloc(sizeof(stencil_pt) * (size_t)(cap > 0 ? cap : 1));
    int n = 0;
    for (int dy = -R; dy <= R; ++dy)
        for (int dx = -R; dx <= R; ++dx) {
            double d2 = (double)(dx * dx + dy * dy);
            if (d2 <= r2) {
                double h = sqrt(r2 - d2);
                if (mode == ORACLE_F32_MODEL) h = (double)(float)h;
                s[n].dx = dx;
                s[n].dy = dy;
                s[n].h = h;
                ++n;
            }
        }
    *count = n;
    return s;
}

static double round_end(double v, int mode) {
    return mode == ORACLE_F32_MODEL ? (double)(float)v : v;
}

typedef struct {
    ivl* v;
    int64_t n, cap;
} ivec;

static void ivec_push(ivec* a, double lo, double hi) {
    if (a->n == a->cap) {
        a->cap = a->cap ? 2 * a->cap : 256;
        a->v = (ivl*)realloc(a->v, sizeof(ivl) * (size_t)a->cap);
    }
    a->v[a->n].lo = lo;
    a->v[a->n].hi = hi;
    a->n++;
}

/* Sort and merge in place; returns the number of merged intervals. */
static int64_t union_sorted(ivl* v, int64_t n) {
    if (n == 0) return 0;
    qsort(v, (size_t)n, sizeof(ivl), cmp_ivl);
    int64_t m = 0;
    for (int64_t i = 1; i < n; ++i) {
        if (v[i].lo <= v[m].hi) {
            if (v[i].hi > v[m].hi) v[m].hi = v[i].hi;
        } else {
            v[++m] = v[i];
        }
    }
    return m + 1;
}

/*
 * Offset of the requested columns.
 *
 * nx, ny       grid size; column id = y * nx + x
 * col_ptr      [nx*ny + 1] offsets into the interval list
 * z            [2 * col_ptr[nx*ny]] (z_in, z_out) pairs, canonical per column
 * r            ball radius (>= 0)
 * mode         ORACLE_F64 or ORACLE_F32_MODEL
 * op           ORACLE_DILATE or ORACLE_ERODE
 * ncols_req    number of requested output columns, ids in cols_req
 * out_cnt      [ncols_req] number of output intervals per requested column
 * out_z        [2 * cap] output pairs, concatenated in request order
 * Returns the total number of output intervals (written only if <= cap),
 * or -1 on bad arguments.
 */
int64_t oracle_offset(int nx, int ny, const int64_t* col_ptr, const double* z, double r,
                      int mode, int op, int64_t ncols_req, const int64_t* cols_req,
                      int64_t* out_cnt, double* out_z, int64_t cap) {
    if (nx <= 0 || ny <= 0 || !(r >= 0.0) || isinf(r)) return -1;
    int ns = 0;
    stencil_pt* st = make_stencil(r, mode, &ns);
    ivl** res = (ivl**)calloc((size_t)(ncols_req > 0 ? ncols_req : 1), sizeof(ivl*));
    int64_t total = 0;

#pragma omp parallel reduction(+ : total)
    {
        ivec cand = {0, 0, 0};
#pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < ncols_req; ++q) {
            int64_t c = cols_req[q];
            int x = (int)(c % nx), y = (int)(c / nx);
            cand.n = 0;
            for (int k = 0; k < ns; ++k) {
                int xx = x + st[k].dx, yy = y + st[k].dy;
                if (xx < 0 || xx >= nx || yy < 0 || yy >= ny) continue;
                int64_t cc = (int64_t)yy * nx + xx;
                int64_t b = col_ptr[cc], e = col_ptr[cc + 1];
                double h = st[k].h;
                if (op == ORACLE_DILATE) {
                    for (int64_t i = b; i < e; ++i)
                        ivec_push(&cand, round_end(z[2 * i] - h, mode),
                                  round_end(z[2 * i + 1] + h, mode));
                } else {
                    /* closed gaps of the in-grid column, unbounded at both ends */
                    double prev = -INFINITY;
                    for (int64_t i = b; i < e; ++i) {
                        ivec_push(&cand, round_end(prev - h, mode),
                                  round_end(z[2 * i] + h, mode));
                        prev = z[2 * i + 1];
                    }
                    ivec_push(&cand, round_end(prev - h, mode), INFINITY);
                }
            }
            int64_t m = union_sorted(cand.v, cand.n);
            ivl* out;
            int64_t k_out = 0;
            if (op == ORACLE_DILATE) {
                out = (ivl*)malloc(sizeof(ivl) * (size_t)(m > 0 ? m : 1));
                memcpy(out, cand.v, sizeof(ivl) * (size_t)m);
                k_out = m;
            } else {
                /* complement of the union; keep positive-length pieces */
                out = (ivl*)malloc(sizeof(ivl) * (size_t)(m + 1));
                double lo = -INFINITY;
                for (int64_t i = 0; i <= m; ++i) {
                    double hi = (i < m) ? cand.v[i].lo : INFINITY;
                    if (hi > lo) {
                        out[k_out].lo = lo;
                        out[k_out].hi = hi;
                        ++k_out;
                    }
                    if (i < m) lo = cand.v[i].hi;
                }
            }
            res[q] = out;
            out_cnt[q] = k_out;
            total += k_out;
        }
        free(cand.v);
    }

    if (total <= cap) {
        int64_t o = 0;
        for (int64_t q = 0; q < ncols_req; ++q) {
            for (int64_t i = 0; i < out_cnt[q]; ++i) {
                out_z[2 * o] = res[q][i].lo;
                out_z[2 * o + 1] = res[q][i].hi;
                ++o;
            }
        }
    }
    for (int64_t q = 0; q < ncols_req; ++q) free(res[q]);
    free(res);
    free(st);
    return total;
}

/* Number of OpenMP threads the oracle will use. */
int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
