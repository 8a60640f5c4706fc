/*
 * oracle.c -- plain, slow, obviously correct CPU oracle for the Euclidean
 * epsilon self-join (Gowanlock & Karsin, "GPU Accelerated Similarity
 * Self-Join for Multi-Dimensional Data").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header, table or constant with
 * the HIP library.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 * (no FMA contraction: every multiply and add below is a separately rounded
 * IEEE-754 binary64 operation).
 *
 * The canonical predicate (Section 3.1, problem statement): points a and b are
 * a result pair when dist(a,b) <= eps, dist being the L2 norm over all n
 * dimensions.  Written in squared form in binary64:
 *     eps2 = eps * eps                                (one rounding)
 *     acc  = sum over t = 0..d-1, in ORIGINAL dimension order, of
 *            diff_t * diff_t with diff_t = (double)a_t - (double)b_t
 *     pair iff acc <= eps2
 * The result holds ordered tuples (a, b), a and b both in D, so it contains
 * every (i, i) and both (i, j) and (j, i) (Section 3.1; the selectivity
 * equation of Section 5.2 subtracts |D| self pairs from |R|).
 */
#define _GNU_SOURCE /* qsort_r: comparators take their context as an argument */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif


/* Canonical squared distance (Section 3.1), original dimension order. */
static double canon_sq(const float *a, const float *b, uint32_t d)
{
    double acc = 0.0;
    for (uint32_t t = 0; t < d; ++t) {
        double diff = (double)a[t] - (double)b[t];
        double sq = diff * diff;
        acc = acc + sq;
    }
    return acc;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------------
 * O1: nested-loop join over all ordered pairs (Section 3.1: the O(|D|^2)
 * nested loop).  Pass 1 counts per query row, pass 2 fills; output is in
 * ascending (i, j) order.  Returns |R|, or -1 when cap is too small (counts
 * are still written to row_counts when non-NULL).
 * ------------------------------------------------------------------------- */
int64_t oracle_bruteforce(const float *P, uint64_t n, uint32_t d, double eps,
                          uint64_t *row_counts, uint32_t *out_i,
                          uint32_t *out_j, double *out_s, uint64_t cap)
{
    const double eps2 = eps * eps;
    uint64_t *cnt = (uint64_t *)calloc(n ? n : 1, sizeof(uint64_t));
    if (!cnt) return -2;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        uint64_t c = 0;
        for (uint64_t j = 0; j < n; ++j)
            if (canon_sq(P + (uint64_t)i * d, P + j * d, d) <= eps2) ++c;
        cnt[i] = c;
    }
    uint64_t total = 0;
    for (uint64_t i = 0; i < n; ++i) {
        if (row_counts) row_counts[i] = cnt[i];
        uint64_t c = cnt[i];
        cnt[i] = total;
        total += c;
    }
    if (out_j == NULL) { free(cnt); return (int64_t)total; }
    if (total > cap) { free(cnt); return -1; }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < (int64_t)n; ++i) {
        uint64_t w = cnt[i];
        for (uint64_t j = 0; j < n; ++j) {
            double s = canon_sq(P + (uint64_t)i * d, P + j * d, d);
            if (s <= eps2) {
                if (out_i) out_i[w] = (uint32_t)i;
                out_j[w] = (uint32_t)j;
                if (out_s) out_s[w] = s;
                ++w;
            }
        }
    }
    free(cnt);
    return (int64_t)total;
}

/* ---------------------------------------------------------------------------
 * O1q: the general similarity join Q join_eps E of Section 3.1 (the self-join
 * is the case Q = E): every pair (q, e), q a row of Q and e a row of E, with
 * the canonical squared distance <= fl(eps*eps), nested loops over all m*n
 * pairs, output in ascending (q, e) order.  Same count/fill passes and
 * return convention as O1.
 * ------------------------------------------------------------------------- */
int64_t oracle_join(const float *Q, uint64_t m, const float *E, uint64_t n,
                    uint32_t d, double eps, uint64_t *row_counts,
                    uint32_t *out_i, uint32_t *out_j, double *out_s,
                    uint64_t cap)
{
    const double eps2 = eps * eps;
    uint64_t *cnt = (uint64_t *)calloc(m ? m : 1, sizeof(uint64_t));
    if (!cnt) return -2;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < (int64_t)m; ++q) {
        uint64_t c = 0;
        for (uint64_t e = 0; e < n; ++e)
            if (canon_sq(Q + (uint64_t)q * d, E + e * d, d) <= eps2) ++c;
        cnt[q] = c;
    }
    uint64_t total = 0;
    for (uint64_t q = 0; q < m; ++q) {
        if (row_counts) row_counts[q] = cnt[q];
        uint64_t c = cnt[q];
        cnt[q] = total;
        total += c;
    }
    if (out_j == NULL) { free(cnt); return (int64_t)total; }
    if (total > cap) { free(cnt); return -1; }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < (int64_t)m; ++q) {
        uint64_t w = cnt[q];
        for (uint64_t e = 0; e < n; ++e) {
            double s = canon_sq(Q + (uint64_t)q * d, E + e * d, d);
            if (s <= eps2) {
                if (out_i) out_i[w] = (uint32_t)q;
                out_j[w] = (uint32_t)e;
                if (out_s) out_s[w] = s;
                ++w;
            }
        }
    }
    free(cnt);
    return (int64_t)total;
}

/* O1 restricted to a list of query rows: the full row of each listed query
 * (all j in ascending order).  Same predicate and ordering as above. */
int64_t oracle_rows(const float *P, uint64_t n, uint32_t d, double eps,
                    const uint64_t *rows, uint64_t nrows, uint64_t *row_counts,
                    uint32_t *out_j, double *out_s, uint64_t cap)
{
    const double eps2 = eps * eps;
    uint64_t *cnt = (uint64_t *)calloc(nrows ? nrows : 1, sizeof(uint64_t));
    if (!cnt) return -2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < (int64_t)nrows; ++r) {
        const float *q = P + rows[r] * d;
        uint64_t c = 0;
        for (uint64_t j = 0; j < n; ++j)
            if (canon_sq(q, P + j * d, d) <= eps2) ++c;
        cnt[r] = c;
    }
    uint64_t total = 0;
    for (uint64_t r = 0; r < nrows; ++r) {
        if (row_counts) row_counts[r] = cnt[r];
        uint64_t c = cnt[r];
        cnt[r] = total;
        total += c;
    }
    if (out_j == NULL) { free(cnt); return (int64_t)total; }
    if (total > cap) { free(cnt); return -1; }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < (int64_t)nrows; ++r) {
        const float *q = P + rows[r] * d;
        uint64_t w = cnt[r];
        for (uint64_t j = 0; j < n; ++j) {
            double s = canon_sq(q, P + j * d, d);
            if (s <= eps2) {
                out_j[w] = (uint32_t)j;
                if (out_s) out_s[w] = s;
                ++w;
            }
        }
    }
    free(cnt);
    return (int64_t)total;
}

/* For each listed row, the K smallest canonical squared distances to the
 * other points (self index excluded), ascending.  Used only to calibrate
 * eps for a target selectivity S_D (Section 5.2). Rows with fewer than K
 * other points are padded with +inf. */
int oracle_rows_smallest(const float *P, uint64_t n, uint32_t d,
                         const uint64_t *rows, uint64_t nrows, uint32_t K,
                         double *out)
{
    if (K == 0) return 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < (int64_t)nrows; ++r) {
        double *heap = out + (uint64_t)r * K; /* max-heap of the K smallest */
        uint32_t hs = 0;
        const uint64_t qi = rows[r];
        const float *q = P + qi * d;
        for (uint64_t j = 0; j < n; ++j) {
            if (j == qi) continue;
            double s = canon_sq(q, P + j * d, d);
            if (hs < K) {
                uint32_t c = hs++;
                heap[c] = s;
                while (c > 0) {
                    uint32_t p = (c - 1) / 2;
                    if (heap[p] >= heap[c]) break;
                    double t = heap[p]; heap[p] = heap[c]; heap[c] = t;
                    c = p;
                }
            } else if (s < heap[0]) {
                heap[0] = s;
                uint32_t c = 0;
                for (;;) {
                    uint32_t l = 2 * c + 1, rr = l + 1, m = c;
                    if (l < hs && heap[l] > heap[m]) m = l;
                    if (rr < hs && heap[rr] > heap[m]) m = rr;
                    if (m == c) break;
                    double t = heap[m]; heap[m] = heap[c]; heap[c] = t;
                    c = m;
                }
            }
        }
        for (uint32_t c = hs; c < K; ++c) heap[c] = INFINITY;
        /* heap-sort ascending in place */
        for (uint32_t end = hs; end > 1; --end) {
            double t = heap[0]; heap[0] = heap[end - 1]; heap[end - 1] = t;
            uint32_t lim = end - 1, c = 0;
            for (;;) {
                uint32_t l = 2 * c + 1, rr = l + 1, m = c;
                if (l < lim && heap[l] > heap[m]) m = l;
                if (rr < lim && heap[rr] > heap[m]) m = rr;
                if (m == c) break;
                double tt = heap[m]; heap[m] = heap[c]; heap[c] = tt;
                c = m;
            }
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * O2: CPU grid variant (Section 3.2.1 grid index; Section 4.1 indexing only
 * k of the n dimensions; Algorithm 1's SelfJoinKernel loop over adjacent
 * cells, one query point at a time).
 *
 * Cells have side w = eps * width_factor over the k dimensions listed in
 * `dims`; the cell coordinate of x along dimension r is
 * floor((x - origin_r) / w), origin_r = 0 when origin_zero != 0 (the paper's
 * illustrative convention) else the minimum of dimension r.  For each query
 * the 3^k cells around its own cell are looked up by binary search over the
 * sorted non-empty cells, and every point of each found cell is tested with
 * the canonical predicate over ALL d dimensions in original order.
 * Output is in ascending (i, j) order.  *n_candidates receives the number of
 * ordered candidate pairs tested (the sum over queries of the sizes of the
 * adjacent non-empty cells).
 * ------------------------------------------------------------------------- */
typedef struct {
    const int64_t *coord; /* [n][k] cell coordinates */
    uint32_t k;
} grid_ctx;

static int cmp_coord(const int64_t *a, const int64_t *b, uint32_t k)
{
    for (uint32_t r = 0; r < k; ++r) {
        if (a[r] < b[r]) return -1;
        if (a[r] > b[r]) return 1;
    }
    return 0;
}

static int cmp_point(const void *pa, const void *pb, void *arg)
{
    const grid_ctx *g = (const grid_ctx *)arg;
    uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    int c = cmp_coord(g->coord + (uint64_t)a * g->k, g->coord + (uint64_t)b * g->k, g->k);
    if (c) return c;
    return (a > b) - (a < b);
}

static int cmp_u32(const void *pa, const void *pb)
{
    uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    return (a > b) - (a < b);
}

/* Cell coordinates of every point (exposed for the Figure 1 / Figure 2 pins). */
int oracle_cell_coords(const float *P, uint64_t n, uint32_t d, double eps,
                       uint32_t k, const uint32_t *dims, int origin_zero,
                       double width_factor, int64_t *coord)
{
    const double w = eps * width_factor;
    for (uint32_t r = 0; r < k; ++r) {
        const uint32_t t = dims[r];
        double org = 0.0;
        if (!origin_zero) {
            org = INFINITY;
            for (uint64_t i = 0; i < n; ++i)
                if ((double)P[i * d + t] < org) org = (double)P[i * d + t];
        }
        for (uint64_t i = 0; i < n; ++i)
            coord[i * k + r] = (int64_t)floor(((double)P[i * d + t] - org) / w);
    }
    return 0;
}

int64_t oracle_grid(const float *P, uint64_t n, uint32_t d, double eps,
                    uint32_t k, const uint32_t *dims, int origin_zero,
                    double width_factor, uint32_t *out_i, uint32_t *out_j,
                    uint64_t cap, uint64_t *n_candidates)
{
    const double eps2 = eps * eps;
    if (n_candidates) *n_candidates = 0;
    if (n == 0) return 0;
    if (k == 0 || k > 20) return -3;
    int64_t *coord = (int64_t *)malloc(n * k * sizeof(int64_t));
    uint32_t *order = (uint32_t *)malloc(n * sizeof(uint32_t));
    uint64_t *rowcnt = (uint64_t *)calloc(n, sizeof(uint64_t));
    uint64_t *offs = (uint64_t *)calloc(n, sizeof(uint64_t));
    uint64_t *cand = (uint64_t *)calloc(n, sizeof(uint64_t));
    uint64_t *cstart = (uint64_t *)malloc((n + 1) * sizeof(uint64_t));
    if (!coord || !order || !rowcnt || !offs || !cand || !cstart) {
        free(coord); free(order); free(rowcnt); free(offs); free(cand); free(cstart);
        return -2;
    }
    oracle_cell_coords(P, n, d, eps, k, dims, origin_zero, width_factor, coord);

    /* points grouped by cell: sort by coordinate vector (lookup array) */
    for (uint64_t i = 0; i < n; ++i) order[i] = (uint32_t)i;
    grid_ctx ctx = {coord, k};
    qsort_r(order, n, sizeof(uint32_t), cmp_point, &ctx);

    /* non-empty cells: first position of each distinct coordinate vector */
    uint64_t ncell = 0;
    for (uint64_t p = 0; p < n; ++p) {
        if (p == 0 || cmp_coord(coord + (uint64_t)order[p] * k,
                                coord + (uint64_t)order[p - 1] * k, k) != 0)
            cstart[ncell++] = p;
    }
    cstart[ncell] = n;

    uint64_t n_off = 1;
    for (uint32_t r = 0; r < k; ++r) n_off *= 3;

    int64_t result = 0;
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            uint64_t total = 0, c_all = 0;
            for (uint64_t i = 0; i < n; ++i) {
                offs[i] = total;
                total += rowcnt[i];
                c_all += cand[i];
            }
            if (n_candidates) *n_candidates = c_all;
            result = (int64_t)total;
            if (out_j == NULL) break;
            if (total > cap) { result = -1; break; }
        }
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = 0; i < (int64_t)n; ++i) {
            int64_t nb[20];
            uint64_t c = 0, tested = 0, w = offs[i];
            const int64_t *ci = coord + (uint64_t)i * k;
            for (uint64_t o = 0; o < n_off; ++o) {
                uint64_t rem = o; /* radix-3 digit r gives offset digit - 1 */
                for (uint32_t r = 0; r < k; ++r) {
                    nb[r] = ci[r] + (int64_t)(rem % 3) - 1;
                    rem /= 3;
                }
                /* binary search for the neighbour cell among non-empty cells */
                uint64_t lo = 0, hi = ncell;
                while (lo < hi) {
                    uint64_t mid = lo + (hi - lo) / 2;
                    const int64_t *cm = coord + (uint64_t)order[cstart[mid]] * k;
                    if (cmp_coord(cm, nb, k) < 0) lo = mid + 1; else hi = mid;
                }
                if (lo == ncell ||
                    cmp_coord(coord + (uint64_t)order[cstart[lo]] * k, nb, k) != 0)
                    continue;
                for (uint64_t p = cstart[lo]; p < cstart[lo + 1]; ++p) {
                    uint32_t j = order[p];
                    ++tested;
                    if (canon_sq(P + (uint64_t)i * d, P + (uint64_t)j * d, d) <= eps2) {
                        if (pass == 1) out_j[w++] = j;
                        else ++c;
                    }
                }
            }
            if (pass == 0) {
                rowcnt[i] = c;
                cand[i] = tested;
            } else {
                qsort(out_j + offs[i], w - offs[i], sizeof(uint32_t), cmp_u32);
                if (out_i)
                    for (uint64_t q = offs[i]; q < w; ++q) out_i[q] = (uint32_t)i;
            }
        }
    }
    free(coord); free(order); free(rowcnt); free(offs); free(cand); free(cstart);
    return result;
}

/* Candidate points the grid search of O2 visits for one query point
 * (Algorithm 1, getAdjCells plus the loop over the adjacent cells): all
 * points of the non-empty cells among the 3^k cells around the query's cell.
 * Writes up to cap point ids, returns how many there are (ascending by cell,
 * then by id). */
int64_t oracle_grid_candidates(const float *P, uint64_t n, uint32_t d,
                               double eps, uint32_t k, const uint32_t *dims,
                               int origin_zero, double width_factor,
                               uint64_t query, uint32_t *out_j, uint64_t cap)
{
    if (k == 0 || k > 20 || query >= n) return -3;
    int64_t *coord = (int64_t *)malloc(n * k * sizeof(int64_t));
    if (!coord) return -2;
    oracle_cell_coords(P, n, d, eps, k, dims, origin_zero, width_factor, coord);
    const int64_t *cq = coord + query * k;
    uint64_t w = 0;
    /* a point is a candidate iff every indexed coordinate is within one cell
     * of the query's; listing by offset vector then id keeps the cell order */
    uint64_t n_off = 1;
    for (uint32_t r = 0; r < k; ++r) n_off *= 3;
    for (uint64_t o = 0; o < n_off; ++o) {
        int64_t nb[20];
        uint64_t rem = o;
        for (uint32_t r = 0; r < k; ++r) { nb[r] = cq[r] + (int64_t)(rem % 3) - 1; rem /= 3; }
        for (uint64_t j = 0; j < n; ++j)
            if (cmp_coord(coord + j * k, nb, k) == 0) {
                if (w < cap) out_j[w] = (uint32_t)j;
                ++w;
            }
    }
    free(coord);
    return (int64_t)w;
}

/* ---------------------------------------------------------------------------
 * SORTIDU (Section 4.3): the candidates one query visits when the points of
 * every cell are sorted by an un-indexed dimension u.  For each adjacent
 * cell (Algorithm 1's 3^k box, as in oracle_grid_candidates): the cell's
 * points are sorted by increasing u (ties by id); a binary search finds the
 * first point r whose u is within eps of the query's, |p(u) - r(u)| <= eps,
 * and the scan runs from r until the first point s with |p(u) - s(u)| > eps.
 * Differences are taken in binary64.  Output: cells in offset order, points
 * in increasing u inside each cell.  Returns the count (-1 when cap is too
 * small, counts still exact; -2 no memory; -3 bad arguments).
 * ------------------------------------------------------------------------- */
typedef struct {
    const float *P;
    uint32_t d, u;
} u_ctx;

static int cmp_by_u(const void *pa, const void *pb, void *arg)
{
    const u_ctx *c = (const u_ctx *)arg;
    const uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    const float ua = c->P[(uint64_t)a * c->d + c->u];
    const float ub = c->P[(uint64_t)b * c->d + c->u];
    if (ua < ub) return -1;
    if (ua > ub) return 1;
    return (a > b) - (a < b);
}

int64_t oracle_sortidu_candidates(const float *P, uint64_t n, uint32_t d,
                                  double eps, uint32_t k, const uint32_t *dims,
                                  int origin_zero, double width_factor,
                                  uint32_t u, uint64_t query, uint32_t *out_j,
                                  uint64_t cap)
{
    if (k == 0 || k > 20 || query >= n || u >= d) return -3;
    int64_t *coord = (int64_t *)malloc(n * k * sizeof(int64_t));
    uint32_t *cell = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    if (!coord || !cell) { free(coord); free(cell); return -2; }
    oracle_cell_coords(P, n, d, eps, k, dims, origin_zero, width_factor, coord);
    const int64_t *cq = coord + query * k;
    const double pu = (double)P[query * d + u];
    uint64_t n_off = 1, w = 0;
    for (uint32_t r = 0; r < k; ++r) n_off *= 3;
    u_ctx uctx = {P, d, u};
    for (uint64_t o = 0; o < n_off; ++o) {
        int64_t nb[20];
        uint64_t rem = o;
        for (uint32_t r = 0; r < k; ++r) { nb[r] = cq[r] + (int64_t)(rem % 3) - 1; rem /= 3; }
        /* the cell's points, sorted by u */
        uint64_t m = 0;
        for (uint64_t j = 0; j < n; ++j)
            if (cmp_coord(coord + j * k, nb, k) == 0) cell[m++] = (uint32_t)j;
        qsort_r(cell, m, sizeof(uint32_t), cmp_by_u, &uctx);
        /* r: first point with u >= p(u) - eps, i.e. the smallest u within eps */
        uint64_t lo = 0, hi = m;
        while (lo < hi) {
            const uint64_t mid = (lo + hi) / 2;
            const double cu = (double)P[(uint64_t)cell[mid] * d + u];
            if (pu - cu > eps) lo = mid + 1; else hi = mid;
        }
        /* scan from r until s, the first point farther than eps along u */
        for (uint64_t i = lo; i < m; ++i) {
            const double cu = (double)P[(uint64_t)cell[i] * d + u];
            if (fabs(pu - cu) > eps) break;
            if (w < cap) out_j[w] = cell[i];
            ++w;
        }
    }
    free(coord);
    free(cell);
    if (out_j && w > cap) return -1;
    return (int64_t)w;
}
