/*
 * xdrop_oracle.c -- CPU oracle for seed-and-extend X-Drop alignment.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow definition that the
 * GPU library is checked against.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header or
 * constant with the HIP library, and nothing in the library may call it.
 *
 * What is computed (paper: Sec. 2.2 recurrence and X-Drop rule, Sec. 3 and
 * Algorithm 1 for the antidiagonal order, the threshold timing and the
 * termination test, Sec. 4.1.1 and 4.1.2 for the seed and the left / right
 * split):
 *
 *   Cells (x, y), 0 <= x <= m, 0 <= y <= n: x symbols of a (the query side,
 *   the paper's H) and y symbols of b (the target side, the paper's V) are
 *   consumed.  Antidiagonal d = x + y.  -inf is a separate state, never a
 *   number.
 *     S(0,0) = 0, T_0 = 0                                   (Sec. 2.2)
 *     for d = 1 .. m+n, every cell on d:
 *       R = max of the terms whose predecessor lies inside the matrix and is
 *           finite:  S(x-1,y-1) + sim(a[x-1], b[y-1]),
 *                    S(x-1,y) + gap,   S(x,y-1) + gap        (Sec. 2.2 eq.)
 *       S(x,y) = R   if R exists and R >= T_{d-1} - X,  else -inf
 *                    (pruned iff R < T - X, strict; Sec. 2.2 and Alg. 1)
 *     T_d = max(T_{d-1}, max of S over d)   (T only changes between
 *                                            antidiagonals, Alg. 1)
 *   best = T_{m+n}; end = lexicographic maximum of (S, -d, -x) over finite
 *   cells, i.e. the first cell reaching the best score in antidiagonal order,
 *   lowest x on ties (the paper is silent; this is the chosen reading).
 *   W (live-span cells) = 1 + sum over d >= 1 of |[lo_d, hi_d]| with
 *     lo_d = max(min(L_{d-1}, L_{d-2}+1), max(0, d-n))
 *     hi_d = min(max(U_{d-1}+1, U_{d-2}+1), min(m, d))
 *   where L_e / U_e are the lowest / highest x of a finite cell on e and an
 *   antidiagonal without finite cells contributes no term.  This is the span
 *   the memory-restricted band of Sec. 3 must cover so that no cell reachable
 *   through the diagonal (d-2) dependency is lost.
 *
 *   Seed (q, t, q_pos, t_pos, k) (Sec. 4.1.1, Sec. 4.3 tuple e_c):
 *     seed_score = sum_{u<k} sim(q[q_pos+u], t[t_pos+u])
 *     left  = E(reverse q[0:q_pos], reverse t[0:t_pos])   (op() read backwards)
 *     right = E(q[q_pos+k:], t[t_pos+k:])
 *     score = left + seed_score + right,
 *     q_begin = q_pos - left.x, t_begin = t_pos - left.y,
 *     q_end = q_pos + k + right.x, t_end = t_pos + k + right.y.
 *
 * Two tiers compute the same definition:
 *   xo_extend_dense : the literal (m+1)(n+1) matrix, every cell, antidiagonal
 *                     order (used for small pairs and for traceback).
 *   xo_extend_span  : every antidiagonal's [lo_d, hi_d] slice is kept (nothing
 *                     is discarded, so it is still the whole matrix: cells
 *                     outside the kept slices are -inf by the argument above).
 *                     Stops once antidiagonals d-1 and d-2 are both without a
 *                     finite cell, after which every cell is -inf.
 * Arithmetic is int64.  Parity pinning: hand-worked tables, X -> infinity
 * against a row-major textbook DP and brute-force path enumeration, closed
 * forms and invariants (see the tests).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define XO_OK 0
#define XO_E_INVALID (-1)
#define XO_E_RANGE (-2)
#define XO_E_NOMEM (-3)
#define XO_E_SYMBOL (-6)

typedef struct {
    int64_t best;   /* T at the end */
    int64_t x, y;   /* end position of the best cell */
    int64_t cells;  /* W, live-span cells */
} xo_ext;

typedef struct {
    int32_t alphabet_size;
    const int32_t *matrix; /* alphabet_size x alphabet_size, row = a symbol */
    int64_t gap;           /* added once per gap symbol (normally <= 0) */
    int64_t X;             /* X >= 0 */
} xo_scoring;

/* A cell value: 'fin' is 0 for -inf. */
typedef struct {
    int64_t v;
    int fin;
} xo_cell;

static int64_t xo_sim(const xo_scoring *sc, uint8_t ca, uint8_t cb)
{
    return (int64_t)sc->matrix[(int)ca * sc->alphabet_size + (int)cb];
}

/* Update a running maximum with a finite candidate. */
static void xo_take(xo_cell *r, int64_t cand)
{
    if (!r->fin || cand > r->v) {
        r->v = cand;
        r->fin = 1;
    }
}

static int64_t xo_min64(int64_t a, int64_t b) { return a < b ? a : b; }
static int64_t xo_max64(int64_t a, int64_t b) { return a > b ? a : b; }

/* Span [lo, hi] of antidiagonal d from the finite ranges of d-1 and d-2. */
static void xo_span(int64_t d, int64_t m, int64_t n, int alive1, int64_t L1,
                    int64_t U1, int alive2, int64_t L2, int64_t U2,
                    int64_t *lo, int64_t *hi)
{
    int64_t clo = INT64_MAX, chi = INT64_MIN;
    if (alive1) {
        clo = xo_min64(clo, L1);
        chi = xo_max64(chi, U1 + 1);
    }
    if (alive2) {
        clo = xo_min64(clo, L2 + 1);
        chi = xo_max64(chi, U2 + 1);
    }
    *lo = xo_max64(clo, xo_max64(0, d - n));
    *hi = xo_min64(chi, xo_min64(m, d));
}

/* ------------------------------------------------------------------------
 * Dense tier: the literal matrix.  out_S (optional, (m+1)*(n+1) row-major by
 * x) receives cell values and out_fin the finite flags, for traceback tests.
 * ---------------------------------------------------------------------- */
int xo_extend_dense(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n,
                    const xo_scoring *sc, xo_ext *out, int64_t *out_S,
                    uint8_t *out_fin)
{
    if (m < 0 || n < 0 || sc->X < 0)
        return XO_E_INVALID;
    int64_t cols = n + 1;
    size_t ncell = (size_t)(m + 1) * (size_t)(n + 1);
    xo_cell *S = (xo_cell *)malloc(ncell * sizeof(xo_cell));
    /* per-antidiagonal finite range, needed for W */
    int64_t *L = (int64_t *)malloc((size_t)(m + n + 1) * sizeof(int64_t));
    int64_t *U = (int64_t *)malloc((size_t)(m + n + 1) * sizeof(int64_t));
    int *alive = (int *)malloc((size_t)(m + n + 1) * sizeof(int));
    if (!S || !L || !U || !alive) {
        free(S); free(L); free(U); free(alive);
        return XO_E_NOMEM;
    }
    for (size_t i = 0; i < ncell; i++)
        S[i].fin = 0;

    S[0].v = 0;
    S[0].fin = 1;
    int64_t T = 0, bx = 0, by = 0;
    L[0] = U[0] = 0;
    alive[0] = 1;

    for (int64_t d = 1; d <= m + n; d++) {
        int64_t xlo = xo_max64(0, d - n), xhi = xo_min64(m, d);
        int64_t dmax = 0, dmax_x = -1; /* best finite cell of this d */
        alive[d] = 0;
        for (int64_t x = xlo; x <= xhi; x++) {
            int64_t y = d - x;
            xo_cell r = {0, 0};
            if (x >= 1 && y >= 1) {
                xo_cell p = S[(x - 1) * cols + (y - 1)];
                if (p.fin)
                    xo_take(&r, p.v + xo_sim(sc, a[x - 1], b[y - 1]));
            }
            if (x >= 1) {
                xo_cell p = S[(x - 1) * cols + y];
                if (p.fin)
                    xo_take(&r, p.v + sc->gap);
            }
            if (y >= 1) {
                xo_cell p = S[x * cols + (y - 1)];
                if (p.fin)
                    xo_take(&r, p.v + sc->gap);
            }
            /* X-Drop rule against the best score of the earlier antidiagonals */
            if (r.fin && !(r.v < T - sc->X)) {
                S[x * cols + y] = r;
                if (!alive[d]) {
                    alive[d] = 1;
                    L[d] = x;
                }
                U[d] = x;
                if (dmax_x < 0 || r.v > dmax) {
                    dmax = r.v;
                    dmax_x = x;
                }
            }
        }
        if (dmax_x >= 0 && dmax > T) { /* strict: earliest d wins ties */
            T = dmax;
            bx = dmax_x;
            by = d - dmax_x;
        }
    }

    int64_t W = 1;
    for (int64_t d = 1; d <= m + n; d++) {
        int64_t lo, hi;
        int a2 = d >= 2 ? alive[d - 2] : 0;
        xo_span(d, m, n, alive[d - 1], L[d - 1], U[d - 1], a2,
                d >= 2 ? L[d - 2] : 0, d >= 2 ? U[d - 2] : 0, &lo, &hi);
        if (lo <= hi)
            W += hi - lo + 1;
    }

    out->best = T;
    out->x = bx;
    out->y = by;
    out->cells = W;
    if (out_S && out_fin) {
        for (size_t i = 0; i < ncell; i++) {
            out_S[i] = S[i].fin ? S[i].v : 0;
            out_fin[i] = (uint8_t)S[i].fin;
        }
    }
    free(S); free(L); free(U); free(alive);
    return XO_OK;
}

/* ------------------------------------------------------------------------
 * Span tier: keeps the [lo_d, hi_d] slice of every antidiagonal.
 * ---------------------------------------------------------------------- */
typedef struct {
    int64_t lo, hi;  /* kept slice (lo > hi: empty) */
    int64_t off;     /* start of the slice in the value store */
    int alive;
    int64_t L, U;    /* finite range */
} xo_diag;

/* Value of cell (x, d-x) from the kept slices; -inf outside them. */
static xo_cell xo_get(const xo_diag *D, const xo_cell *store, int64_t d,
                      int64_t x)
{
    xo_cell none = {0, 0};
    if (d < 0)
        return none;
    const xo_diag *e = &D[d];
    if (x < e->lo || x > e->hi)
        return none;
    return store[e->off + (x - e->lo)];
}

/* widths (optional, m+n+1 entries): hi_d - lo_d + 1 per antidiagonal, 0 when
 * empty -- the working band of Sec. 6.1.  finite (optional, 2*(m+n+1)
 * entries): L_d, U_d per antidiagonal, -1, -1 when it holds no finite cell. */
int xo_extend_span(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n,
                   const xo_scoring *sc, xo_ext *out, int32_t *widths,
                   int64_t *finite)
{
    if (m < 0 || n < 0 || sc->X < 0)
        return XO_E_INVALID;
    int64_t nd = m + n + 1;
    xo_diag *D = (xo_diag *)calloc((size_t)nd, sizeof(xo_diag));
    size_t cap = 1024, used = 0;
    xo_cell *store = (xo_cell *)malloc(cap * sizeof(xo_cell));
    if (!D || !store) {
        free(D); free(store);
        return XO_E_NOMEM;
    }
    D[0].lo = D[0].hi = 0;
    D[0].off = 0;
    D[0].alive = 1;
    D[0].L = D[0].U = 0;
    store[0].v = 0;
    store[0].fin = 1;
    used = 1;
    if (widths) {
        widths[0] = 1;
        for (int64_t d = 1; d < nd; d++)
            widths[d] = 0;
    }
    if (finite) {
        finite[0] = finite[1] = 0;
        for (int64_t d = 1; d < nd; d++)
            finite[2 * d] = finite[2 * d + 1] = -1;
    }

    int64_t T = 0, bx = 0, by = 0, W = 1;
    for (int64_t d = 1; d <= m + n; d++) {
        xo_diag *e = &D[d];
        int a1 = D[d - 1].alive, a2 = d >= 2 ? D[d - 2].alive : 0;
        if (!a1 && !a2) { /* every later cell is -inf */
            for (int64_t r = d; r <= m + n; r++) {
                D[r].lo = 1;
                D[r].hi = 0;
            }
            break;
        }
        xo_span(d, m, n, a1, D[d - 1].L, D[d - 1].U, a2,
                a2 ? D[d - 2].L : 0, a2 ? D[d - 2].U : 0, &e->lo, &e->hi);
        e->alive = 0;
        if (e->lo > e->hi) {
            e->off = (int64_t)used;
            continue;
        }
        int64_t len = e->hi - e->lo + 1;
        W += len;
        if (widths)
            widths[d] = (int32_t)len;
        if (used + (size_t)len > cap) {
            while (used + (size_t)len > cap)
                cap *= 2;
            xo_cell *ns = (xo_cell *)realloc(store, cap * sizeof(xo_cell));
            if (!ns) {
                free(D); free(store);
                return XO_E_NOMEM;
            }
            store = ns;
        }
        e->off = (int64_t)used;
        int64_t dmax = 0, dmax_x = -1;
        for (int64_t x = e->lo; x <= e->hi; x++) {
            int64_t y = d - x;
            xo_cell r = {0, 0};
            if (x >= 1 && y >= 1) {
                xo_cell p = xo_get(D, store, d - 2, x - 1);
                if (p.fin)
                    xo_take(&r, p.v + xo_sim(sc, a[x - 1], b[y - 1]));
            }
            if (x >= 1) {
                xo_cell p = xo_get(D, store, d - 1, x - 1);
                if (p.fin)
                    xo_take(&r, p.v + sc->gap);
            }
            if (y >= 1) {
                xo_cell p = xo_get(D, store, d - 1, x);
                if (p.fin)
                    xo_take(&r, p.v + sc->gap);
            }
            xo_cell s = {0, 0};
            if (r.fin && !(r.v < T - sc->X)) {
                s = r;
                if (!e->alive) {
                    e->alive = 1;
                    e->L = x;
                }
                e->U = x;
                if (dmax_x < 0 || r.v > dmax) {
                    dmax = r.v;
                    dmax_x = x;
                }
            }
            store[used + (size_t)(x - e->lo)] = s;
        }
        used += (size_t)len;
        if (finite && e->alive) {
            finite[2 * d] = e->L;
            finite[2 * d + 1] = e->U;
        }
        if (dmax_x >= 0 && dmax > T) {
            T = dmax;
            bx = dmax_x;
            by = d - dmax_x;
        }
    }
    out->best = T;
    out->x = bx;
    out->y = by;
    out->cells = W;
    free(D);
    free(store);
    return XO_OK;
}

/* ------------------------------------------------------------------------
 * Seed level and batch.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t q, t;
    int32_t q_pos, t_pos, k;
} xo_seed;

typedef struct {
    int64_t score, left, right, seed_score;
    int64_t q_begin, q_end, t_begin, t_end;
    int64_t cells;
    int64_t status;
} xo_seed_result;

/* dense_limit: pairs with (m+1)(n+1) <= dense_limit use the dense tier. */
static int xo_run(const uint8_t *a, int64_t m, const uint8_t *b, int64_t n,
                  const xo_scoring *sc, int64_t dense_limit, xo_ext *e)
{
    if ((m + 1) * (n + 1) <= dense_limit)
        return xo_extend_dense(a, m, b, n, sc, e, NULL, NULL);
    return xo_extend_span(a, m, b, n, sc, e, NULL, NULL);
}

int xo_seed_extend(const uint8_t *q, int64_t qlen, const uint8_t *t,
                   int64_t tlen, int64_t q_pos, int64_t t_pos, int64_t k,
                   const xo_scoring *sc, int64_t dense_limit,
                   xo_seed_result *r)
{
    memset(r, 0, sizeof(*r));
    if (k < 0 || q_pos < 0 || t_pos < 0 || q_pos + k > qlen ||
        t_pos + k > tlen) {
        r->status = XO_E_RANGE;
        return XO_OK;
    }
    for (int64_t i = 0; i < qlen; i++)
        if (q[i] >= sc->alphabet_size) {
            r->status = XO_E_SYMBOL;
            return XO_OK;
        }
    for (int64_t i = 0; i < tlen; i++)
        if (t[i] >= sc->alphabet_size) {
            r->status = XO_E_SYMBOL;
            return XO_OK;
        }
    int64_t seed = 0;
    for (int64_t u = 0; u < k; u++)
        seed += xo_sim(sc, q[q_pos + u], t[t_pos + u]);

    /* left extension: both prefixes read backwards */
    uint8_t *la = (uint8_t *)malloc((size_t)q_pos + 1);
    uint8_t *lb = (uint8_t *)malloc((size_t)t_pos + 1);
    if (!la || !lb) {
        free(la); free(lb);
        return XO_E_NOMEM;
    }
    for (int64_t i = 0; i < q_pos; i++)
        la[i] = q[q_pos - 1 - i];
    for (int64_t j = 0; j < t_pos; j++)
        lb[j] = t[t_pos - 1 - j];
    xo_ext L, R;
    int rc = xo_run(la, q_pos, lb, t_pos, sc, dense_limit, &L);
    free(la);
    free(lb);
    if (rc != XO_OK)
        return rc;
    rc = xo_run(q + q_pos + k, qlen - q_pos - k, t + t_pos + k,
                tlen - t_pos - k, sc, dense_limit, &R);
    if (rc != XO_OK)
        return rc;
    r->left = L.best;
    r->right = R.best;
    r->seed_score = seed;
    r->score = L.best + seed + R.best;
    r->q_begin = q_pos - L.x;
    r->t_begin = t_pos - L.y;
    r->q_end = q_pos + k + R.x;
    r->t_end = t_pos + k + R.y;
    r->cells = L.cells + R.cells;
    r->status = XO_OK;
    return XO_OK;
}

/* Batch over seeds.  seqs: one code per byte; offsets: n_seqs+1 entries.
 * Returns the number of worker threads used in *threads_used. */
#ifdef _OPENMP
#include <omp.h>
#endif
int xo_batch(const uint8_t *seqs, const int64_t *offsets, int64_t n_seqs,
             const xo_seed *seeds, int64_t n_seeds, const xo_scoring *sc,
             int64_t dense_limit, int32_t n_threads, xo_seed_result *out,
             int32_t *threads_used)
{
    int err = XO_OK;
    int used = 1;
#ifdef _OPENMP
    if (n_threads > 0)
        omp_set_num_threads(n_threads);
#pragma omp parallel
    {
#pragma omp single
        used = omp_get_num_threads();
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < n_seeds; s++) {
            const xo_seed *sd = &seeds[s];
            if (sd->q < 0 || sd->q >= n_seqs || sd->t < 0 || sd->t >= n_seqs) {
                memset(&out[s], 0, sizeof(out[s]));
                out[s].status = XO_E_RANGE;
                continue;
            }
            int rc = xo_seed_extend(seqs + offsets[sd->q],
                                    offsets[sd->q + 1] - offsets[sd->q],
                                    seqs + offsets[sd->t],
                                    offsets[sd->t + 1] - offsets[sd->t],
                                    sd->q_pos, sd->t_pos, sd->k, sc,
                                    dense_limit, &out[s]);
            if (rc != XO_OK) {
#pragma omp critical
                err = rc;
            }
        }
    }
#else
    (void)n_threads;
    for (int64_t s = 0; s < n_seeds; s++) {
        const xo_seed *sd = &seeds[s];
        if (sd->q < 0 || sd->q >= n_seqs || sd->t < 0 || sd->t >= n_seqs) {
            memset(&out[s], 0, sizeof(out[s]));
            out[s].status = XO_E_RANGE;
            continue;
        }
        int rc = xo_seed_extend(seqs + offsets[sd->q],
                                offsets[sd->q + 1] - offsets[sd->q],
                                seqs + offsets[sd->t],
                                offsets[sd->t + 1] - offsets[sd->t], sd->q_pos,
                                sd->t_pos, sd->k, sc, dense_limit, &out[s]);
        if (rc != XO_OK)
            err = rc;
    }
#endif
    if (threads_used)
        *threads_used = used;
    return err;
}
