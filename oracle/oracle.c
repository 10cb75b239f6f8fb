/*
 * oracle.c -- plain, slow reference implementation of the APRIL
 * intermediate filter (Georgiadis, Tzirita Zacharatou, Mamoulis:
 * "Raster Interval Object Approximations for Spatial Intersection Joins").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or table with the GPU library; both only read the same seeded
 * synthetic inputs.
 *
 * What it computes, step by step, each in the most direct form:
 *
 *  grid      A 2^N x 2^N grid over the square data space (Sec. 3.1).  All
 *            coordinates are multiples of 2^-30; they are converted to
 *            integer lattice units relative to the grid origin, and every
 *            predicate below is evaluated exactly in 128-bit integers.
 *            Cell (i, j) (i = column along x, j = row along y) is the
 *            closed square [iW, (i+1)W] x [jW, (j+1)W].
 *
 *  classify  Sec. 4.1 splits cells into Full / Partial / Empty by how much
 *            of the cell the polygon covers.  Read with closed sets (so that
 *            polygons that only touch still share a cell):
 *              Empty   : the closed cell does not meet the closed polygon;
 *              Full    : the closed cell lies inside the closed polygon;
 *              Partial : anything else.
 *            Decided per cell by brute force: an edge meeting the open cell
 *            makes it Partial; otherwise the cell centre's side decides
 *            (inside -> Full; outside -> Partial if an edge meets the closed
 *            cell, else Empty).  Only edges whose y-range meets the cell's
 *            row, and whose x-range meets the cell's column, are tested (the
 *            others cannot meet the cell; only edges spanning the row's
 *            centre line can cross the centre's ray).
 *
 *  hilbert   Cells are numbered along the Hilbert curve (Sec. 3.2), the
 *            textbook quadrant-by-quadrant rotate/reflect conversion.
 *            Order 1: (0,0)->0, (0,1)->1, (1,1)->2, (1,0)->3.
 *
 *  lists     The A-list holds all Partial and Full cells, the F-list the
 *            Full cells; ids are sorted and runs of consecutive ids merged
 *            into maximal half-open intervals [start, end) (Sec. 3.2, 4.1).
 *
 *  filter    Alg. 2: IntervalJoin(A(r),A(s)) false -> true negative;
 *            IntervalJoin(A(r),F(s)) or IntervalJoin(F(r),A(s)) true ->
 *            true hit; otherwise indecisive.  IntervalJoin is the merge
 *            loop of Alg. 2: compare the heads, stop on an overlap, else
 *            advance the list whose head ends first (X on ties).  The loop
 *            also records how many leading elements of each list it read.
 *
 *  mbr join  All pairs whose closed bounding rectangles intersect (the
 *            candidate pairs the MBR filter hands to the intermediate
 *            filter, Sec. 2).
 *
 *  exact     Exact polygon intersection (closed sets): two simple polygons
 *            share a point iff two of their edges meet or one contains a
 *            vertex of the other.  Used only to check the oracle's own true
 *            hits and true negatives.
 */
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

#define ORC_OK 0
#define ORC_E_INVALID -1
#define ORC_E_GRID -2
#define ORC_E_NOMEM -3

/* ------------------------------------------------------------------ grid */

typedef struct {
    double x0, y0;
    int64_t W;      /* cell side in lattice units */
    int order;
    int64_t n;      /* cells per side */
} grid_t;

static int make_grid(double x0, double y0, double side, int order, grid_t *g)
{
    if (order < 1 || order > 16) return ORC_E_INVALID;
    double sl = side * 1073741824.0;              /* side in lattice units */
    int64_t cells = (int64_t)1 << order;
    int64_t W = (int64_t)(sl / (double)cells);
    if (W < 1 || (double)(W * cells) != sl) return ORC_E_GRID;
    g->x0 = x0; g->y0 = y0; g->W = W; g->order = order; g->n = cells;
    return ORC_OK;
}

/* exact lattice coordinate of v relative to origin o (both multiples of 2^-30) */
static int lattice(double v, double o, int64_t *out)
{
    double d = (v - o) * 1073741824.0;
    if (!(d > -9.0e15 && d < 9.0e15)) return ORC_E_GRID;
    int64_t q = (int64_t)d;
    if ((double)q != d) return ORC_E_INVALID;     /* not on the lattice */
    *out = q;
    return ORC_OK;
}

/* ------------------------------------------------------------- predicates */

/* a/b compared with c/d, b > 0, d > 0: returns -1, 0, +1 */
static int frac_cmp(i128 a, i128 b, i128 c, i128 d)
{
    i128 l = a * d, r = c * b;
    return (l < r) ? -1 : (l > r) ? 1 : 0;
}

/*
 * Does the segment p->q meet the box [bx0,bx1] x [by0,by1]?
 * open == 0: closed box; open == 1: open box (interior only).
 * Parametric form p + t (q - p), t in [0,1]; every axis constraint bounds t
 * from below and above; the set of admissible t is non-empty iff the largest
 * lower bound is below (closed box: not above) the smallest upper bound.
 * For the open box every axis bound is strict and 0 < 1, so strict
 * comparison is exact there.
 */
static int seg_meets_box(int64_t px, int64_t py, int64_t qx, int64_t qy,
                         int64_t bx0, int64_t by0, int64_t bx1, int64_t by1, int open)
{
    i128 ln = 0, ld = 1;   /* lower bound of t: ln/ld */
    i128 un = 1, ud = 1;   /* upper bound of t: un/ud */
    int64_t p[2] = {px, py}, d[2] = {qx - px, qy - py};
    int64_t lo[2] = {bx0, by0}, hi[2] = {bx1, by1};
    for (int k = 0; k < 2; k++) {
        if (d[k] == 0) {
            if (open) { if (!(lo[k] < p[k] && p[k] < hi[k])) return 0; }
            else      { if (!(lo[k] <= p[k] && p[k] <= hi[k])) return 0; }
            continue;
        }
        i128 a, b, den;
        if (d[k] > 0) { a = (i128)lo[k] - p[k]; b = (i128)hi[k] - p[k]; den = d[k]; }
        else          { a = (i128)p[k] - hi[k]; b = (i128)p[k] - lo[k]; den = -(i128)d[k]; }
        /* t >= a/den and t <= b/den (strict when open) */
        if (frac_cmp(a, den, ln, ld) > 0) { ln = a; ld = den; }
        if (frac_cmp(b, den, un, ud) < 0) { un = b; ud = den; }
    }
    int c = frac_cmp(ln, ld, un, ud);
    return open ? (c < 0) : (c <= 0);
}

/* sign of (b - a) x (c - a) */
static int orient(int64_t ax, int64_t ay, int64_t bx, int64_t by, int64_t cx, int64_t cy)
{
    i128 v = (i128)(bx - ax) * (cy - ay) - (i128)(by - ay) * (cx - ax);
    return (v > 0) - (v < 0);
}

/* c on the closed segment a-b, given orient(a,b,c) == 0 */
static int on_seg(int64_t ax, int64_t ay, int64_t bx, int64_t by, int64_t cx, int64_t cy)
{
    return (cx >= (ax < bx ? ax : bx)) && (cx <= (ax > bx ? ax : bx)) &&
           (cy >= (ay < by ? ay : by)) && (cy <= (ay > by ? ay : by));
}

/* closed segments a-b and c-d share a point */
static int seg_seg(int64_t ax, int64_t ay, int64_t bx, int64_t by,
                   int64_t cx, int64_t cy, int64_t dx, int64_t dy)
{
    int o1 = orient(ax, ay, bx, by, cx, cy), o2 = orient(ax, ay, bx, by, dx, dy);
    int o3 = orient(cx, cy, dx, dy, ax, ay), o4 = orient(cx, cy, dx, dy, bx, by);
    if (o1 * o2 < 0 && o3 * o4 < 0) return 1;
    if (o1 == 0 && on_seg(ax, ay, bx, by, cx, cy)) return 1;
    if (o2 == 0 && on_seg(ax, ay, bx, by, dx, dy)) return 1;
    if (o3 == 0 && on_seg(cx, cy, dx, dy, ax, ay)) return 1;
    if (o4 == 0 && on_seg(cx, cy, dx, dy, bx, by)) return 1;
    return 0;
}

/*
 * Crossing-number test of point (X, Y) against the polygon with vertices
 * (vx[k], vy[k]); all coordinates in the same integer units.  Counts the
 * edges crossed by the ray from the point towards +x, with the half-open
 * rule (an edge counts if exactly one endpoint lies strictly above the
 * ray).  Odd -> inside.  Exact for points off the boundary; callers only
 * ask about such points.  `edges` (optional) restricts the scan to the
 * listed edge indices; the others must not cross the ray's line.
 */
static int crossing_inside(const int64_t *vx, const int64_t *vy, int64_t nv,
                           const int64_t *edges, int64_t ne, int64_t X, int64_t Y)
{
    int in = 0;
    for (int64_t t = 0; t < ne; t++) {
        int64_t k = edges ? edges[t] : t;
        int64_t k2 = (k + 1 == nv) ? 0 : k + 1;
        int64_t ax = vx[k], ay = vy[k], bx = vx[k2], by = vy[k2];
        if ((ay > Y) == (by > Y)) continue;
        /* x of the crossing is ax + (Y - ay)(bx - ax)/(by - ay); compare with X */
        i128 den = (i128)by - ay;
        i128 num = ((i128)ax - X) * den + ((i128)Y - ay) * ((i128)bx - ax);
        /* crossing x - X = num/den > 0 ? */
        if ((num > 0 && den > 0) || (num < 0 && den < 0)) in ^= 1;
    }
    return in;
}

/* ---------------------------------------------------------------- hilbert */

/*
 * Position of cell (x, y) along the order-`order` Hilbert curve.  At each
 * level the cell's quadrant (rx, ry) contributes its rank 0..3 along the
 * curve times the quadrant size; then the coordinates are mapped into the
 * quadrant's own frame (the lower quadrants are transposed, the lower-right
 * one also reflected) before the next level.
 */
uint64_t orc_hilbert(int order, uint64_t x, uint64_t y)
{
    uint64_t d = 0;
    for (uint64_t s = (uint64_t)1 << (order - 1); s > 0; s >>= 1) {
        uint64_t rx = (x & s) ? 1 : 0;
        uint64_t ry = (y & s) ? 1 : 0;
        d += s * s * ((3 * rx) ^ ry);
        x &= s - 1;
        y &= s - 1;
        if (ry == 0) {
            if (rx == 1) { x = s - 1 - x; y = s - 1 - y; }
            uint64_t t = x; x = y; y = t;
        }
    }
    return d;
}

void orc_hilbert_many(int order, const uint64_t *x, const uint64_t *y, int64_t n, uint64_t *d)
{
    for (int64_t k = 0; k < n; k++) d[k] = orc_hilbert(order, x[k], y[k]);
}

/* ------------------------------------------------------------ classify */

#define CELL_EMPTY 0
#define CELL_PARTIAL 1
#define CELL_FULL 2

typedef struct {
    int64_t *x, *y;     /* lattice coords relative to the grid origin */
    int64_t nv;
    int64_t minx, miny, maxx, maxy;
} poly_t;

static int load_poly(const grid_t *g, const double *xy, int64_t nv, poly_t *p)
{
    if (nv < 3) return ORC_E_INVALID;
    p->x = (int64_t *)malloc(sizeof(int64_t) * nv);
    p->y = (int64_t *)malloc(sizeof(int64_t) * nv);
    if (!p->x || !p->y) { free(p->x); free(p->y); return ORC_E_NOMEM; }
    p->nv = nv;
    for (int64_t k = 0; k < nv; k++) {
        int rc = lattice(xy[2 * k], g->x0, &p->x[k]);
        if (!rc) rc = lattice(xy[2 * k + 1], g->y0, &p->y[k]);
        if (rc) { free(p->x); free(p->y); return rc; }
        if (k == 0 || p->x[k] < p->minx) p->minx = p->x[k];
        if (k == 0 || p->y[k] < p->miny) p->miny = p->y[k];
        if (k == 0 || p->x[k] > p->maxx) p->maxx = p->x[k];
        if (k == 0 || p->y[k] > p->maxy) p->maxy = p->y[k];
    }
    /* guard ring: the polygon must stay clear of the outermost cells */
    int64_t lo = g->W, hi = (g->n - 1) * g->W;
    if (p->minx <= lo || p->miny <= lo || p->maxx >= hi || p->maxy >= hi) {
        free(p->x); free(p->y); return ORC_E_GRID;
    }
    return ORC_OK;
}

static int64_t floordiv(int64_t a, int64_t b) { int64_t q = a / b; if ((a % b) && ((a < 0) != (b < 0))) q--; return q; }
static int64_t ceildiv(int64_t a, int64_t b) { return -floordiv(-a, b); }

typedef void (*cell_cb)(void *ctx, int64_t i, int64_t j, int cls);

/* Visit every cell of the polygon's cell window with its class. */
static int classify_poly(const grid_t *g, const poly_t *p, cell_cb cb, void *ctx)
{
    const int64_t W = g->W, nv = p->nv;
    /* cells whose closed extent meets [min, max] */
    int64_t i0 = ceildiv(p->minx, W) - 1, i1 = floordiv(p->maxx, W);
    int64_t j0 = ceildiv(p->miny, W) - 1, j1 = floordiv(p->maxy, W);
    int64_t *row = (int64_t *)malloc(sizeof(int64_t) * nv);
    int64_t *mid = (int64_t *)malloc(sizeof(int64_t) * nv);
    int64_t *X2 = (int64_t *)malloc(sizeof(int64_t) * nv);
    int64_t *Y2 = (int64_t *)malloc(sizeof(int64_t) * nv);
    if (!row || !mid || !X2 || !Y2) { free(row); free(mid); free(X2); free(Y2); return ORC_E_NOMEM; }
    for (int64_t k = 0; k < nv; k++) { X2[k] = 2 * p->x[k]; Y2[k] = 2 * p->y[k]; }
    for (int64_t j = j0; j <= j1; j++) {
        int64_t by0 = j * W, by1 = (j + 1) * W;
        int64_t nrow = 0, nmid = 0, yc2 = (2 * j + 1) * W;
        for (int64_t k = 0; k < nv; k++) {
            int64_t k2 = (k + 1 == nv) ? 0 : k + 1;
            int64_t ylo = p->y[k] < p->y[k2] ? p->y[k] : p->y[k2];
            int64_t yhi = p->y[k] > p->y[k2] ? p->y[k] : p->y[k2];
            if (yhi >= by0 && ylo <= by1) row[nrow++] = k;
            if ((Y2[k] > yc2) != (Y2[k2] > yc2)) mid[nmid++] = k;
        }
        for (int64_t i = i0; i <= i1; i++) {
            int64_t bx0 = i * W, bx1 = (i + 1) * W;
            int open_touch = 0, closed_touch = 0;
            for (int64_t t = 0; t < nrow && !open_touch; t++) {
                int64_t k = row[t], k2 = (k + 1 == nv) ? 0 : k + 1;
                /* an edge whose x-range misses the cell's cannot meet it */
                int64_t xlo = p->x[k] < p->x[k2] ? p->x[k] : p->x[k2];
                int64_t xhi = p->x[k] > p->x[k2] ? p->x[k] : p->x[k2];
                if (xhi < bx0 || xlo > bx1) continue;
                if (seg_meets_box(p->x[k], p->y[k], p->x[k2], p->y[k2], bx0, by0, bx1, by1, 1))
                    open_touch = 1;
                else if (!closed_touch &&
                         seg_meets_box(p->x[k], p->y[k], p->x[k2], p->y[k2], bx0, by0, bx1, by1, 0))
                    closed_touch = 1;
            }
            int cls;
            if (open_touch) cls = CELL_PARTIAL;
            else {
                /* no edge meets the open cell, so the centre is off the boundary */
                int in = crossing_inside(X2, Y2, nv, mid, nmid, (2 * i + 1) * W, yc2);
                cls = in ? CELL_FULL : (closed_touch ? CELL_PARTIAL : CELL_EMPTY);
            }
            cb(ctx, i, j, cls);
        }
    }
    free(row); free(mid); free(X2); free(Y2);
    return ORC_OK;
}

/* ------------------------------------------------------------ intervals */

typedef struct { uint64_t *v; int64_t n, cap; } vec_t;

static int vec_push(vec_t *a, uint64_t x)
{
    if (a->n == a->cap) {
        int64_t nc = a->cap ? a->cap * 2 : 1024;
        uint64_t *nv = (uint64_t *)realloc(a->v, sizeof(uint64_t) * nc);
        if (!nv) return ORC_E_NOMEM;
        a->v = nv; a->cap = nc;
    }
    a->v[a->n++] = x;
    return ORC_OK;
}

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x < y) ? -1 : (x > y);
}

/* sorted ids -> maximal half-open runs, appended as (start, end) pairs */
static int intervalize(vec_t *ids, vec_t *out)
{
    qsort(ids->v, ids->n, sizeof(uint64_t), cmp_u64);
    int64_t k = 0;
    while (k < ids->n) {
        uint64_t s = ids->v[k], e = s + 1;
        k++;
        while (k < ids->n && ids->v[k] == e) { e++; k++; }
        if (vec_push(out, s) || vec_push(out, e)) return ORC_E_NOMEM;
    }
    return ORC_OK;
}

typedef struct { const grid_t *g; vec_t a, f; int err; } collect_t;

static void collect_cb(void *ctx, int64_t i, int64_t j, int cls)
{
    collect_t *c = (collect_t *)ctx;
    if (cls == CELL_EMPTY) return;
    uint64_t d = orc_hilbert(c->g->order, (uint64_t)i, (uint64_t)j);
    if (vec_push(&c->a, d)) c->err = ORC_E_NOMEM;
    if (cls == CELL_FULL && vec_push(&c->f, d)) c->err = ORC_E_NOMEM;
}

/* The A- and F-lists of one polygon as malloc'd (start,end) pair arrays. */
static int lists_of_polygon(const grid_t *g, const double *xy, int64_t nv,
                            vec_t *A, vec_t *F)
{
    poly_t p;
    int rc = load_poly(g, xy, nv, &p);
    if (rc) return rc;
    collect_t c = {g, {0, 0, 0}, {0, 0, 0}, 0};
    rc = classify_poly(g, &p, collect_cb, &c);
    free(p.x); free(p.y);
    if (!rc) rc = c.err;
    if (!rc) rc = intervalize(&c.a, A);
    if (!rc) rc = intervalize(&c.f, F);
    free(c.a.v); free(c.f.v);
    return rc;
}

/* ----------------------------------------------------- public: classify */

typedef struct { int64_t *cells; int64_t n, cap; int err; } cellbuf_t;

static void cellbuf_cb(void *ctx, int64_t i, int64_t j, int cls)
{
    cellbuf_t *b = (cellbuf_t *)ctx;
    if (b->n == b->cap) {
        int64_t nc = b->cap ? b->cap * 2 : 4096;
        int64_t *nv = (int64_t *)realloc(b->cells, sizeof(int64_t) * 3 * nc);
        if (!nv) { b->err = ORC_E_NOMEM; return; }
        b->cells = nv; b->cap = nc;
    }
    b->cells[3 * b->n] = i; b->cells[3 * b->n + 1] = j; b->cells[3 * b->n + 2] = cls;
    b->n++;
}

/*
 * Classify every cell of one polygon's cell window.  Returns a malloc'd
 * array of (i, j, class) triples in *out (free with orc_free) and its length.
 */
int orc_classify(double x0, double y0, double side, int order,
                 const double *xy, int64_t nv, int64_t **out, int64_t *n_out)
{
    grid_t g;
    int rc = make_grid(x0, y0, side, order, &g);
    if (rc) return rc;
    poly_t p;
    rc = load_poly(&g, xy, nv, &p);
    if (rc) return rc;
    cellbuf_t b = {0, 0, 0, 0};
    rc = classify_poly(&g, &p, cellbuf_cb, &b);
    free(p.x); free(p.y);
    if (!rc) rc = b.err;
    if (rc) { free(b.cells); return rc; }
    *out = b.cells; *n_out = b.n;
    return ORC_OK;
}

/*
 * Classes of given cells of one polygon: cell t is (i, j) = (ij[2t],
 * ij[2t + 1]) and cls[t] gets CELL_EMPTY / CELL_PARTIAL / CELL_FULL, decided
 * by the same brute-force rule as orc_classify, for polygons whose whole
 * cell window is too large to classify (checks by sampled cells).  As in
 * orc_classify, the cells are taken row by row: an edge whose y-range misses
 * the row cannot meet its cells, and only edges across the row's centre line
 * can cross a centre's ray; every other edge is tested for every cell.
 */
static int cmp_row(const void *a, const void *b)   /* (row, index) pairs by row */
{
    const int64_t ja = ((const int64_t *)a)[0], jb = ((const int64_t *)b)[0];
    return ja < jb ? -1 : ja > jb;
}

int orc_classify_cells(double x0, double y0, double side, int order, const double *xy, int64_t nv,
                       const int64_t *ij, int64_t n, uint8_t *cls)
{
    grid_t g;
    int rc = make_grid(x0, y0, side, order, &g);
    if (rc) return rc;
    poly_t p;
    rc = load_poly(&g, xy, nv, &p);
    if (rc) return rc;
    const int64_t W = g.W, m = p.nv;
    int64_t *X2 = (int64_t *)malloc(sizeof(int64_t) * m);
    int64_t *Y2 = (int64_t *)malloc(sizeof(int64_t) * m);
    int64_t *row = (int64_t *)malloc(sizeof(int64_t) * m);
    int64_t *mid = (int64_t *)malloc(sizeof(int64_t) * m);
    int64_t *ord = (int64_t *)malloc(sizeof(int64_t) * 2 * (n ? n : 1));   /* (row, cell index) */
    if (!X2 || !Y2 || !row || !mid || !ord) {
        free(X2); free(Y2); free(row); free(mid); free(ord); free(p.x); free(p.y);
        return ORC_E_NOMEM;
    }
    for (int64_t k = 0; k < m; k++) { X2[k] = 2 * p.x[k]; Y2[k] = 2 * p.y[k]; }
    /* cells grouped by row (the order within a row does not matter) */
    for (int64_t t = 0; t < n; t++) { ord[2 * t] = ij[2 * t + 1]; ord[2 * t + 1] = t; }
    qsort(ord, (size_t)n, 2 * sizeof(int64_t), cmp_row);
    for (int64_t u = 0; u < n;) {
        const int64_t j = ord[2 * u];
        const int64_t by0 = j * W, by1 = (j + 1) * W, yc2 = (2 * j + 1) * W;
        int64_t nrow = 0, nmid = 0;
        for (int64_t k = 0; k < m; k++) {
            const int64_t k2 = (k + 1 == m) ? 0 : k + 1;
            const int64_t ylo = p.y[k] < p.y[k2] ? p.y[k] : p.y[k2], yhi = p.y[k] > p.y[k2] ? p.y[k] : p.y[k2];
            if (yhi >= by0 && ylo <= by1) row[nrow++] = k;
            if ((Y2[k] > yc2) != (Y2[k2] > yc2)) mid[nmid++] = k;
        }
        for (; u < n && ord[2 * u] == j; u++) {
            const int64_t t = ord[2 * u + 1], i = ij[2 * t];
            const int64_t bx0 = i * W, bx1 = (i + 1) * W;
            int open_touch = 0, closed_touch = 0;
            for (int64_t q = 0; q < nrow && !open_touch; q++) {
                const int64_t k = row[q], k2 = (k + 1 == m) ? 0 : k + 1;
                const int64_t xlo = p.x[k] < p.x[k2] ? p.x[k] : p.x[k2], xhi = p.x[k] > p.x[k2] ? p.x[k] : p.x[k2];
                if (xhi < bx0 || xlo > bx1) continue;
                if (seg_meets_box(p.x[k], p.y[k], p.x[k2], p.y[k2], bx0, by0, bx1, by1, 1))
                    open_touch = 1;
                else if (!closed_touch && seg_meets_box(p.x[k], p.y[k], p.x[k2], p.y[k2], bx0, by0, bx1, by1, 0))
                    closed_touch = 1;
            }
            if (open_touch) cls[t] = CELL_PARTIAL;
            else {
                const int in = crossing_inside(X2, Y2, m, mid, nmid, (2 * i + 1) * W, yc2);
                cls[t] = in ? CELL_FULL : (closed_touch ? CELL_PARTIAL : CELL_EMPTY);
            }
        }
    }
    free(X2); free(Y2); free(row); free(mid); free(ord); free(p.x); free(p.y);
    return ORC_OK;
}

void orc_free(void *p) { free(p); }

/* ------------------------------------------------- public: build lists */

typedef struct {
    grid_t g;
    const double *xy;
    const int64_t *voff;
    int64_t n;
    vec_t *A, *F;
    _Atomic int64_t next;
    _Atomic int err;
} build_job_t;

static void *build_worker(void *arg)
{
    build_job_t *J = (build_job_t *)arg;
    for (;;) {
        int64_t k = atomic_fetch_add(&J->next, 1);
        if (k >= J->n || atomic_load(&J->err)) break;
        int rc = lists_of_polygon(&J->g, J->xy + 2 * J->voff[k], J->voff[k + 1] - J->voff[k],
                                  &J->A[k], &J->F[k]);
        if (rc) { int z = 0; atomic_compare_exchange_strong(&J->err, &z, rc); }
    }
    return NULL;
}

typedef struct {
    int64_t n;
    vec_t *A, *F;
} orc_lists;

static int run_threads(void *(*fn)(void *), void *arg, int nthreads)
{
    if (nthreads <= 1) { fn(arg); return 1; }
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * nthreads);
    int started = 0;
    for (int t = 0; t < nthreads; t++)
        if (pthread_create(&th[t], NULL, fn, arg) == 0) started++;
        else break;
    if (started == 0) fn(arg);
    for (int t = 0; t < started; t++) pthread_join(th[t], NULL);
    free(th);
    return started ? started : 1;
}

void orc_lists_free(orc_lists *L)
{
    if (!L) return;
    for (int64_t k = 0; k < L->n; k++) { free(L->A[k].v); free(L->F[k].v); }
    free(L->A); free(L->F); free(L);
}

/* Build the A- and F-lists of polygons voff[k]..voff[k+1] of xy. */
int orc_build(double x0, double y0, double side, int order, const double *xy,
              const int64_t *voff, int64_t n, int nthreads, orc_lists **out)
{
    build_job_t J;
    int rc = make_grid(x0, y0, side, order, &J.g);
    if (rc) return rc;
    J.xy = xy; J.voff = voff; J.n = n;
    J.A = (vec_t *)calloc(n ? n : 1, sizeof(vec_t));
    J.F = (vec_t *)calloc(n ? n : 1, sizeof(vec_t));
    if (!J.A || !J.F) { free(J.A); free(J.F); return ORC_E_NOMEM; }
    atomic_init(&J.next, 0);
    atomic_init(&J.err, 0);
    run_threads(build_worker, &J, nthreads);
    orc_lists *L = (orc_lists *)malloc(sizeof(orc_lists));
    L->n = n; L->A = J.A; L->F = J.F;
    if (atomic_load(&J.err)) { orc_lists_free(L); return atomic_load(&J.err); }
    *out = L;
    return ORC_OK;
}

void orc_lists_sizes(const orc_lists *L, int64_t *nA, int64_t *nF)
{
    int64_t a = 0, f = 0;
    for (int64_t k = 0; k < L->n; k++) { a += L->A[k].n / 2; f += L->F[k].n / 2; }
    *nA = a; *nF = f;
}

/* Copy into CSR + SoA arrays sized from orc_lists_sizes. */
void orc_lists_export(const orc_lists *L, uint64_t *offA, uint32_t *sA, uint32_t *eA,
                      uint64_t *offF, uint32_t *sF, uint32_t *eF)
{
    uint64_t a = 0, f = 0;
    for (int64_t k = 0; k < L->n; k++) {
        offA[k] = a; offF[k] = f;
        for (int64_t t = 0; t < L->A[k].n; t += 2) { sA[a] = (uint32_t)L->A[k].v[t]; eA[a] = (uint32_t)L->A[k].v[t + 1]; a++; }
        for (int64_t t = 0; t < L->F[k].n; t += 2) { sF[f] = (uint32_t)L->F[k].v[t]; eF[f] = (uint32_t)L->F[k].v[t + 1]; f++; }
    }
    offA[L->n] = a; offF[L->n] = f;
}

/* ------------------------------------------------------- public: filter */

/*
 * IntervalJoin of Alg. 2 over X = [xs, xe)[0..n) and Y = [ys, ye)[0..m).
 * Returns 1 on the first overlapping pair of heads.  *rx, *ry receive how
 * many leading elements of X and Y the loop read.
 */
int orc_interval_join(const uint32_t *xs, const uint32_t *xe, uint64_t n,
                      const uint32_t *ys, const uint32_t *ye, uint64_t m,
                      uint64_t *rx, uint64_t *ry)
{
    uint64_t i = 0, j = 0, ri = 0, rj = 0;
    int found = 0;
    while (i < n && j < m) {
        ri = i + 1; rj = j + 1;                       /* heads read */
        if (xs[i] < ye[j] && ys[j] < xe[i]) { found = 1; break; }
        if (xe[i] <= ye[j]) i++; else j++;
    }
    if (rx) *rx = ri;
    if (ry) *ry = rj;
    return found;
}

#define V_TN 0
#define V_TH 1
#define V_IND 2

typedef struct {
    const uint64_t *oAr, *oFr, *oAs, *oFs;
    const uint32_t *sAr, *eAr, *sFr, *eFr, *sAs, *eAs, *sFs, *eFs;
    const uint32_t *r, *s;
    int64_t P;
    uint8_t *verdict;
    uint64_t *bytes;
    _Atomic int64_t next;
} filter_job_t;

static uint64_t umax(uint64_t a, uint64_t b) { return a > b ? a : b; }

/*
 * Alg. 2 on one pair.  Also returns the bytes it had to move: 8 for the
 * pair's two ids, 16 per list whose [begin, end) offsets it looked up
 * (two 8-byte CSR offsets), 8 per distinct interval read (two 4-byte
 * endpoints), 1 for the verdict.
 */
static uint8_t april_pair(const filter_job_t *J, uint32_t r, uint32_t s, uint64_t *bytes)
{
    const uint64_t ar0 = J->oAr[r], ar1 = J->oAr[r + 1], as0 = J->oAs[s], as1 = J->oAs[s + 1];
    uint64_t x, y, ax_r = 0, ax_s = 0, n_fr = 0, n_fs = 0, lists = 2;
    uint8_t v;
    if (!orc_interval_join(J->sAr + ar0, J->eAr + ar0, ar1 - ar0,
                           J->sAs + as0, J->eAs + as0, as1 - as0, &x, &y)) {
        ax_r = x; ax_s = y; v = V_TN;
    } else {
        ax_r = x; ax_s = y;
        const uint64_t fs0 = J->oFs[s], fs1 = J->oFs[s + 1];
        lists++;
        if (orc_interval_join(J->sAr + ar0, J->eAr + ar0, ar1 - ar0,
                              J->sFs + fs0, J->eFs + fs0, fs1 - fs0, &x, &y)) {
            ax_r = umax(ax_r, x); n_fs = y; v = V_TH;
        } else {
            ax_r = umax(ax_r, x); n_fs = y;
            const uint64_t fr0 = J->oFr[r], fr1 = J->oFr[r + 1];
            lists++;
            int hit = orc_interval_join(J->sFr + fr0, J->eFr + fr0, fr1 - fr0,
                                        J->sAs + as0, J->eAs + as0, as1 - as0, &x, &y);
            n_fr = x; ax_s = umax(ax_s, y);
            v = hit ? V_TH : V_IND;
        }
    }
    if (bytes) *bytes = 8 + 16 * lists + 8 * (ax_r + ax_s + n_fr + n_fs) + 1;
    return v;
}

static void *filter_worker(void *arg)
{
    filter_job_t *J = (filter_job_t *)arg;
    const int64_t chunk = 4096;
    for (;;) {
        int64_t b = atomic_fetch_add(&J->next, chunk);
        if (b >= J->P) break;
        int64_t e = b + chunk < J->P ? b + chunk : J->P;
        for (int64_t p = b; p < e; p++) {
            uint64_t by;
            J->verdict[p] = april_pair(J, J->r[p], J->s[p], &by);
            if (J->bytes) J->bytes[p] = by;
        }
    }
    return NULL;
}

/*
 * Alg. 2 over n_pairs candidate pairs (r[p], s[p]).  verdict[p] receives
 * 0 = true negative, 1 = true hit, 2 = indecisive; bytes (optional) the
 * per-pair bytes moved.  Returns the number of threads used.
 */
int orc_filter(const uint64_t *oAr, const uint32_t *sAr, const uint32_t *eAr,
               const uint64_t *oFr, const uint32_t *sFr, const uint32_t *eFr,
               const uint64_t *oAs, const uint32_t *sAs, const uint32_t *eAs,
               const uint64_t *oFs, const uint32_t *sFs, const uint32_t *eFs,
               const uint32_t *r, const uint32_t *s, int64_t P,
               uint8_t *verdict, uint64_t *bytes, int nthreads)
{
    filter_job_t J;
    J.oAr = oAr; J.oFr = oFr; J.oAs = oAs; J.oFs = oFs;
    J.sAr = sAr; J.eAr = eAr; J.sFr = sFr; J.eFr = eFr;
    J.sAs = sAs; J.eAs = eAs; J.sFs = sFs; J.eFs = eFs;
    J.r = r; J.s = s; J.P = P; J.verdict = verdict; J.bytes = bytes;
    atomic_init(&J.next, 0);
    return run_threads(filter_worker, &J, nthreads);
}

/* ----------------------------------------------------- public: mbr join */

typedef struct { double x0, y0, x1, y1; } box_t;

static void poly_box(const double *xy, int64_t nv, box_t *b)
{
    b->x0 = b->x1 = xy[0]; b->y0 = b->y1 = xy[1];
    for (int64_t k = 1; k < nv; k++) {
        double x = xy[2 * k], y = xy[2 * k + 1];
        if (x < b->x0) b->x0 = x;
        if (x > b->x1) b->x1 = x;
        if (y < b->y0) b->y0 = y;
        if (y > b->y1) b->y1 = y;
    }
}

static int boxes_meet(const box_t *a, const box_t *b)
{
    return a->x0 <= b->x1 && b->x0 <= a->x1 && a->y0 <= b->y1 && b->y0 <= a->y1;
}

typedef struct { double key; int64_t id; } keyed_t;

static int cmp_keyed(const void *a, const void *b)
{
    const keyed_t *x = (const keyed_t *)a, *y = (const keyed_t *)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

typedef struct {
    const box_t *R, *S;
    int64_t nR, nS;
    const keyed_t *sorted;   /* S by x0 */
    double maxw;
    vec_t *per_r;            /* candidate s ids per r */
    _Atomic int64_t next;
    _Atomic int err;
} mbr_job_t;

static void *mbr_worker(void *arg)
{
    mbr_job_t *J = (mbr_job_t *)arg;
    for (;;) {
        int64_t r = atomic_fetch_add(&J->next, 1);
        if (r >= J->nR) break;
        const box_t *a = &J->R[r];
        /* every s with x0 in [a.x0 - maxw, a.x1] (the others cannot meet a) */
        double lo = a->x0 - J->maxw;
        int64_t L = 0, H = J->nS;
        while (L < H) { int64_t M = (L + H) / 2; if (J->sorted[M].key < lo) L = M + 1; else H = M; }
        vec_t *out = &J->per_r[r];
        for (int64_t t = L; t < J->nS && J->sorted[t].key <= a->x1; t++) {
            int64_t s = J->sorted[t].id;
            if (boxes_meet(a, &J->S[s]) && vec_push(out, (uint64_t)s)) { atomic_store(&J->err, ORC_E_NOMEM); return NULL; }
        }
        qsort(out->v, out->n, sizeof(uint64_t), cmp_u64);
    }
    return NULL;
}

typedef struct { int64_t n; vec_t *per_r; } orc_pairs;

int orc_mbr_join(const double *xyR, const int64_t *voffR, int64_t nR,
                 const double *xyS, const int64_t *voffS, int64_t nS,
                 int nthreads, orc_pairs **out, int64_t *n_pairs)
{
    box_t *R = (box_t *)malloc(sizeof(box_t) * (nR ? nR : 1));
    box_t *S = (box_t *)malloc(sizeof(box_t) * (nS ? nS : 1));
    keyed_t *sorted = (keyed_t *)malloc(sizeof(keyed_t) * (nS ? nS : 1));
    vec_t *per_r = (vec_t *)calloc(nR ? nR : 1, sizeof(vec_t));
    if (!R || !S || !sorted || !per_r) { free(R); free(S); free(sorted); free(per_r); return ORC_E_NOMEM; }
    double maxw = 0;
    for (int64_t k = 0; k < nR; k++) poly_box(xyR + 2 * voffR[k], voffR[k + 1] - voffR[k], &R[k]);
    for (int64_t k = 0; k < nS; k++) {
        poly_box(xyS + 2 * voffS[k], voffS[k + 1] - voffS[k], &S[k]);
        if (S[k].x1 - S[k].x0 > maxw) maxw = S[k].x1 - S[k].x0;
        sorted[k].key = S[k].x0; sorted[k].id = k;
    }
    qsort(sorted, nS, sizeof(keyed_t), cmp_keyed);
    mbr_job_t J;
    J.R = R; J.S = S; J.nR = nR; J.nS = nS; J.sorted = sorted; J.maxw = maxw; J.per_r = per_r;
    atomic_init(&J.next, 0);
    atomic_init(&J.err, 0);
    run_threads(mbr_worker, &J, nthreads);
    free(R); free(S); free(sorted);
    orc_pairs *P = (orc_pairs *)malloc(sizeof(orc_pairs));
    P->n = nR; P->per_r = per_r;
    int64_t tot = 0;
    for (int64_t k = 0; k < nR; k++) tot += per_r[k].n;
    *out = P; *n_pairs = tot;
    return atomic_load(&J.err);
}

void orc_pairs_export(const orc_pairs *P, uint32_t *r, uint32_t *s)
{
    int64_t t = 0;
    for (int64_t k = 0; k < P->n; k++)
        for (int64_t q = 0; q < P->per_r[k].n; q++) { r[t] = (uint32_t)k; s[t] = (uint32_t)P->per_r[k].v[q]; t++; }
}

void orc_pairs_free(orc_pairs *P)
{
    if (!P) return;
    for (int64_t k = 0; k < P->n; k++) free(P->per_r[k].v);
    free(P->per_r); free(P);
}

/* ------------------------------------------------ public: exact geometry */

/*
 * Do the closed polygons a (na vertices) and b (nb vertices) share a point?
 * Coordinates must be lattice multiples (any common origin).  Returns 1/0,
 * or a negative error.
 */
int orc_polygons_intersect(const double *a, int64_t na, const double *b, int64_t nb)
{
    int64_t *ax = (int64_t *)malloc(sizeof(int64_t) * 2 * na);
    int64_t *bx = (int64_t *)malloc(sizeof(int64_t) * 2 * nb);
    if (!ax || !bx) { free(ax); free(bx); return ORC_E_NOMEM; }
    int64_t *ay = ax + na, *by = bx + nb;
    int rc = ORC_OK;
    for (int64_t k = 0; k < na && !rc; k++) { rc = lattice(a[2 * k], 0.0, &ax[k]); if (!rc) rc = lattice(a[2 * k + 1], 0.0, &ay[k]); }
    for (int64_t k = 0; k < nb && !rc; k++) { rc = lattice(b[2 * k], 0.0, &bx[k]); if (!rc) rc = lattice(b[2 * k + 1], 0.0, &by[k]); }
    if (rc) { free(ax); free(bx); return rc; }
    int hit = 0;
    for (int64_t k = 0; k < na && !hit; k++) {
        int64_t k2 = (k + 1 == na) ? 0 : k + 1;
        for (int64_t q = 0; q < nb && !hit; q++) {
            int64_t q2 = (q + 1 == nb) ? 0 : q + 1;
            hit = seg_seg(ax[k], ay[k], ax[k2], ay[k2], bx[q], by[q], bx[q2], by[q2]);
        }
    }
    /* no boundary contact: one contains the other, or they are disjoint */
    if (!hit) hit = crossing_inside(bx, by, nb, NULL, nb, ax[0], ay[0]);
    if (!hit) hit = crossing_inside(ax, ay, na, NULL, na, bx[0], by[0]);
    free(ax); free(bx);
    return hit;
}

/* Exact twice-area (shoelace) of a polygon in lattice units^2, as two int64 halves. */
void orc_twice_area(const double *xy, int64_t nv, int64_t *hi, uint64_t *lo)
{
    i128 acc = 0;
    for (int64_t k = 0; k < nv; k++) {
        int64_t k2 = (k + 1 == nv) ? 0 : k + 1;
        int64_t x1 = 0, y1 = 0, x2 = 0, y2 = 0;
        lattice(xy[2 * k], 0.0, &x1); lattice(xy[2 * k + 1], 0.0, &y1);
        lattice(xy[2 * k2], 0.0, &x2); lattice(xy[2 * k2 + 1], 0.0, &y2);
        acc += (i128)x1 * y2 - (i128)x2 * y1;
    }
    *hi = (int64_t)(acc >> 64);
    *lo = (uint64_t)acc;
}

/* ------------------------------------------ public: query variants (Sec. 4.3, 5.3) */

/*
 * Within join (Sec. 4.3.2): is r within s?  Two of Alg. 2's steps:
 *   AA-join: no overlap -> true negative (r and s are disjoint);
 *   every interval of A(r) inside one interval of F(s) -> true hit (every
 *   cell r meets is Full in s, so r lies inside s);
 *   otherwise indecisive.
 * F-lists hold maximal runs, so an A(r) interval inside F(s) as a cell set
 * lies inside a single F(s) interval.  The test walks both lists once.
 */
static int a_inside_f(const uint32_t *as, const uint32_t *ae, uint64_t n,
                      const uint32_t *fs, const uint32_t *fe, uint64_t m)
{
    uint64_t j = 0;
    for (uint64_t i = 0; i < n; i++) {
        while (j < m && fe[j] <= as[i]) j++;       /* F intervals ending before this A starts */
        if (j == m || !(fs[j] <= as[i] && ae[i] <= fe[j])) return 0;
    }
    return 1;
}

int orc_filter_within(const uint64_t *oAr, const uint32_t *sAr, const uint32_t *eAr,
                      const uint64_t *oAs, const uint32_t *sAs, const uint32_t *eAs,
                      const uint64_t *oFs, const uint32_t *sFs, const uint32_t *eFs,
                      const uint32_t *r, const uint32_t *s, int64_t P, uint8_t *verdict)
{
    for (int64_t p = 0; p < P; p++) {
        const uint64_t a0 = oAr[r[p]], a1 = oAr[r[p] + 1];
        const uint64_t b0 = oAs[s[p]], b1 = oAs[s[p] + 1];
        const uint64_t f0 = oFs[s[p]], f1 = oFs[s[p] + 1];
        if (!orc_interval_join(sAr + a0, eAr + a0, a1 - a0, sAs + b0, eAs + b0, b1 - b0, NULL, NULL))
            verdict[p] = V_TN;
        else if (a_inside_f(sAr + a0, eAr + a0, a1 - a0, sFs + f0, eFs + f0, f1 - f0))
            verdict[p] = V_TH;
        else
            verdict[p] = V_IND;
    }
    return ORC_OK;
}

/*
 * Linestring approximation (Sec. 4.3.3): a linestring covers no cell, so it
 * is kept as the sorted list of the ids of the cells whose closed square one
 * of its segments meets (all of them Partial).  Brute force: every cell of
 * each segment's bounding window is tested against the segment.
 */
typedef struct { uint64_t *off; uint32_t *ids; int64_t n; } orc_cells;

int orc_build_cells(double x0, double y0, double side, int order, const double *xy,
                    const int64_t *voff, int64_t n, orc_cells **out)
{
    grid_t g;
    int rc = make_grid(x0, y0, side, order, &g);
    if (rc) return rc;
    orc_cells *C = (orc_cells *)calloc(1, sizeof(orc_cells));
    if (!C) return ORC_E_NOMEM;
    C->n = n;
    C->off = (uint64_t *)malloc(sizeof(uint64_t) * (n + 1));
    vec_t all = {0, 0, 0};
    if (!C->off) { free(C); return ORC_E_NOMEM; }
    C->off[0] = 0;
    for (int64_t k = 0; k < n && !rc; k++) {
        const int64_t v0 = voff[k], nv = voff[k + 1] - voff[k];
        if (nv < 2) { rc = ORC_E_INVALID; break; }
        int64_t *X = (int64_t *)malloc(sizeof(int64_t) * nv), *Y = (int64_t *)malloc(sizeof(int64_t) * nv);
        if (!X || !Y) { free(X); free(Y); rc = ORC_E_NOMEM; break; }
        for (int64_t v = 0; v < nv && !rc; v++) {
            rc = lattice(xy[2 * (v0 + v)], g.x0, &X[v]);
            if (!rc) rc = lattice(xy[2 * (v0 + v) + 1], g.y0, &Y[v]);
            /* the same guard ring as for polygons */
            if (!rc && (X[v] <= g.W || Y[v] <= g.W || X[v] >= (g.n - 1) * g.W || Y[v] >= (g.n - 1) * g.W))
                rc = ORC_E_GRID;
        }
        vec_t ids = {0, 0, 0};
        for (int64_t v = 0; v + 1 < nv && !rc; v++) {
            const int64_t mnx = X[v] < X[v + 1] ? X[v] : X[v + 1], mxx = X[v] < X[v + 1] ? X[v + 1] : X[v];
            const int64_t mny = Y[v] < Y[v + 1] ? Y[v] : Y[v + 1], mxy = Y[v] < Y[v + 1] ? Y[v + 1] : Y[v];
            /* cells (i, j) with iW <= mxx and (i+1)W >= mnx, same for j */
            for (int64_t j = ceildiv(mny, g.W) - 1; j <= floordiv(mxy, g.W) && !rc; j++)
                for (int64_t i = ceildiv(mnx, g.W) - 1; i <= floordiv(mxx, g.W) && !rc; i++)
                    if (seg_meets_box(X[v], Y[v], X[v + 1], Y[v + 1], i * g.W, j * g.W, (i + 1) * g.W,
                                      (j + 1) * g.W, 0))
                        rc = vec_push(&ids, orc_hilbert(g.order, (uint64_t)i, (uint64_t)j));
        }
        free(X); free(Y);
        if (!rc) {
            qsort(ids.v, ids.n, sizeof(uint64_t), cmp_u64);
            for (int64_t t = 0; t < ids.n && !rc; t++)
                if (t == 0 || ids.v[t] != ids.v[t - 1]) rc = vec_push(&all, ids.v[t]);
        }
        free(ids.v);
        C->off[k + 1] = (uint64_t)all.n;
    }
    if (!rc) {
        C->ids = (uint32_t *)malloc(sizeof(uint32_t) * (all.n ? all.n : 1));
        if (!C->ids) rc = ORC_E_NOMEM;
        for (int64_t t = 0; t < all.n && !rc; t++) C->ids[t] = (uint32_t)all.v[t];
    }
    free(all.v);
    if (rc) { free(C->off); free(C->ids); free(C); return rc; }
    *out = C;
    return ORC_OK;
}

int64_t orc_cells_size(const orc_cells *C) { return (int64_t)C->off[C->n]; }

void orc_cells_export(const orc_cells *C, uint64_t *off, uint32_t *ids)
{
    memcpy(off, C->off, sizeof(uint64_t) * (C->n + 1));
    memcpy(ids, C->ids, sizeof(uint32_t) * C->off[C->n]);
}

void orc_cells_free(orc_cells *C)
{
    if (!C) return;
    free(C->off); free(C->ids); free(C);
}

/*
 * Polygon-linestring join (Sec. 4.3.3): Alg. 2's IntervalJoin with the
 * linestring's cell ids as intervals [c, c+1):
 *   A(p) against the cells: no overlap -> true negative;
 *   F(p) against the cells: an overlap -> true hit;
 *   otherwise indecisive.
 */
int orc_filter_linestrings(const uint64_t *oAp, const uint32_t *sAp, const uint32_t *eAp,
                           const uint64_t *oFp, const uint32_t *sFp, const uint32_t *eFp,
                           const uint64_t *offL, const uint32_t *ids,
                           const uint32_t *pp, const uint32_t *ll, int64_t P, uint8_t *verdict)
{
    for (int64_t q = 0; q < P; q++) {
        const uint64_t c0 = offL[ll[q]], c1 = offL[ll[q] + 1], m = c1 - c0;
        uint32_t *cs = (uint32_t *)malloc(sizeof(uint32_t) * (m ? m : 1));
        uint32_t *ce = (uint32_t *)malloc(sizeof(uint32_t) * (m ? m : 1));
        if (!cs || !ce) { free(cs); free(ce); return ORC_E_NOMEM; }
        for (uint64_t t = 0; t < m; t++) { cs[t] = ids[c0 + t]; ce[t] = ids[c0 + t] + 1; }
        const uint64_t a0 = oAp[pp[q]], a1 = oAp[pp[q] + 1], f0 = oFp[pp[q]], f1 = oFp[pp[q] + 1];
        if (!orc_interval_join(sAp + a0, eAp + a0, a1 - a0, cs, ce, m, NULL, NULL)) verdict[q] = V_TN;
        else if (orc_interval_join(sFp + f0, eFp + f0, f1 - f0, cs, ce, m, NULL, NULL)) verdict[q] = V_TH;
        else verdict[q] = V_IND;
        free(cs); free(ce);
    }
    return ORC_OK;
}

/*
 * Different granularity (Sec. 5.3): R's lists at order NR, S's at order NS
 * on the same data space.  The finer side's A-intervals are mapped to the
 * coarser grid by the paper's equation, a' = [a_start >> n, (a_end - 1) >> n]
 * (inclusive end; n = 2 |NR - NS| bits), and the mapped intervals, which may
 * now touch or overlap, are merged into maximal half-open runs.  Then:
 *   mapped A against the coarse A-list: no overlap -> true negative;
 *   mapped A against the coarse F-list: an overlap -> true hit (the only
 *   one of AF / FA kept: a Full interval at the finer order says nothing
 *   about the coarser one);
 *   otherwise indecisive.
 * With NR == NS nothing is mapped and Alg. 2 runs unchanged.
 */
static uint64_t coarsen(const uint32_t *as, const uint32_t *ae, uint64_t n, int bits, uint32_t *os, uint32_t *oe)
{
    uint64_t k = 0;
    for (uint64_t i = 0; i < n; i++) {
        const uint32_t s = as[i] >> bits, e = ((ae[i] - 1) >> bits) + 1;   /* half-open form of a' */
        if (k && s <= oe[k - 1]) { if (e > oe[k - 1]) oe[k - 1] = e; }   /* touches or overlaps: merge */
        else { os[k] = s; oe[k] = e; k++; }
    }
    return k;
}

int orc_filter_mixed(const uint64_t *oAr, const uint32_t *sAr, const uint32_t *eAr,
                     const uint64_t *oFr, const uint32_t *sFr, const uint32_t *eFr, int NR,
                     const uint64_t *oAs, const uint32_t *sAs, const uint32_t *eAs,
                     const uint64_t *oFs, const uint32_t *sFs, const uint32_t *eFs, int NS,
                     const uint32_t *r, const uint32_t *s, int64_t P, uint8_t *verdict)
{
    if (NR == NS) {
        filter_job_t J;
        J.oAr = oAr; J.oFr = oFr; J.oAs = oAs; J.oFs = oFs;
        J.sAr = sAr; J.eAr = eAr; J.sFr = sFr; J.eFr = eFr;
        J.sAs = sAs; J.eAs = eAs; J.sFs = sFs; J.eFs = eFs;
        for (int64_t p = 0; p < P; p++) verdict[p] = april_pair(&J, r[p], s[p], NULL);
        return ORC_OK;
    }
    const int r_fine = NR > NS, bits = 2 * (r_fine ? NR - NS : NS - NR);
    for (int64_t p = 0; p < P; p++) {
        /* fine side: its A-list; coarse side: A- and F-lists */
        const uint64_t *oAf = r_fine ? oAr : oAs, *oAc = r_fine ? oAs : oAr, *oFc = r_fine ? oFs : oFr;
        const uint32_t *sAf = r_fine ? sAr : sAs, *eAf = r_fine ? eAr : eAs;
        const uint32_t *sAc = r_fine ? sAs : sAr, *eAc = r_fine ? eAs : eAr;
        const uint32_t *sFc = r_fine ? sFs : sFr, *eFc = r_fine ? eFs : eFr;
        const uint32_t of = r_fine ? r[p] : s[p], oc = r_fine ? s[p] : r[p];
        const uint64_t a0 = oAf[of], n = oAf[of + 1] - a0;
        uint32_t *ms = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
        uint32_t *me = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
        if (!ms || !me) { free(ms); free(me); return ORC_E_NOMEM; }
        const uint64_t m = coarsen(sAf + a0, eAf + a0, n, bits, ms, me);
        const uint64_t c0 = oAc[oc], c1 = oAc[oc + 1], f0 = oFc[oc], f1 = oFc[oc + 1];
        if (!orc_interval_join(ms, me, m, sAc + c0, eAc + c0, c1 - c0, NULL, NULL)) verdict[p] = V_TN;
        else if (orc_interval_join(ms, me, m, sFc + f0, eFc + f0, f1 - f0, NULL, NULL)) verdict[p] = V_TH;
        else verdict[p] = V_IND;
        free(ms); free(me);
    }
    return ORC_OK;
}

/*
 * Exact geometry for the variants' soundness checks.
 *   orc_point_in_closed_polygon: the point lies inside or on the boundary.
 *   orc_linestring_meets_polygon: a segment meets an edge (closed), or the
 *   linestring's first vertex lies inside the polygon.
 */
int orc_point_in_closed_polygon(const double *poly, int64_t nv, double px, double py)
{
    int64_t *x = (int64_t *)malloc(sizeof(int64_t) * 2 * nv);
    if (!x) return ORC_E_NOMEM;
    int64_t *y = x + nv, X, Y;
    int rc = lattice(px, 0.0, &X);
    if (!rc) rc = lattice(py, 0.0, &Y);
    for (int64_t k = 0; k < nv && !rc; k++) {
        rc = lattice(poly[2 * k], 0.0, &x[k]);
        if (!rc) rc = lattice(poly[2 * k + 1], 0.0, &y[k]);
    }
    if (rc) { free(x); return rc; }
    int on = 0;
    for (int64_t k = 0; k < nv && !on; k++) {
        const int64_t k2 = (k + 1 == nv) ? 0 : k + 1;
        on = orient(x[k], y[k], x[k2], y[k2], X, Y) == 0 && on_seg(x[k], y[k], x[k2], y[k2], X, Y);
    }
    const int in = on || crossing_inside(x, y, nv, NULL, nv, X, Y);
    free(x);
    return in;
}

int orc_linestring_meets_polygon(const double *line, int64_t nl, const double *poly, int64_t np)
{
    int64_t *lx = (int64_t *)malloc(sizeof(int64_t) * 2 * nl), *px = (int64_t *)malloc(sizeof(int64_t) * 2 * np);
    if (!lx || !px) { free(lx); free(px); return ORC_E_NOMEM; }
    int64_t *ly = lx + nl, *py = px + np;
    int rc = ORC_OK;
    for (int64_t k = 0; k < nl && !rc; k++) { rc = lattice(line[2 * k], 0.0, &lx[k]); if (!rc) rc = lattice(line[2 * k + 1], 0.0, &ly[k]); }
    for (int64_t k = 0; k < np && !rc; k++) { rc = lattice(poly[2 * k], 0.0, &px[k]); if (!rc) rc = lattice(poly[2 * k + 1], 0.0, &py[k]); }
    if (rc) { free(lx); free(px); return rc; }
    int hit = 0;
    for (int64_t a = 0; a + 1 < nl && !hit; a++)
        for (int64_t b = 0; b < np && !hit; b++) {
            const int64_t b2 = (b + 1 == np) ? 0 : b + 1;
            hit = seg_seg(lx[a], ly[a], lx[a + 1], ly[a + 1], px[b], py[b], px[b2], py[b2]);
        }
    if (!hit) hit = crossing_inside(px, py, np, NULL, np, lx[0], ly[0]);
    free(lx); free(px);
    return hit;
}
