/*
 * oracle.c -- plain, slow CPU reference of the SPH hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU baseline of the
 * benchmark do.  It shares no code, header or table with the HIP library.
 *
 * Floating point is FP64 except where a decision must be taken in the storage
 * precision (the neighbour criterion, App. E), which is then evaluated in
 * float or double exactly as written, with FMA contraction disabled (the file
 * is built with -ffp-contract=off).
 *
 * Parity pins are the test-suite's job; every function below is written as
 * the plain definition of what the paper's algorithms compute:
 *   Morton encoding ........ App. B.1 (interleave X0 Y0 Z0 X1 ...)
 *   delta operator ......... App. B, Eq. delta_ab (clz of XOR)
 *   stable sort ............ App. D.1 "Sort by key" (ties by original index)
 *   keep mask + reduction .. App. C, Alg. 1 (Jacobi passes) + compaction
 *   radix tree ............. App. B.7 and its Table (recursive top-down split)
 *   cell boxes ............. App. B.6 Eqs. lowboundbox/highboundbox, App. E h_max
 *   neighbour sets ......... App. E, object-object criterion, chi-extended
 *   h / rho root ........... App. F Eq. rhoh, Sect. 2.1 Eqs. SPHmass/rhosphsum
 *   Omega .................. Sect. 2.1 Eq. sphomega
 *   force, du/dt ........... Sect. 2.1 Eqs. sphvel, sphuint (+ AV, conductivity)
 *   leapfrog, CFL .......... App. G.1 (KDK) and G.2 (timestep)
 *   kernel family .......... Sect. 2.1.1: M4, M5, M6 B-splines, Wendland C2, C4, C6
 *   corrector re-run ....... App. G.1 (Eqs. deltavi, cvleapfrog), CFL multiplier
 *   shock detection ........ App. G (Eq. evolalphaanalytic and the implicit update)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_BITS 21
#define ORC_GRID (1u << ORC_BITS)

int orc_version(void) { return 1; }

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* Morton codes (App. B.1): map to [0,1), sample a 2^21 grid per axis,  */
/* interleave bit by bit with X as the most significant of each triple. */
/* ------------------------------------------------------------------ */
static uint32_t quantize_bits(double v, double lo, double scale, int bits)
{
    double t = (v - lo) * scale;
    double f = floor(t);
    double top = (double)((1u << bits) - 1u);
    if (!(f >= 0.0)) f = 0.0;                     /* also catches NaN */
    if (f > top) f = top;                         /* 1 is excluded */
    return (uint32_t)f;
}

static uint32_t quantize(double v, double lo, double scale)
{
    return quantize_bits(v, lo, scale, ORC_BITS);
}

/* Interleave `bits`-bit integers into a 3*bits-bit code in the low bits:  */
/* triple k (k = 0 the most significant) holds X_k Y_k Z_k, X first.       */
uint64_t orc_interleave_bits(uint32_t X, uint32_t Y, uint32_t Z, int bits)
{
    uint64_t key = 0;
    for (int k = 0; k < bits; ++k) {
        int src = bits - 1 - k;                   /* X_k is bit (bits-1-k) of X */
        int dst = 3 * (bits - 1 - k);             /* triple k sits at bits dst+2..dst */
        key |= (uint64_t)((X >> src) & 1u) << (dst + 2);
        key |= (uint64_t)((Y >> src) & 1u) << (dst + 1);
        key |= (uint64_t)((Z >> src) & 1u) << (dst + 0);
    }
    return key;
}

uint64_t orc_interleave(uint32_t X, uint32_t Y, uint32_t Z)
{
    return orc_interleave_bits(X, Y, Z, ORC_BITS);
}

void orc_deinterleave(uint64_t key, uint32_t *X, uint32_t *Y, uint32_t *Z)
{
    uint32_t a = 0, b = 0, c = 0;
    for (int k = 0; k < ORC_BITS; ++k) {
        int src = ORC_BITS - 1 - k;
        int dst = 3 * (ORC_BITS - 1 - k);
        a |= (uint32_t)((key >> (dst + 2)) & 1u) << src;
        b |= (uint32_t)((key >> (dst + 1)) & 1u) << src;
        c |= (uint32_t)((key >> (dst + 0)) & 1u) << src;
    }
    *X = a; *Y = b; *Z = c;
}

/* Morton codes with `bits` per axis (App. B.1 with beta = bits; 10 bits  */
/* per axis gives the 30-bit codes of Sect. 5.2.1).                        */
void orc_morton_bits(int64_t n, const double *x, const double *y, const double *z,
                     const double *lo, const double *hi, int bits, uint64_t *key)
{
    double s[3];
    for (int d = 0; d < 3; ++d) s[d] = (double)(1u << bits) / (hi[d] - lo[d]);
    for (int64_t i = 0; i < n; ++i) {
        uint32_t X = quantize_bits(x[i], lo[0], s[0], bits);
        uint32_t Y = quantize_bits(y[i], lo[1], s[1], bits);
        uint32_t Z = quantize_bits(z[i], lo[2], s[2], bits);
        key[i] = orc_interleave_bits(X, Y, Z, bits);
    }
}

void orc_morton(int64_t n, const double *x, const double *y, const double *z,
                const double *lo, const double *hi, uint64_t *key)
{
    double s[3];
    for (int d = 0; d < 3; ++d) s[d] = (double)ORC_GRID / (hi[d] - lo[d]);
    for (int64_t i = 0; i < n; ++i) {
        uint32_t X = quantize(x[i], lo[0], s[0]);
        uint32_t Y = quantize(y[i], lo[1], s[1]);
        uint32_t Z = quantize(z[i], lo[2], s[2]);
        key[i] = orc_interleave(X, Y, Z);
    }
}

/* ------------------------------------------------------------------ */
/* delta operator (Eq. delta_ab): length of the longest common prefix.  */
/* ------------------------------------------------------------------ */
static int delta64(uint64_t a, uint64_t b)
{
    uint64_t v = a ^ b;
    if (v == 0) return 64;
    int c = 0;
    while (!(v & (1ull << 63))) { v <<= 1; ++c; }
    return c;
}

int orc_delta(uint64_t a, uint64_t b) { return delta64(a, b); }

/* ------------------------------------------------------------------ */
/* Sort by key, keeping the original index (ties: original order).     */
/* ------------------------------------------------------------------ */
typedef struct { uint64_t k; uint32_t i; } kv_t;

static int kv_cmp(const void *pa, const void *pb)
{
    const kv_t *a = (const kv_t *)pa, *b = (const kv_t *)pb;
    if (a->k < b->k) return -1;
    if (a->k > b->k) return 1;
    return (a->i > b->i) - (a->i < b->i);
}

void orc_sort(int64_t n, const uint64_t *key, uint32_t *eps, uint64_t *mu)
{
    kv_t *t = (kv_t *)malloc(sizeof(kv_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) { t[i].k = key[i]; t[i].i = (uint32_t)i; }
    qsort(t, (size_t)n, sizeof(kv_t), kv_cmp);
    for (int64_t i = 0; i < n; ++i) { eps[i] = t[i].i; mu[i] = t[i].k; }
    free(t);
}

/* ------------------------------------------------------------------ */
/* Keep mask, reduction passes and compaction (App. C, Alg. 1).        */
/* Each pass reads the previous mask and writes a new one.  A missing   */
/* neighbour (outside [0,n)) contributes a prefix length of -1.         */
/* ------------------------------------------------------------------ */
int64_t orc_leaves(int64_t n, const uint64_t *mu, int n_red,
                   uint8_t *xi, uint32_t *id, uint64_t *mu_leaf)
{
    if (n <= 0) { id[0] = 0; return 0; }
    for (int64_t i = 0; i < n; ++i) xi[i] = (i == 0) ? 1 : (mu[i] != mu[i - 1]);
    uint8_t *old = (uint8_t *)malloc((size_t)n);
    for (int pass = 0; pass < n_red; ++pass) {
        memcpy(old, xi, (size_t)n);
        for (int64_t i = 0; i < n; ++i) {
            if (!old[i]) { xi[i] = 0; continue; }
            int64_t im1 = i - 1;
            while (im1 >= 0 && !old[im1]) --im1;
            int64_t im2 = im1 - 1;
            while (im2 >= 0 && !old[im2]) --im2;
            int64_t ip1 = i + 1;
            while (ip1 < n && !old[ip1]) ++ip1;
            int d0 = (ip1 < n) ? delta64(mu[i], mu[ip1]) : -1;
            int dm1 = (im1 >= 0) ? delta64(mu[im1], mu[i]) : -1;
            int dm2 = (im1 >= 0 && im2 >= 0) ? delta64(mu[im2], mu[im1]) : -1;
            int removable = (d0 < dm1) && (dm2 < dm1);
            xi[i] = removable ? 0 : 1;
        }
    }
    free(old);
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (xi[i]) { id[k] = (uint32_t)i; mu_leaf[k] = mu[i]; ++k; }
    }
    id[k] = (uint32_t)n;
    return k;
}

/* ------------------------------------------------------------------ */
/* Binary radix tree, plain top-down definition (App. B.7, its Table):  */
/* a leaf range [f,l] is split after the last code whose bit at the     */
/* first differing position (counted from the MSB) is 0.  The node of   */
/* a range is numbered by its end that touches the split of its parent: */
/* left child = split index g, right child = g+1; a child is a leaf     */
/* (flag 1) when its range holds a single leaf.  endrange = other end.  */
/* parent[] is indexed by node: internal nodes 0..nl-2, then leaves.    */
/* ------------------------------------------------------------------ */
typedef struct {
    const uint64_t *mu;
    uint32_t *lc, *rc, *er, *par;
    uint8_t *lf, *rf;
    int64_t ni;
} tree_ctx;

static void split_range(tree_ctx *t, int64_t node, int64_t f, int64_t l)
{
    int p = delta64(t->mu[f], t->mu[l]);
    uint64_t bit = 1ull << (63 - p);
    int64_t g = f;
    while (g + 1 <= l && !(t->mu[g + 1] & bit)) ++g;
    t->er[node] = (uint32_t)((node == f) ? l : f);
    t->lc[node] = (uint32_t)g;
    t->rc[node] = (uint32_t)(g + 1);
    t->lf[node] = (uint8_t)(g == f);
    t->rf[node] = (uint8_t)(g + 1 == l);
    if (g == f) t->par[t->ni + g] = (uint32_t)node;
    else { t->par[g] = (uint32_t)node; split_range(t, g, f, g); }
    if (g + 1 == l) t->par[t->ni + g + 1] = (uint32_t)node;
    else { t->par[g + 1] = (uint32_t)node; split_range(t, g + 1, g + 1, l); }
}

void orc_radix_tree(int64_t nl, const uint64_t *mu_leaf, uint32_t *lchild,
                    uint32_t *rchild, uint8_t *lflag, uint8_t *rflag,
                    uint32_t *endrange, uint32_t *parent)
{
    if (nl <= 0) return;
    tree_ctx t = { mu_leaf, lchild, rchild, endrange, parent, lflag, rflag, nl - 1 };
    if (nl == 1) { parent[0] = 0xffffffffu; return; }
    parent[0] = 0xffffffffu;
    split_range(&t, 0, 0, nl - 1);
}

/* Leaf range [first,last] of every node (internal, then leaves). */
static void node_ranges(int64_t nl, const uint32_t *er, int64_t *first, int64_t *last)
{
    int64_t ni = nl - 1;
    for (int64_t i = 0; i < ni; ++i) {
        int64_t a = i, b = er[i];
        first[i] = a < b ? a : b;
        last[i] = a < b ? b : a;
    }
    for (int64_t k = 0; k < nl; ++k) { first[ni + k] = k; last[ni + k] = k; }
}

/* ------------------------------------------------------------------ */
/* Integer prefix boxes (App. B.6): the prefix class of a node is all   */
/* codes sharing its first `len` bits; p0 = code & mask, p1 = p0 | ~mask */
/* decoded into inclusive integer corners.  For an internal node len is */
/* delta(first, last); a leaf takes its parent's length + 1 (the whole  */
/* domain for a single-leaf tree).                                      */
/* ------------------------------------------------------------------ */
void orc_prefix_boxes(int64_t nl, const uint64_t *mu_leaf, const uint32_t *endrange,
                      const uint32_t *parent, uint32_t *box /* 6 per node */,
                      int32_t *plen /* per node */)
{
    int64_t ni = nl - 1, nn = 2 * nl - 1;
    int64_t *first = (int64_t *)malloc(sizeof(int64_t) * (size_t)nn);
    int64_t *last = (int64_t *)malloc(sizeof(int64_t) * (size_t)nn);
    node_ranges(nl, endrange, first, last);
    for (int64_t v = 0; v < nn; ++v) {
        int len;
        if (v < ni) len = delta64(mu_leaf[first[v]], mu_leaf[last[v]]);
        else if (nl == 1) len = 0;
        else {
            int64_t p = parent[v];
            len = delta64(mu_leaf[first[p]], mu_leaf[last[p]]) + 1;
        }
        /* bit 63 is never set by the encoding; it always belongs to the prefix */
        uint64_t mask = (len >= 64) ? ~0ull : ~((~0ull) >> len);
        uint64_t code = mu_leaf[first[v]];
        uint64_t p0 = code & mask;
        uint64_t p1 = p0 | (~mask & 0x7fffffffffffffffull);
        uint32_t X0, Y0, Z0, X1, Y1, Z1;
        orc_deinterleave(p0, &X0, &Y0, &Z0);
        orc_deinterleave(p1, &X1, &Y1, &Z1);
        box[6 * v + 0] = X0; box[6 * v + 1] = Y0; box[6 * v + 2] = Z0;
        box[6 * v + 3] = X1; box[6 * v + 4] = Y1; box[6 * v + 5] = Z1;
        plen[v] = len;
    }
    free(first); free(last);
}

/* Tight boxes and h_max of every node by brute force over its particles. */
void orc_tight_boxes(int64_t nl, const uint32_t *id, const uint32_t *endrange,
                     const double *xs, const double *ys, const double *zs,
                     const double *hs, double *bmin /*3/node*/, double *bmax,
                     double *hmax)
{
    int64_t nn = 2 * nl - 1;
    int64_t *first = (int64_t *)malloc(sizeof(int64_t) * (size_t)nn);
    int64_t *last = (int64_t *)malloc(sizeof(int64_t) * (size_t)nn);
    node_ranges(nl, endrange, first, last);
    for (int64_t v = 0; v < nn; ++v) {
        double lo[3] = { INFINITY, INFINITY, INFINITY };
        double hi[3] = { -INFINITY, -INFINITY, -INFINITY };
        double hm = -INFINITY;
        for (int64_t j = id[first[v]]; j < (int64_t)id[last[v] + 1]; ++j) {
            double p[3] = { xs[j], ys[j], zs[j] };
            for (int d = 0; d < 3; ++d) {
                if (p[d] < lo[d]) lo[d] = p[d];
                if (p[d] > hi[d]) hi[d] = p[d];
            }
            if (hs[j] > hm) hm = hs[j];
        }
        for (int d = 0; d < 3; ++d) { bmin[3 * v + d] = lo[d]; bmax[3 * v + d] = hi[d]; }
        hmax[v] = hm;
    }
    free(first); free(last);
}

/* ------------------------------------------------------------------ */
/* Uniform cell grid used to enumerate candidate pairs.  It is only a   */
/* search structure: every accepted pair is decided by the exact test. */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    int nc[3];
    double lo[3], L[3], cs[3];
    int periodic;
    int64_t *start;  /* ncell+1 */
    int64_t *idx;    /* n */
} grid_t;

static int64_t cell_of(const grid_t *g, double v, int d)
{
    int64_t c = (int64_t)floor((v - g->lo[d]) / g->cs[d]);
    if (c < 0) c = 0;
    if (c >= g->nc[d]) c = g->nc[d] - 1;
    return c;
}

static void grid_build(grid_t *g, int64_t n, const double *x, const double *y,
                       const double *z, const double *lo, const double *hi,
                       int periodic, double cell)
{
    g->n = n;
    g->periodic = periodic;
    const double *P[3] = { x, y, z };
    for (int d = 0; d < 3; ++d) {
        double a = lo[d], b = hi[d];
        if (!periodic) {     /* isolated: the data extent */
            a = INFINITY; b = -INFINITY;
            for (int64_t i = 0; i < n; ++i) { if (P[d][i] < a) a = P[d][i]; if (P[d][i] > b) b = P[d][i]; }
            if (n == 0) { a = 0; b = 1; }
        }
        g->lo[d] = a;
        g->L[d] = b - a;
        int nc = (int)floor(g->L[d] / cell);
        if (nc < 1) nc = 1;
        if (nc > 512) nc = 512;
        g->nc[d] = nc;
        g->cs[d] = (g->L[d] > 0) ? g->L[d] / nc : 1.0;
        if (!periodic && g->L[d] <= 0) g->cs[d] = 1.0;
    }
    int64_t ncell = (int64_t)g->nc[0] * g->nc[1] * g->nc[2];
    g->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    g->idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *cid = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = (cell_of(g, x[i], 0) * g->nc[1] + cell_of(g, y[i], 1)) * g->nc[2]
                    + cell_of(g, z[i], 2);
        cid[i] = c;
        g->start[c + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) g->start[c + 1] += g->start[c];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncell + 1));
    memcpy(fill, g->start, sizeof(int64_t) * (size_t)(ncell + 1));
    for (int64_t i = 0; i < n; ++i) g->idx[fill[cid[i]]++] = i;
    free(fill);
    free(cid);
}

static void grid_free(grid_t *g) { free(g->start); free(g->idx); }

/* Visit every particle whose cell lies within `radius` of (px,py,pz).  */
/* The callback gets candidate index b; duplicates are impossible since */
/* each cell is visited at most once.                                   */
typedef void (*visit_fn)(void *user, int64_t b);

static void grid_visit(const grid_t *g, double px, double py, double pz,
                       double radius, visit_fn fn, void *user)
{
    double p[3] = { px, py, pz };
    int64_t c0[3], span[3];
    int all[3];
    for (int d = 0; d < 3; ++d) {
        int64_t reach = (int64_t)ceil(radius / g->cs[d]) + 1;
        c0[d] = cell_of(g, p[d], d);
        all[d] = (2 * reach + 1 >= g->nc[d]);
        span[d] = reach;
    }
    int64_t lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        if (all[d]) { lo[d] = 0; hi[d] = g->nc[d] - 1; }
        else { lo[d] = c0[d] - span[d]; hi[d] = c0[d] + span[d]; }
        if (!g->periodic && !all[d]) {
            if (lo[d] < 0) lo[d] = 0;
            if (hi[d] > g->nc[d] - 1) hi[d] = g->nc[d] - 1;
        }
    }
    for (int64_t a = lo[0]; a <= hi[0]; ++a) {
        int64_t ca = ((a % g->nc[0]) + g->nc[0]) % g->nc[0];
        for (int64_t b = lo[1]; b <= hi[1]; ++b) {
            int64_t cb = ((b % g->nc[1]) + g->nc[1]) % g->nc[1];
            for (int64_t c = lo[2]; c <= hi[2]; ++c) {
                int64_t cc = ((c % g->nc[2]) + g->nc[2]) % g->nc[2];
                int64_t cell = (ca * g->nc[1] + cb) * g->nc[2] + cc;
                for (int64_t k = g->start[cell]; k < g->start[cell + 1]; ++k) fn(user, g->idx[k]);
            }
        }
    }
}

/* Minimum-image separation r_a - r_b in FP64. */
static void sep64(const double *L, int periodic, double xa, double ya, double za,
                  double xb, double yb, double zb, double *d)
{
    d[0] = xa - xb; d[1] = ya - yb; d[2] = za - zb;
    if (periodic) {
        for (int k = 0; k < 3; ++k) {
            if (d[k] > 0.5 * L[k]) d[k] -= L[k];
            else if (d[k] < -0.5 * L[k]) d[k] += L[k];
        }
    }
}

/* ------------------------------------------------------------------ */
/* Neighbour sets in the storage precision T (App. E, object-object     */
/* criterion with the chi-extended cache radius):                      */
/*   dx = x_b - x_a;  periodic: once, dx -= L if dx > L/2, += L if     */
/*   dx < -L/2;  r2 = fma(dz, dz, fma(dy, dy, dx*dx)) (fused, each      */
/*   rounded once: the paper fixes no rounding for this sum);           */
/*   rc = (T)(R*chi) * max(h_a, h_b);  accept iff r2 < rc*rc.           */
/* Indices are positions in the given arrays, listed in ascending      */
/* order; the particle itself is included.                              */
/* ------------------------------------------------------------------ */
#define DEFINE_NEIGH(T, SUF, FMA)                                               \
static int crit_##SUF(const T *x, const T *y, const T *z, const T *h,          \
                      int periodic, const T *Lt, const T *Ht, T rkc,           \
                      int64_t a, int64_t b)                                    \
{                                                                              \
    T dx = x[b] - x[a], dy = y[b] - y[a], dz = z[b] - z[a];                    \
    if (periodic) {                                                            \
        if (dx > Ht[0]) dx = dx - Lt[0]; else if (dx < -Ht[0]) dx = dx + Lt[0];\
        if (dy > Ht[1]) dy = dy - Lt[1]; else if (dy < -Ht[1]) dy = dy + Lt[1];\
        if (dz > Ht[2]) dz = dz - Lt[2]; else if (dz < -Ht[2]) dz = dz + Lt[2];\
    }                                                                          \
    T r2 = FMA(dz, dz, FMA(dy, dy, dx * dx));                                  \
    T hm = h[a] > h[b] ? h[a] : h[b];                                          \
    T rc = rkc * hm;                                                           \
    T rc2 = rc * rc;                                                           \
    return r2 < rc2;                                                           \
}                                                                              \
typedef struct { int64_t *buf; int64_t cnt, cap; const T *x, *y, *z, *h;       \
                 int periodic; const T *Lt, *Ht; T rkc; int64_t a; } nctx_##SUF;\
static void visit_##SUF(void *u, int64_t b)                                    \
{                                                                              \
    nctx_##SUF *c = (nctx_##SUF *)u;                                           \
    if (crit_##SUF(c->x, c->y, c->z, c->h, c->periodic, c->Lt, c->Ht, c->rkc,  \
                   c->a, b)) {                                                 \
        if (c->cnt == c->cap) {                                                \
            c->cap = c->cap ? 2 * c->cap : 256;                                \
            c->buf = (int64_t *)realloc(c->buf, sizeof(int64_t) * (size_t)c->cap);\
        }                                                                      \
        c->buf[c->cnt++] = b;                                                  \
    }                                                                          \
}                                                                              \
int64_t orc_neigh_##SUF(int64_t n, const T *x, const T *y, const T *z,         \
                        const T *h, const double *lo, const double *hi,        \
                        int periodic, double r_kern_chi, int brute,            \
                        int64_t nt, const int64_t *targets,                    \
                        uint64_t *offsets, uint32_t *list, int64_t cap)        \
{                                                                              \
    /* targets == NULL: every particle (nt = n); else the listed ones */       \
    if (!targets) nt = n;                                                      \
    T Lt[3], Ht[3];                                                            \
    double lo_d[3], hi_d[3];                                                   \
    for (int d = 0; d < 3; ++d) {                                              \
        Lt[d] = (T)(hi[d] - lo[d]); Ht[d] = (T)(0.5 * (hi[d] - lo[d]));        \
        lo_d[d] = lo[d]; hi_d[d] = hi[d];                                      \
    }                                                                          \
    T rkc = (T)r_kern_chi;                                                     \
    double *xd = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));   \
    double *yd = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));   \
    double *zd = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));   \
    double hmax = 0;                                                           \
    for (int64_t i = 0; i < n; ++i) {                                          \
        xd[i] = x[i]; yd[i] = y[i]; zd[i] = z[i];                              \
        if ((double)h[i] > hmax) hmax = h[i];                                  \
    }                                                                          \
    double rsearch = r_kern_chi * hmax * 1.001 + 1e-12;                        \
    grid_t g;                                                                  \
    grid_build(&g, n, xd, yd, zd, lo_d, hi_d, periodic, brute ? 1e300 : rsearch);\
    int64_t *cnt = (int64_t *)calloc((size_t)(nt > 0 ? nt : 1), sizeof(int64_t));\
    int64_t **lists = (int64_t **)calloc((size_t)(nt > 0 ? nt : 1), sizeof(int64_t *));\
    _Pragma("omp parallel for schedule(dynamic, 256)")                         \
    for (int64_t t = 0; t < nt; ++t) {                                         \
        const int64_t a = targets ? targets[t] : t;                            \
        nctx_##SUF c = { NULL, 0, 0, x, y, z, h, periodic, Lt, Ht, rkc, a };   \
        if (brute) { for (int64_t b = 0; b < n; ++b) visit_##SUF(&c, b); }     \
        else grid_visit(&g, xd[a], yd[a], zd[a], rsearch, visit_##SUF, &c);    \
        /* ascending order: insertion sort of the (short) list */              \
        for (int64_t i = 1; i < c.cnt; ++i) {                                  \
            int64_t v = c.buf[i], j = i - 1;                                   \
            while (j >= 0 && c.buf[j] > v) { c.buf[j + 1] = c.buf[j]; --j; }   \
            c.buf[j + 1] = v;                                                  \
        }                                                                      \
        cnt[t] = c.cnt; lists[t] = c.buf;                                      \
    }                                                                          \
    int64_t total = 0;                                                         \
    for (int64_t t = 0; t < nt; ++t) { offsets[t] = (uint64_t)total; total += cnt[t]; }\
    offsets[nt] = (uint64_t)total;                                             \
    if (total <= cap) {                                                        \
        for (int64_t t = 0; t < nt; ++t)                                       \
            for (int64_t k = 0; k < cnt[t]; ++k)                               \
                list[offsets[t] + k] = (uint32_t)lists[t][k];                  \
    }                                                                          \
    for (int64_t t = 0; t < nt; ++t) free(lists[t]);                           \
    free(lists); free(cnt); free(xd); free(yd); free(zd); grid_free(&g);       \
    return total <= cap ? total : -total;                                      \
}

DEFINE_NEIGH(float, f32, fmaf)
DEFINE_NEIGH(double, f64, fma)

/* ------------------------------------------------------------------ */
/* Kernel functions f(q) of Sect. 2.1.1 (Eq. rhosphsum): the Schoenberg  */
/* B-splines M4, M5, M6 and the Wendland functions C2, C4, C6, in their  */
/* textbook forms with support radius R (q in units of h) and the 3-D    */
/* normalisation C_norm such that int W dV = 1:                         */
/*   M4: R = 2,   C = 1/pi,       f = 1 - 3/2 q^2 + 3/4 q^3 (q<1),     */
/*                                    (2-q)^3/4 (1<=q<2)                */
/*   M5: R = 5/2, C = 1/(20 pi),  f = (5/2-q)^4 - 5 (3/2-q)^4           */
/*                                    + 10 (1/2-q)^4, each term only    */
/*                                    while its bracket is positive     */
/*   M6: R = 3,   C = 1/(120 pi), f = (3-q)^5 - 6 (2-q)^5 + 15 (1-q)^5, */
/*                                    same rule                         */
/*   C2: R = 2,   C = 21/(16 pi),   f = (1-q/2)^4 (1 + 2q)              */
/*   C4: R = 2,   C = 495/(256 pi), f = (1-q/2)^6 (1 + 3q + 35/12 q^2)  */
/*   C6: R = 2,   C = 1365/(512 pi),f = (1-q/2)^8 (1 + 4q + 25/4 q^2    */
/*                                    + 4 q^3)                          */
/* f'(q) is the derivative of each piece, written out by the product    */
/* and chain rules.                                                     */
/* ------------------------------------------------------------------ */
enum { K_M4 = 0, K_M5 = 1, K_M6 = 2, K_C2 = 3, K_C4 = 4, K_C6 = 5, K_NUM = 6 };

static double pos(double t) { return t > 0.0 ? t : 0.0; }

static double kern_R(int k)
{
    switch (k) {
    case K_M5: return 2.5;
    case K_M6: return 3.0;
    default: return 2.0;
    }
}

static double kern_C(int k)
{
    switch (k) {
    case K_M4: return 1.0 / M_PI;
    case K_M5: return 1.0 / (20.0 * M_PI);
    case K_M6: return 1.0 / (120.0 * M_PI);
    case K_C2: return 21.0 / (16.0 * M_PI);
    case K_C4: return 495.0 / (256.0 * M_PI);
    default:   return 1365.0 / (512.0 * M_PI);
    }
}

static double kern_f(int k, double q)
{
    if (!(q < kern_R(k))) return 0.0;
    switch (k) {
    case K_M4:
        if (q < 1.0) return 1.0 - 1.5 * q * q + 0.75 * q * q * q;
        { double t = 2.0 - q; return 0.25 * t * t * t; }
    case K_M5: {
        double a = pos(2.5 - q), b = pos(1.5 - q), c = pos(0.5 - q);
        return pow(a, 4) - 5.0 * pow(b, 4) + 10.0 * pow(c, 4);
    }
    case K_M6: {
        double a = pos(3.0 - q), b = pos(2.0 - q), c = pos(1.0 - q);
        return pow(a, 5) - 6.0 * pow(b, 5) + 15.0 * pow(c, 5);
    }
    case K_C2: { double t = 1.0 - 0.5 * q; return pow(t, 4) * (1.0 + 2.0 * q); }
    case K_C4: { double t = 1.0 - 0.5 * q; return pow(t, 6) * (1.0 + 3.0 * q + 35.0 / 12.0 * q * q); }
    default:   { double t = 1.0 - 0.5 * q;
                 return pow(t, 8) * (1.0 + 4.0 * q + 6.25 * q * q + 4.0 * q * q * q); }
    }
}

static double kern_df(int k, double q)
{
    if (!(q < kern_R(k))) return 0.0;
    switch (k) {
    case K_M4:
        if (q < 1.0) return -3.0 * q + 2.25 * q * q;
        { double t = 2.0 - q; return -0.75 * t * t; }
    case K_M5: {
        double a = pos(2.5 - q), b = pos(1.5 - q), c = pos(0.5 - q);
        return -4.0 * pow(a, 3) + 20.0 * pow(b, 3) - 40.0 * pow(c, 3);
    }
    case K_M6: {
        double a = pos(3.0 - q), b = pos(2.0 - q), c = pos(1.0 - q);
        return -5.0 * pow(a, 4) + 30.0 * pow(b, 4) - 75.0 * pow(c, 4);
    }
    case K_C2: {   /* d/dq [t^4 (1+2q)], dt/dq = -1/2 */
        double t = 1.0 - 0.5 * q;
        return 4.0 * pow(t, 3) * (-0.5) * (1.0 + 2.0 * q) + pow(t, 4) * 2.0;
    }
    case K_C4: {
        double t = 1.0 - 0.5 * q;
        return 6.0 * pow(t, 5) * (-0.5) * (1.0 + 3.0 * q + 35.0 / 12.0 * q * q)
               + pow(t, 6) * (3.0 + 35.0 / 6.0 * q);
    }
    default: {
        double t = 1.0 - 0.5 * q;
        return 8.0 * pow(t, 7) * (-0.5) * (1.0 + 4.0 * q + 6.25 * q * q + 4.0 * q * q * q)
               + pow(t, 8) * (4.0 + 12.5 * q + 12.0 * q * q);
    }
    }
}

int orc_kernel_count(void) { return K_NUM; }
double orc_kernel_support(int k) { return kern_R(k); }
double orc_kernel_norm(int k) { return kern_C(k); }
double orc_kernel_f(int k, double q) { return kern_f(k, q); }
double orc_kernel_df(int k, double q) { return kern_df(k, q); }
double orc_m4_f(double q) { return kern_f(K_M4, q); }
double orc_m4_df(double q) { return kern_df(K_M4, q); }

/* W(r,h) = C_norm f(r/h) / h^3 (Eq. rhosphsum). */
static double W(int k, double r, double h) { return kern_C(k) * kern_f(k, r / h) / (h * h * h); }
/* dW/dh at fixed r = -C_norm (3 f + q f') / h^4. */
static double dWdh(int k, double r, double h)
{
    double q = r / h;
    return -kern_C(k) * (3.0 * kern_f(k, q) + q * kern_df(k, q)) / (h * h * h * h);
}
/* F(r,h) = rhat . grad_a W = C_norm f'(q) / h^4. */
static double Fgrad(int k, double r, double h) { return kern_C(k) * kern_df(k, r / h) / (h * h * h * h); }

/* ------------------------------------------------------------------ */
/* Smoothing length (App. F): h_a is the root of                       */
/*    g(h) = sum_b m W(r_ab, h) - m (hfact/h)^3                          */
/* over all b within 2h.  Bracket by geometric expansion from the       */
/* initial h, then safeguarded Newton/bisection to 1e-13 relative.      */
/* rho_a = m (hfact/h_a)^3 and                                          */
/* Omega_a = 1 + h_a/(3 rho_a) sum_b m dW_ab(h_a)/dh_a (Eq. sphomega    */
/* with dh/drho = -h/(3 rho) from Eq. rhoh).                            */
/* flags: bit0 no bracket / no convergence, bit1 >1 sign change seen.   */
/* ------------------------------------------------------------------ */
typedef struct { double *r; int64_t cnt, cap; const double *x, *y, *z; const double *L;
                 int periodic; int64_t a; double rmax; } rctx_t;

static void visit_r(void *u, int64_t b)
{
    rctx_t *c = (rctx_t *)u;
    double d[3];
    sep64(c->L, c->periodic, c->x[c->a], c->y[c->a], c->z[c->a], c->x[b], c->y[b], c->z[b], d);
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (r < c->rmax) {
        if (c->cnt == c->cap) {
            c->cap = c->cap ? 2 * c->cap : 256;
            c->r = (double *)realloc(c->r, sizeof(double) * (size_t)c->cap);
        }
        c->r[c->cnt++] = r;
    }
}

static void g_eval(int kern, const double *r, int64_t n, double h, double m, double hfact,
                   double *g, double *dg)
{
    double s = 0, ds = 0;
    for (int64_t k = 0; k < n; ++k) { s += W(kern, r[k], h); ds += dWdh(kern, r[k], h); }
    double hf3 = hfact * hfact * hfact;
    *g = m * s - m * hf3 / (h * h * h);
    *dg = m * ds + 3.0 * m * hf3 / (h * h * h * h);
}

void orc_density(int64_t n, const double *x, const double *y, const double *z,
                 const double *h0, const double *lo, const double *hi, int periodic,
                 double m, double hfact, int kern, int64_t nt, const int64_t *targets,
                 double *h_out, double *rho_out, double *omega_out, int32_t *flags)
{
    const double R = kern_R(kern);
    double L[3];
    for (int d = 0; d < 3; ++d) L[d] = hi[d] - lo[d];
    double hmax = 0;
    for (int64_t i = 0; i < n; ++i) if (h0[i] > hmax) hmax = h0[i];
    grid_t g;
    grid_build(&g, n, x, y, z, lo, hi, periodic, R * hmax);
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t a = targets ? targets[t] : t;
        int32_t flag = 0;
        double reach = 2.0 * R * h0[a];
        rctx_t c = { NULL, 0, 0, x, y, z, L, periodic, a, 0 };
        double hroot = h0[a];
        for (int attempt = 0; attempt < 8; ++attempt) {
            c.cnt = 0; c.rmax = reach;
            grid_visit(&g, x[a], y[a], z[a], reach, visit_r, &c);
            /* bracket: g(lo) < 0 < g(hi), both with R h <= reach */
            double hlo = h0[a], hhi = h0[a], glo, ghi, dg;
            double hcap = reach / R;
            g_eval(kern, c.r, c.cnt, hlo, m, hfact, &glo, &dg);
            int ok = 1;
            if (glo > 0) {                   /* root below: shrink */
                ghi = glo; hhi = hlo;
                while (glo > 0) {
                    hhi = hlo; ghi = glo; hlo /= 1.2;
                    g_eval(kern, c.r, c.cnt, hlo, m, hfact, &glo, &dg);
                    if (hlo < 1e-12 * h0[a]) { ok = 0; break; }
                }
            } else {                         /* root above: grow */
                g_eval(kern, c.r, c.cnt, hhi, m, hfact, &ghi, &dg);
                while (ghi <= 0) {
                    hlo = hhi; glo = ghi; hhi *= 1.2;
                    if (hhi > hcap) { ok = -1; break; }
                    g_eval(kern, c.r, c.cnt, hhi, m, hfact, &ghi, &dg);
                }
            }
            if (ok == -1) { reach *= 2.0; continue; }
            if (!ok) { flag |= 1; break; }
            /* sign changes on a coarse grid inside the bracket */
            {
                int changes = 0; double gp = glo;
                for (int k = 1; k <= 16; ++k) {
                    double hk = hlo + (hhi - hlo) * k / 16.0, gk, dk;
                    g_eval(kern, c.r, c.cnt, hk, m, hfact, &gk, &dk);
                    if ((gk > 0) != (gp > 0)) ++changes;
                    gp = gk;
                }
                if (changes > 1) flag |= 2;
            }
            double hcur = 0.5 * (hlo + hhi);
            int conv = 0;
            for (int it = 0; it < 200; ++it) {
                double gv, dv;
                g_eval(kern, c.r, c.cnt, hcur, m, hfact, &gv, &dv);
                if (gv > 0) hhi = hcur; else hlo = hcur;
                double hn = (dv != 0) ? hcur - gv / dv : 0.5 * (hlo + hhi);
                if (!(hn > hlo && hn < hhi)) hn = 0.5 * (hlo + hhi);
                if (fabs(hn - hcur) <= 1e-13 * hcur || (hhi - hlo) <= 1e-14 * hcur) {
                    hcur = hn; conv = 1; break;
                }
                hcur = hn;
            }
            if (!conv) flag |= 1;
            hroot = hcur;
            break;
        }
        double rho = m * (hfact / hroot) * (hfact / hroot) * (hfact / hroot);
        double ds = 0;
        c.cnt = 0; c.rmax = R * hroot;
        grid_visit(&g, x[a], y[a], z[a], R * hroot, visit_r, &c);
        for (int64_t k = 0; k < c.cnt; ++k) ds += dWdh(kern, c.r[k], hroot);
        h_out[t] = hroot;
        rho_out[t] = rho;
        omega_out[t] = 1.0 + hroot / (3.0 * rho) * m * ds;
        if (flags) flags[t] = flag;
        free(c.r);
    }
    grid_free(&g);
}

/* Plain SPH density sum at a given h (Eq. SPHmass), for the pins. */
void orc_density_sum(int64_t n, const double *x, const double *y, const double *z,
                     const double *h, const double *lo, const double *hi, int periodic,
                     double m, int kern, int64_t nt, const int64_t *targets, double *rho_sum,
                     double *dsum_dh)
{
    const double R = kern_R(kern);
    double L[3];
    for (int d = 0; d < 3; ++d) L[d] = hi[d] - lo[d];
    double hmax = 0;
    for (int64_t i = 0; i < n; ++i) if (h[i] > hmax) hmax = h[i];
    grid_t g;
    grid_build(&g, n, x, y, z, lo, hi, periodic, R * hmax);
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t a = targets ? targets[t] : t;
        rctx_t c = { NULL, 0, 0, x, y, z, L, periodic, a, R * h[a] };
        grid_visit(&g, x[a], y[a], z[a], R * h[a], visit_r, &c);
        double s = 0, ds = 0;
        for (int64_t k = 0; k < c.cnt; ++k) { s += W(kern, c.r[k], h[a]); ds += dWdh(kern, c.r[k], h[a]); }
        rho_sum[t] = m * s;
        if (dsum_dh) dsum_dh[t] = m * ds;
        free(c.r);
    }
    grid_free(&g);
}

/* ------------------------------------------------------------------ */
/* Force and energy equations (Sect. 2.1, Eqs. sphvel and sphuint with  */
/* the AV terms q^a_ab, q^b_ab and the conductivity Lambda_cond), over  */
/* b != a with 0 < r_ab < 2 max(h_a, h_b):                              */
/*   dv_a/dt = -sum_b m [ (P_a+q^a)/(rho_a^2 Om_a) F(h_a)                */
/*                      + (P_b+q^b)/(rho_b^2 Om_b) F(h_b) ] rhat_ab     */
/*   du_a/dt =  sum_b m (P_a+q^a)/(rho_a^2 Om_a) w F(h_a) + Lambda_a    */
/*   Lambda_a = sum_b m beta_u vsig_u (u_a-u_b) (F(h_a)/(Om_a rho_a)     */
/*                                            + F(h_b)/(Om_b rho_b))/2  */
/* with w = v_ab . rhat_ab, vsig = alpha c_s + beta |w| (alpha per      */
/* particle when an array is given, Sect. 2.1.1 alpha_a^AV),            */
/* q = -rho vsig w / 2 when w < 0, vsig_u = sqrt(|P_a-P_b|/((rho_a+rho_b)/2)),*/
/* P = (gamma-1) rho u, c_s = sqrt(gamma P / rho).                      */
/* Also returned: vsig_dt (max signal speed, floor c_s) and the scales  */
/* S_a = sum of the magnitudes of the per-pair terms, used to judge the */
/* error of a sum whose terms cancel.                                    */
/* ------------------------------------------------------------------ */
typedef struct { int64_t *b; int64_t cnt, cap; const double *x, *y, *z; const double *L;
                 int periodic; int64_t a; double rmax; } bctx_t;

static void visit_b(void *u, int64_t b)
{
    bctx_t *c = (bctx_t *)u;
    double d[3];
    sep64(c->L, c->periodic, c->x[c->a], c->y[c->a], c->z[c->a], c->x[b], c->y[b], c->z[b], d);
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (r2 < c->rmax * c->rmax) {
        if (c->cnt == c->cap) {
            c->cap = c->cap ? 2 * c->cap : 256;
            c->b = (int64_t *)realloc(c->b, sizeof(int64_t) * (size_t)c->cap);
        }
        c->b[c->cnt++] = b;
    }
}

void orc_force(int64_t n, const double *x, const double *y, const double *z,
               const double *vx, const double *vy, const double *vz, const double *u,
               const double *h, const double *rho, const double *omega,
               const double *lo, const double *hi, int periodic, double m,
               double gamma, double alpha, const double *alpha_arr, double beta, double beta_u,
               int kern, int64_t nt, const int64_t *targets,
               double *ax, double *ay, double *az, double *dudt, double *vsig_dt,
               double *scale_a, double *scale_u)
{
    const double R = kern_R(kern);
    double L[3];
    for (int d = 0; d < 3; ++d) L[d] = hi[d] - lo[d];
    double hmax = 0;
    for (int64_t i = 0; i < n; ++i) if (h[i] > hmax) hmax = h[i];
    grid_t g;
    grid_build(&g, n, x, y, z, lo, hi, periodic, R * hmax);
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t a = targets ? targets[t] : t;
        double reach = R * (h[a] > hmax ? h[a] : hmax);
        bctx_t c = { NULL, 0, 0, x, y, z, L, periodic, a, reach };
        grid_visit(&g, x[a], y[a], z[a], reach, visit_b, &c);
        double Pa = (gamma - 1.0) * rho[a] * u[a];
        double ca = sqrt(gamma * Pa / rho[a]);
        double Aa = Pa / (rho[a] * rho[a] * omega[a]);
        double acc[3] = { 0, 0, 0 }, du = 0, lam = 0, sa = 0, su = 0, vmax = ca;
        for (int64_t k = 0; k < c.cnt; ++k) {
            int64_t b = c.b[k];
            if (b == a) continue;
            double d[3];
            sep64(L, periodic, x[a], y[a], z[a], x[b], y[b], z[b], d);
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            double hm = h[a] > h[b] ? h[a] : h[b];
            if (!(r > 0.0) || !(r < R * hm)) continue;
            double rh[3] = { d[0] / r, d[1] / r, d[2] / r };
            double vab[3] = { vx[a] - vx[b], vy[a] - vy[b], vz[a] - vz[b] };
            double w = vab[0] * rh[0] + vab[1] * rh[1] + vab[2] * rh[2];
            double Pb = (gamma - 1.0) * rho[b] * u[b];
            double cb = sqrt(gamma * Pb / rho[b]);
            double al_a = alpha_arr ? alpha_arr[a] : alpha, al_b = alpha_arr ? alpha_arr[b] : alpha;
            double vsa = al_a * ca + beta * fabs(w);
            double vsb = al_b * cb + beta * fabs(w);
            double qa = (w < 0) ? -0.5 * rho[a] * vsa * w : 0.0;
            double qb = (w < 0) ? -0.5 * rho[b] * vsb * w : 0.0;
            double Fa = Fgrad(kern, r, h[a]), Fb = Fgrad(kern, r, h[b]);
            double ta = (Pa + qa) / (rho[a] * rho[a] * omega[a]) * Fa;
            double tb = (Pb + qb) / (rho[b] * rho[b] * omega[b]) * Fb;
            double f = m * (ta + tb);
            acc[0] -= f * rh[0]; acc[1] -= f * rh[1]; acc[2] -= f * rh[2];
            sa += fabs(f);
            double e = m * (Pa + qa) / (rho[a] * rho[a] * omega[a]) * w * Fa;
            double vsu = sqrt(fabs(Pa - Pb) / (0.5 * (rho[a] + rho[b])));
            double l = m * beta_u * vsu * (u[a] - u[b]) * 0.5
                       * (Fa / (omega[a] * rho[a]) + Fb / (omega[b] * rho[b]));
            du += e; lam += l;
            su += fabs(e) + fabs(l);
            if (vsa > vmax) vmax = vsa;
        }
        (void)Aa;
        ax[t] = acc[0]; ay[t] = acc[1]; az[t] = acc[2];
        dudt[t] = du + lam;
        if (vsig_dt) vsig_dt[t] = vmax;
        if (scale_a) scale_a[t] = sa;
        if (scale_u) scale_u[t] = su;
        free(c.b);
    }
    grid_free(&g);
}

/* ------------------------------------------------------------------ */
/* CFL timestep (App. G.2): min over a of                               */
/*   min(C_cour h_a / vsig_a, C_force sqrt(h_a / |a_a|)).               */
/* ------------------------------------------------------------------ */
double orc_cfl(int64_t n, const double *h, const double *vsig, const double *ax,
               const double *ay, const double *az, double c_cour, double c_force)
{
    double dt = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        double t1 = (vsig[i] > 0) ? c_cour * h[i] / vsig[i] : INFINITY;
        double am = sqrt(ax[i] * ax[i] + ay[i] * ay[i] + az[i] * az[i]);
        double t2 = (am > 0) ? c_force * sqrt(h[i] / am) : INFINITY;
        double t = t1 < t2 ? t1 : t2;
        if (t < dt) dt = t;
    }
    return dt;
}

/* ------------------------------------------------------------------ */
/* SPH gradient of a vector field (the estimate used by the shock       */
/* detector, with the same kernel gradient and Omega as the force):     */
/*   (d_j f_i)_a = -1/(rho_a Omega_a) sum_b m (f_a - f_b)_i              */
/*                 (rhat_ab)_j F_ab(h_a)                                 */
/* over b within R h_a.  out: 9 per target, row-major [i][j] = d_j f_i.  */
/* ------------------------------------------------------------------ */
void orc_gradient(int64_t n, const double *x, const double *y, const double *z,
                  const double *fx, const double *fy, const double *fz, const double *h,
                  const double *rho, const double *omega, const double *lo, const double *hi,
                  int periodic, double m, int kern, int64_t nt, const int64_t *targets,
                  double *out)
{
    const double R = kern_R(kern);
    double L[3];
    for (int d = 0; d < 3; ++d) L[d] = hi[d] - lo[d];
    double hmax = 0;
    for (int64_t i = 0; i < n; ++i) if (h[i] > hmax) hmax = h[i];
    grid_t g;
    grid_build(&g, n, x, y, z, lo, hi, periodic, R * hmax);
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t a = targets ? targets[t] : t;
        bctx_t c = { NULL, 0, 0, x, y, z, L, periodic, a, R * h[a] };
        grid_visit(&g, x[a], y[a], z[a], R * h[a], visit_b, &c);
        double G[3][3] = { { 0 } };
        const double *F[3] = { fx, fy, fz };
        for (int64_t k = 0; k < c.cnt; ++k) {
            int64_t b = c.b[k];
            double d[3];
            sep64(L, periodic, x[a], y[a], z[a], x[b], y[b], z[b], d);
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (!(r > 0.0)) continue;
            double Fa = Fgrad(kern, r, h[a]);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    G[i][j] += m * (F[i][a] - F[i][b]) * (d[j] / r) * Fa;
        }
        double s = -1.0 / (rho[a] * omega[a]);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) out[9 * t + 3 * i + j] = s * G[i][j];
        free(c.b);
    }
    grid_free(&g);
}

/* ------------------------------------------------------------------ */
/* Parameters of the step.                                              */
/* ------------------------------------------------------------------ */
typedef struct {
    double hfact, gamma, alpha, beta, beta_u, c_cour, c_force;
    int kernel;
    /* corrector re-runs (App. G.1): while max_a |dv_a| > eps_v v_rms and  */
    /* fewer than max_rerun re-runs were made, the force is evaluated       */
    /* again with v* <- v^{n+1} (u* <- u^{n+1}) and the corrector re-applied */
    double eps_v;
    int max_rerun;
    /* shock-detection switch (App. G, Shock detection)                     */
    int alpha_switch;
    double alpha_min, alpha_max, sigma_decay;
} orc_params;

/* ------------------------------------------------------------------ */
/* Shock detector and the implicit alpha update (App. G, Eq.             */
/* evolalphaanalytic and the two lines after it), for every particle,    */
/* at the new positions with h, rho, Omega of the density pass:          */
/*   grad v* and grad a^n by orc_gradient, div v = tr(grad v),           */
/*   curl v from its antisymmetric part,                                  */
/*   d(div v)/dt = div a - sum_ij (d_j v_i)(d_i v_j),                      */
/*   xi = (div v)^2 / ((div v)^2 + |curl v|^2) (0 when both vanish),      */
/*   A = xi max(-d(div v)/dt, 0),                                         */
/*   alpha_loc = max(alpha_min, alpha_max 10 h^2 A / (10 h^2 A + c_s^2)), */
/*   tau = h / (sigma_decay c_s),                                         */
/*   alpha^{n+1} = max((alpha^n + alpha_loc dt/tau) / (1 + dt/tau),      */
/*                     alpha_loc).                                        */
/* c_s = sqrt(gamma (gamma-1) u*).  The paper gives the update and      */
/* refers to Phantom for alpha_loc and tau; the forms above are this     */
/* implementation's reading (Cullen-Dehnen switch with a Balsara-type    */
/* limiter).  Outputs (optional): alpha_loc, div v, d(div v)/dt.         */
/* ------------------------------------------------------------------ */
void orc_alpha_switch(int64_t n, const double *x, const double *y, const double *z,
                      const double *vx, const double *vy, const double *vz,
                      const double *ax, const double *ay, const double *az, const double *u,
                      const double *h, const double *rho, const double *omega,
                      const double *alpha_n, const double *lo, const double *hi, int periodic,
                      double m, const orc_params *P, double dt, double *alpha_out,
                      double *aloc_out, double *divv_out, double *ddiv_out)
{
    size_t sz = sizeof(double) * 9 * (size_t)(n > 0 ? n : 1);
    double *gv = malloc(sz), *ga = malloc(sz);
    orc_gradient(n, x, y, z, vx, vy, vz, h, rho, omega, lo, hi, periodic, m, P->kernel, n, NULL, gv);
    orc_gradient(n, x, y, z, ax, ay, az, h, rho, omega, lo, hi, periodic, m, P->kernel, n, NULL, ga);
    for (int64_t a = 0; a < n; ++a) {
        const double *V = gv + 9 * a, *A = ga + 9 * a;   /* [i][j] = d_j f_i */
        double divv = V[0] + V[4] + V[8];
        double diva = A[0] + A[4] + A[8];
        double cx = V[3 * 2 + 1] - V[3 * 1 + 2];          /* d_y v_z - d_z v_y */
        double cy = V[3 * 0 + 2] - V[3 * 2 + 0];          /* d_z v_x - d_x v_z */
        double cz = V[3 * 1 + 0] - V[3 * 0 + 1];          /* d_x v_y - d_y v_x */
        double vv = 0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) vv += V[3 * i + j] * V[3 * j + i];
        double ddiv = diva - vv;
        double d2 = divv * divv, c2 = cx * cx + cy * cy + cz * cz;
        double xi = (d2 + c2 > 0) ? d2 / (d2 + c2) : 0.0;
        double Ash = xi * (ddiv < 0 ? -ddiv : 0.0);
        double cs = sqrt(P->gamma * (P->gamma - 1.0) * u[a]);
        double hh = 10.0 * h[a] * h[a] * Ash;
        double aloc = (hh + cs * cs > 0) ? P->alpha_max * hh / (hh + cs * cs) : 0.0;
        if (aloc < P->alpha_min) aloc = P->alpha_min;
        double al = aloc;
        if (cs > 0) {
            double x_ = dt * P->sigma_decay * cs / h[a];   /* dt / tau */
            al = (alpha_n[a] + aloc * x_) / (1.0 + x_);
            if (al < aloc) al = aloc;
        } else if (alpha_n[a] > aloc) {
            al = alpha_n[a];                               /* tau infinite: no decay */
        }
        alpha_out[a] = al;
        if (aloc_out) aloc_out[a] = aloc;
        if (divv_out) divv_out[a] = divv;
        if (ddiv_out) ddiv_out[a] = ddiv;
    }
    free(gv); free(ga);
}

/* CFL multiplier (App. G, CFL multiplier): halved after a step whose     */
/* corrector had to be re-run, else relaxed towards 1:                    */
/*   lambda^{n+1} = (1 + lambda_stiff lambda^n) / (1 + lambda_stiff).     */
double orc_cfl_multiplier(double lam, int rerun, double lambda_stiff)
{
    if (rerun) return 0.5 * lam;
    return (1.0 + lambda_stiff * lam) / (1.0 + lambda_stiff);
}

/* ------------------------------------------------------------------ */
/* One kick-drift-kick step with a fixed dt (App. G.1), u integrated    */
/* like v.  In: state at t^n (x,v,u,h, alpha if the switch is on) and    */
/* the derivatives a^n, du^n.  Out (in place): state at t^{n+1}, h^{n+1}, */
/* rho, Omega, a^{n+1}, du^{n+1}, alpha^{n+1}.  diag[0] = max |dv|,       */
/* diag[1] = sum |dv|^2, diag[2] = sum |v^{n+1}|^2, diag[3] = CFL dt of    */
/* the new state, diag[4] = corrector re-runs made (of the last           */
/* corrector: dv = v^{n+1} - v*).                                         */
/* ------------------------------------------------------------------ */
void orc_step(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
              double *vz, double *u, double *h, double *ax, double *ay, double *az,
              double *dudt, double *rho, double *omega, double *alpha,
              const double *lo, const double *hi, int periodic, double m,
              const orc_params *P, double dt, double *diag)
{
    double L[3];
    for (int d = 0; d < 3; ++d) L[d] = hi[d] - lo[d];
    size_t sz = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *vhx = malloc(sz), *vhy = malloc(sz), *vhz = malloc(sz), *uh = malloc(sz);
    double *vsx = malloc(sz), *vsy = malloc(sz), *vsz = malloc(sz), *us = malloc(sz);
    double *nax = malloc(sz), *nay = malloc(sz), *naz = malloc(sz), *ndu = malloc(sz);
    double *hn = malloc(sz), *vs = malloc(sz), *al = malloc(sz);
    double *P3[3] = { x, y, z };
    for (int64_t i = 0; i < n; ++i) {
        vhx[i] = vx[i] + 0.5 * dt * ax[i];
        vhy[i] = vy[i] + 0.5 * dt * ay[i];
        vhz[i] = vz[i] + 0.5 * dt * az[i];
        uh[i] = u[i] + 0.5 * dt * dudt[i];
        x[i] += dt * vhx[i]; y[i] += dt * vhy[i]; z[i] += dt * vhz[i];
        if (periodic) {
            for (int d = 0; d < 3; ++d) {
                if (P3[d][i] >= hi[d]) P3[d][i] -= L[d];
                if (P3[d][i] < lo[d]) P3[d][i] += L[d];
            }
        }
        vsx[i] = vhx[i] + 0.5 * dt * ax[i];
        vsy[i] = vhy[i] + 0.5 * dt * ay[i];
        vsz[i] = vhz[i] + 0.5 * dt * az[i];
        us[i] = uh[i] + 0.5 * dt * dudt[i];
    }
    orc_density(n, x, y, z, h, lo, hi, periodic, m, P->hfact, P->kernel, n, NULL, hn, rho, omega,
                NULL);
    const double *alpha_use = NULL;
    if (P->alpha_switch && alpha) {
        /* alpha^{n+1} from v*, grad v*, grad a^n at the new positions */
        orc_alpha_switch(n, x, y, z, vsx, vsy, vsz, ax, ay, az, us, hn, rho, omega, alpha, lo, hi,
                         periodic, m, P, dt, al, NULL, NULL, NULL);
        for (int64_t i = 0; i < n; ++i) alpha[i] = al[i];
        alpha_use = alpha;
    }
    double dvmax = 0, dvsum = 0, vsum = 0;
    int rerun = 0;
    for (;;) {
        orc_force(n, x, y, z, vsx, vsy, vsz, us, hn, rho, omega, lo, hi, periodic, m,
                  P->gamma, P->alpha, alpha_use, P->beta, P->beta_u, P->kernel, n, NULL,
                  nax, nay, naz, ndu, vs, NULL, NULL);
        dvmax = 0; dvsum = 0; vsum = 0;
        for (int64_t i = 0; i < n; ++i) {
            /* v^{n+1} = v^{n+1/2} + dt/2 a^{n+1};  dv = v^{n+1} - v* */
            double nvx = vhx[i] + 0.5 * dt * nax[i];
            double nvy = vhy[i] + 0.5 * dt * nay[i];
            double nvz = vhz[i] + 0.5 * dt * naz[i];
            double dvx = nvx - vsx[i], dvy = nvy - vsy[i], dvz = nvz - vsz[i];
            vx[i] = nvx; vy[i] = nvy; vz[i] = nvz;
            u[i] = uh[i] + 0.5 * dt * ndu[i];
            double dv = sqrt(dvx * dvx + dvy * dvy + dvz * dvz);
            if (dv > dvmax) dvmax = dv;
            dvsum += dv * dv;
            vsum += vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i];
        }
        /* reversibility check: max |dv| against eps_v times the rms velocity */
        int ok = !(P->eps_v > 0) || dvmax <= P->eps_v * sqrt(vsum / (double)(n > 0 ? n : 1));
        if (ok || rerun >= P->max_rerun) break;
        ++rerun;
        for (int64_t i = 0; i < n; ++i) {   /* v* <- v^{n+1}, u* <- u^{n+1} */
            vsx[i] = vx[i]; vsy[i] = vy[i]; vsz[i] = vz[i]; us[i] = u[i];
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        ax[i] = nax[i]; ay[i] = nay[i]; az[i] = naz[i]; dudt[i] = ndu[i];
        h[i] = hn[i];
    }
    if (diag) {
        diag[0] = dvmax; diag[1] = dvsum; diag[2] = vsum;
        diag[3] = orc_cfl(n, h, vs, ax, ay, az, P->c_cour, P->c_force);
        diag[4] = rerun;
    }
    free(vhx); free(vhy); free(vhz); free(uh); free(vsx); free(vsy); free(vsz); free(us);
    free(nax); free(nay); free(naz); free(ndu); free(hn); free(vs); free(al);
}
