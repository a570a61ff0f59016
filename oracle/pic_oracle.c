/*
 * pic_oracle.c -- plain, serial, FP64 reference of the spacetree PIC hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Tests, the smoke check and the CPU-baseline leg
 * of the benchmark call this; the product library never does.  It shares no
 * code, header or table with the GPU library: it rebuilds everything it needs
 * from the refinement masks it is given.
 *
 * What it computes (paper: "Two Particle-in-Grid Realisations on Spacetrees"):
 *   - the k=3 spacetree over the periodic unit box (Sec. 4): root, children
 *     by three cuts per axis, leaves = unrefined cells;
 *   - cell ownership: a particle belongs to the leaf that covers its position
 *     (PIT, Sec. 5.1, Theorem 1) or to the vertex of that leaf whose dual cell
 *     covers it (PIDT, Sec. 4.2 "Storing particles", Sec. 5.2, Theorem 2);
 *   - bins ordered along the Peano space-filling curve (Sec. 4.2 storage remark);
 *   - d-linear restriction R and its transpose (Sec. 3 steps 1 and 3, and the
 *     d-linear shape-function remark): rho = sum_i R(x_i), E_i = R^T(x_i) E;
 *   - the push dv/dt = (q/m) E, dx/dt = v (Sec. 3 step 4) as leapfrog.
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - a particle's cell coordinate is y = fl(x * 3^L) (one rounding); cells
 *     are half-open [i, i+1) in y, and y == 3^L is taken as the last cell;
 *   - PIDT owner = the corner of the particle's leaf nearest to y in the max
 *     norm, ties to the upper corner;
 *   - Peano digit rule: base-3 digits most significant first, axes
 *     interleaved 0..d-1; digit of axis k is complemented (2-digit) iff the
 *     digits already emitted for all other axes sum to an odd number;
 *   - PIT bin key  = peano_l(a) * 3^(d(L-l)) * 64 + l for a level-l leaf a;
 *     PIDT bin key = peano_L(J') * 64 + l with J' = (b*s + (3^L-1)/2) mod 3^L
 *     for the level-l vertex b (s = 3^(L-l)), i.e. the dual grid is indexed on
 *     the half-cell-shifted lattice on which dual cells nest (odd k);
 *   - order inside a bin after a re-bin: particles that stayed, in their old
 *     order, then particles that arrived, in their old order;
 *   - leapfrog with v at half steps; x wraps periodically into [0,1).
 *
 * Parity unpinned (fixed by these readings, not by anything the paper or the
 * mathematics determines): the PIDT owner's tie-break at coarse-fine
 * interfaces, the order inside a bin, the exact PIDT key on adaptive trees,
 * and the PIDT lift count beyond the mechanism the tests check.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MAXD 3

typedef struct {
    int level;
    int64_t a[MAXD];      /* integer coordinates at its own level */
    int32_t child;        /* index of the first of 3^d children (lexicographic slots), -1 for a leaf */
    int32_t leaf;         /* leaf rank in Peano order, -1 for refined cells */
} onode;

typedef struct {
    int dim, L;
    int64_t S;            /* 3^L */
    int64_t n_nodes, cap_nodes;
    onode *nodes;
    int64_t n_leaves;
    int32_t *leaf_node;   /* rank -> node */
    uint64_t *leaf_key;
    int64_t n_vtx;
    int64_t *vtx_lin;     /* sorted linear positions sum p_k S^k */
    int32_t *leaf_vtx;    /* n_leaves * 2^d */
    int64_t n_pidt;
    uint64_t *pidt_key;   /* ascending */
    int32_t *pidt_level;
    int64_t *pidt_b;      /* n_pidt * dim, vertex coordinates at its level */
    int32_t *pidt_vtx;    /* the vertex id at that position */
    int32_t *leaf_pidt;   /* n_leaves * 2^d: bin of each corner at the leaf's level */
} otree;

static int64_t ipow3(int e) { int64_t r = 1; while (e-- > 0) r *= 3; return r; }

/* ---------------------------------------------------------------- Peano index */
uint64_t orc_peano(int dim, int L, const int64_t *coord)
{
    /* digit i (most significant first) of axis k, complemented iff the digits
       already emitted for the other axes have an odd sum */
    int64_t seen[MAXD] = {0, 0, 0};
    uint64_t key = 0;
    for (int i = 0; i < L; ++i) {
        int64_t p = ipow3(L - 1 - i);
        for (int k = 0; k < dim; ++k) {
            int64_t digit = (coord[k] / p) % 3;
            int64_t others = 0;
            for (int j = 0; j < dim; ++j)
                if (j != k) others += seen[j];
            int64_t e = (others % 2) ? 2 - digit : digit;
            key = key * 3 + (uint64_t)e;
            seen[k] += digit;
        }
    }
    return key;
}

/* ---------------------------------------------------------------- tree build */
static int64_t add_node(otree *t, int level, const int64_t *a)
{
    if (t->n_nodes == t->cap_nodes) {
        t->cap_nodes = t->cap_nodes ? 2 * t->cap_nodes : 1024;
        t->nodes = (onode *)realloc(t->nodes, (size_t)t->cap_nodes * sizeof(onode));
    }
    onode *n = &t->nodes[t->n_nodes];
    n->level = level;
    for (int k = 0; k < MAXD; ++k) n->a[k] = k < t->dim ? a[k] : 0;
    n->child = -1;
    n->leaf = -1;
    return t->n_nodes++;
}

static int64_t lex_index(int dim, int64_t n, const int64_t *a)
{
    int64_t r = 0, m = 1;
    for (int k = 0; k < dim; ++k) { r += a[k] * m; m *= n; }
    return r;
}

/* Recursively refine node `id` following the masks. */
static void build_rec(otree *t, int64_t id, const uint8_t *masks, const int64_t *mask_off)
{
    int level = t->nodes[id].level;
    if (level >= t->L) return;
    int64_t a[MAXD];
    for (int k = 0; k < MAXD; ++k) a[k] = t->nodes[id].a[k];
    int64_t n_l = ipow3(level);
    if (!masks[mask_off[level] + lex_index(t->dim, n_l, a)]) return;
    int nch = (int)ipow3(t->dim);
    int64_t first = t->n_nodes;
    for (int slot = 0; slot < nch; ++slot) {
        int64_t c[MAXD] = {0, 0, 0};
        int r = slot;
        for (int k = 0; k < t->dim; ++k) { c[k] = 3 * a[k] + r % 3; r /= 3; }
        add_node(t, level + 1, c);
    }
    t->nodes[id].child = (int32_t)first;
    for (int slot = 0; slot < nch; ++slot) build_rec(t, first + slot, masks, mask_off);
}

static uint64_t leaf_key_of(const otree *t, const onode *n)
{
    uint64_t p = orc_peano(t->dim, n->level, n->a);
    uint64_t span = (uint64_t)ipow3(t->dim * (t->L - n->level));
    return (p * span) * 64u + (uint64_t)n->level;
}

static uint64_t pidt_key_of(const otree *t, int level, const int64_t *b)
{
    int64_t s = ipow3(t->L - level);
    int64_t J[MAXD] = {0, 0, 0};
    for (int k = 0; k < t->dim; ++k) J[k] = (b[k] * s + (t->S - 1) / 2) % t->S;
    return orc_peano(t->dim, t->L, J) * 64u + (uint64_t)level;
}

typedef struct { uint64_t key; int64_t idx; } kv;

static int cmp_kv(const void *x, const void *y)
{
    const kv *a = (const kv *)x, *b = (const kv *)y;
    if (a->key < b->key) return -1;
    if (a->key > b->key) return 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

static int cmp_i64(const void *x, const void *y)
{
    int64_t a = *(const int64_t *)x, b = *(const int64_t *)y;
    return (a > b) - (a < b);
}

static int64_t find_i64(const int64_t *arr, int64_t n, int64_t v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (arr[mid] < v) lo = mid + 1; else hi = mid;
    }
    return (lo < n && arr[lo] == v) ? lo : -1;
}

static int64_t find_u64(const uint64_t *arr, int64_t n, uint64_t v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (arr[mid] < v) lo = mid + 1; else hi = mid;
    }
    return (lo < n && arr[lo] == v) ? lo : -1;
}

void orc_tree_free(void *h)
{
    otree *t = (otree *)h;
    if (!t) return;
    free(t->nodes); free(t->leaf_node); free(t->leaf_key); free(t->vtx_lin);
    free(t->leaf_vtx); free(t->pidt_key); free(t->pidt_level); free(t->pidt_b);
    free(t->pidt_vtx); free(t->leaf_pidt);
    free(t);
}

void *orc_tree_new(int dim, int L, const uint8_t *masks)
{
    if (dim < 2 || dim > 3 || L < 0 || dim * L > 36) return NULL;
    otree *t = (otree *)calloc(1, sizeof(otree));
    t->dim = dim;
    t->L = L;
    t->S = ipow3(L);
    int64_t mask_off[40];
    mask_off[0] = 0;
    for (int l = 0; l < L; ++l) mask_off[l + 1] = mask_off[l] + ipow3(dim * l);
    int64_t zero[MAXD] = {0, 0, 0};
    add_node(t, 0, zero);
    build_rec(t, 0, masks, mask_off);

    /* leaves in Peano order */
    int64_t nl = 0;
    for (int64_t i = 0; i < t->n_nodes; ++i) nl += t->nodes[i].child < 0;
    kv *lk = (kv *)malloc((size_t)nl * sizeof(kv));
    nl = 0;
    for (int64_t i = 0; i < t->n_nodes; ++i)
        if (t->nodes[i].child < 0) { lk[nl].key = leaf_key_of(t, &t->nodes[i]); lk[nl].idx = i; ++nl; }
    qsort(lk, (size_t)nl, sizeof(kv), cmp_kv);
    t->n_leaves = nl;
    t->leaf_node = (int32_t *)malloc((size_t)nl * sizeof(int32_t));
    t->leaf_key = (uint64_t *)malloc((size_t)nl * sizeof(uint64_t));
    for (int64_t r = 0; r < nl; ++r) {
        t->leaf_node[r] = (int32_t)lk[r].idx;
        t->leaf_key[r] = lk[r].key;
        t->nodes[lk[r].idx].leaf = (int32_t)r;
    }
    free(lk);

    /* vertices: distinct corner positions of leaves, lexicographic (axis 0 fastest) */
    int nc = 1 << dim;
    int64_t *lin = (int64_t *)malloc((size_t)(nl * nc) * sizeof(int64_t));
    for (int64_t r = 0; r < nl; ++r) {
        const onode *n = &t->nodes[t->leaf_node[r]];
        int64_t s = ipow3(L - n->level);
        for (int c = 0; c < nc; ++c) {
            int64_t p[MAXD] = {0, 0, 0};
            for (int k = 0; k < dim; ++k) p[k] = ((n->a[k] + ((c >> k) & 1)) * s) % t->S;
            lin[r * nc + c] = lex_index(dim, t->S, p);
        }
    }
    int64_t *srt = (int64_t *)malloc((size_t)(nl * nc) * sizeof(int64_t));
    memcpy(srt, lin, (size_t)(nl * nc) * sizeof(int64_t));
    qsort(srt, (size_t)(nl * nc), sizeof(int64_t), cmp_i64);
    int64_t nv = 0;
    for (int64_t i = 0; i < nl * nc; ++i)
        if (i == 0 || srt[i] != srt[i - 1]) srt[nv++] = srt[i];
    t->n_vtx = nv;
    t->vtx_lin = srt;
    t->leaf_vtx = (int32_t *)malloc((size_t)(nl * nc) * sizeof(int32_t));
    for (int64_t i = 0; i < nl * nc; ++i) t->leaf_vtx[i] = (int32_t)find_i64(srt, nv, lin[i]);
    free(lin);

    /* PIDT bins: (level, vertex of a leaf of that level), ordered by key */
    uint64_t *pk = (uint64_t *)malloc((size_t)(nl * nc) * sizeof(uint64_t));
    for (int64_t r = 0; r < nl; ++r) {
        const onode *n = &t->nodes[t->leaf_node[r]];
        int64_t nlv = ipow3(n->level);
        for (int c = 0; c < nc; ++c) {
            int64_t b[MAXD] = {0, 0, 0};
            for (int k = 0; k < dim; ++k) b[k] = (n->a[k] + ((c >> k) & 1)) % nlv;
            pk[r * nc + c] = pidt_key_of(t, n->level, b);
        }
    }
    uint64_t *ps = (uint64_t *)malloc((size_t)(nl * nc) * sizeof(uint64_t));
    memcpy(ps, pk, (size_t)(nl * nc) * sizeof(uint64_t));
    kv *tmp = (kv *)malloc((size_t)(nl * nc) * sizeof(kv));
    for (int64_t i = 0; i < nl * nc; ++i) { tmp[i].key = ps[i]; tmp[i].idx = 0; }
    qsort(tmp, (size_t)(nl * nc), sizeof(kv), cmp_kv);
    int64_t np = 0;
    for (int64_t i = 0; i < nl * nc; ++i)
        if (i == 0 || tmp[i].key != tmp[i - 1].key) ps[np++] = tmp[i].key;
    free(tmp);
    t->n_pidt = np;
    t->pidt_key = ps;
    t->leaf_pidt = (int32_t *)malloc((size_t)(nl * nc) * sizeof(int32_t));
    t->pidt_level = (int32_t *)malloc((size_t)np * sizeof(int32_t));
    t->pidt_b = (int64_t *)calloc((size_t)(np * dim), sizeof(int64_t));
    t->pidt_vtx = (int32_t *)malloc((size_t)np * sizeof(int32_t));
    for (int64_t r = 0; r < nl; ++r) {
        const onode *n = &t->nodes[t->leaf_node[r]];
        int64_t nlv = ipow3(n->level);
        for (int c = 0; c < nc; ++c) {
            int64_t bin = find_u64(ps, np, pk[r * nc + c]);
            t->leaf_pidt[r * nc + c] = (int32_t)bin;
            t->pidt_level[bin] = n->level;
            for (int k = 0; k < dim; ++k) t->pidt_b[bin * dim + k] = (n->a[k] + ((c >> k) & 1)) % nlv;
            t->pidt_vtx[bin] = t->leaf_vtx[r * nc + c];
        }
    }
    free(pk);
    return t;
}

void orc_tree_sizes(void *h, int64_t *out)
{
    otree *t = (otree *)h;
    out[0] = t->n_nodes;
    out[1] = t->n_leaves;
    out[2] = t->n_vtx;
    out[3] = t->n_pidt;
    out[4] = t->S;
}

void orc_tree_leaves(void *h, uint64_t *key, int32_t *level, int64_t *coord, int32_t *vtx, int32_t *pidt)
{
    otree *t = (otree *)h;
    int nc = 1 << t->dim;
    for (int64_t r = 0; r < t->n_leaves; ++r) {
        const onode *n = &t->nodes[t->leaf_node[r]];
        if (key) key[r] = t->leaf_key[r];
        if (level) level[r] = n->level;
        if (coord) for (int k = 0; k < t->dim; ++k) coord[r * t->dim + k] = n->a[k];
        for (int c = 0; c < nc; ++c) {
            if (vtx) vtx[r * nc + c] = t->leaf_vtx[r * nc + c];
            if (pidt) pidt[r * nc + c] = t->leaf_pidt[r * nc + c];
        }
    }
}

void orc_tree_vertices(void *h, int64_t *pos)
{
    otree *t = (otree *)h;
    for (int64_t v = 0; v < t->n_vtx; ++v) {
        int64_t r = t->vtx_lin[v];
        for (int k = 0; k < t->dim; ++k) { pos[v * t->dim + k] = r % t->S; r /= t->S; }
    }
}

void orc_tree_pidt(void *h, uint64_t *key, int32_t *level, int64_t *b, int32_t *vid)
{
    otree *t = (otree *)h;
    for (int64_t i = 0; i < t->n_pidt; ++i) {
        if (key) key[i] = t->pidt_key[i];
        if (level) level[i] = t->pidt_level[i];
        if (b) for (int k = 0; k < t->dim; ++k) b[i * t->dim + k] = t->pidt_b[i * t->dim + k];
        if (vid) vid[i] = t->pidt_vtx[i];
    }
}

/* ---------------------------------------------------------------- location */
/* Per-particle location data: the leaf covering y = fl(x*S) and the scaled
   position itself. Returns 0 on success, -1 if x lies outside [0,1). */
typedef struct {
    double y[MAXD];
    int64_t I[MAXD];
    int32_t leaf;         /* leaf rank */
    int level;
    int64_t s;            /* leaf width in finest cells */
    int64_t a[MAXD];      /* leaf coordinates at its level */
} oloc;

static int locate_one(const otree *t, const double *x, int64_t stride, int64_t p, oloc *o)
{
    double Sd = (double)t->S;
    for (int k = 0; k < t->dim; ++k) {
        double xk = x[k * stride + p];
        if (!(xk >= 0.0 && xk < 1.0)) return -1;
        o->y[k] = xk * Sd;
        int64_t I = (int64_t)floor(o->y[k]);
        if (I > t->S - 1) I = t->S - 1;   /* y == S: last cell (half-open reading) */
        o->I[k] = I;
    }
    /* root descent: the leaf that covers the cell I */
    int64_t id = 0;
    while (t->nodes[id].child >= 0) {
        int lev = t->nodes[id].level;
        int64_t p3 = ipow3(t->L - lev - 1);
        int64_t slot = 0, m = 1;
        for (int k = 0; k < t->dim; ++k) { slot += ((o->I[k] / p3) % 3) * m; m *= 3; }
        id = t->nodes[id].child + slot;
    }
    const onode *n = &t->nodes[id];
    o->leaf = n->leaf;
    o->level = n->level;
    o->s = ipow3(t->L - n->level);
    for (int k = 0; k < t->dim; ++k) o->a[k] = n->a[k];
    return 0;
}

/* Corner of the particle's leaf nearest to y (max norm, ties up): returns corner index. */
static int owner_corner(const otree *t, const oloc *o)
{
    int c = 0;
    for (int k = 0; k < t->dim; ++k) {
        double off = o->y[k] - (double)(o->a[k] * o->s);        /* exact */
        if (2.0 * off >= (double)o->s) c |= 1 << k;
    }
    return c;
}

/* d-linear weights of the 2^d corners (corner c = sum_k b_k 2^k). */
static void weights(const otree *t, const oloc *o, double *w)
{
    double f[MAXD], g[MAXD];
    double rinv = 1.0 / (double)o->s;
    for (int k = 0; k < t->dim; ++k) {
        f[k] = (o->y[k] - (double)(o->a[k] * o->s)) * rinv;
        g[k] = 1.0 - f[k];
    }
    int nc = 1 << t->dim;
    for (int c = 0; c < nc; ++c) {
        double wc = (c & 1) ? f[0] : g[0];
        for (int k = 1; k < t->dim; ++k) wc = wc * (((c >> k) & 1) ? f[k] : g[k]);
        w[c] = wc;
    }
}

/* x: dim*n SoA. leaf, pidt (nullable): bins; cell (nullable): n*dim finest cell I. */
int orc_locate(void *h, int64_t n, const double *x, int32_t *leaf, int32_t *pidt, int64_t *cell)
{
    otree *t = (otree *)h;
    int nc = 1 << t->dim;
    for (int64_t p = 0; p < n; ++p) {
        oloc o;
        if (locate_one(t, x, n, p, &o)) return -1;
        if (leaf) leaf[p] = o.leaf;
        if (pidt) pidt[p] = t->leaf_pidt[(int64_t)o.leaf * nc + owner_corner(t, &o)];
        if (cell) for (int k = 0; k < t->dim; ++k) cell[p * t->dim + k] = o.I[k];
    }
    return 0;
}

/* Corner weights per particle (n * 2^d) and corner vertex ids, for tests. */
int orc_weights(void *h, int64_t n, const double *x, double *w, int32_t *vtx)
{
    otree *t = (otree *)h;
    int nc = 1 << t->dim;
    for (int64_t p = 0; p < n; ++p) {
        oloc o;
        if (locate_one(t, x, n, p, &o)) return -1;
        weights(t, &o, w + p * nc);
        for (int c = 0; c < nc; ++c) vtx[p * nc + c] = t->leaf_vtx[(int64_t)o.leaf * nc + c];
    }
    return 0;
}

/* ---------------------------------------------------------------- gather + push */
/* One leapfrog step in place.  E: dim * n_vtx (component-major).
   Ep (nullable): gathered field, dim*n.  bin (nullable): new bin per particle
   for `scheme` (0 = PIT leaf, 1 = PIDT vertex). */
int orc_gather_push(void *h, int64_t n, double *x, double *v, const double *E,
                    double qmdt, double dt, double *Ep, int32_t *bin, int scheme)
{
    otree *t = (otree *)h;
    int nc = 1 << t->dim;
    double w[8];
    for (int64_t p = 0; p < n; ++p) {
        oloc o;
        if (locate_one(t, x, n, p, &o)) return -1;
        weights(t, &o, w);
        const int32_t *vt = t->leaf_vtx + (int64_t)o.leaf * nc;
        for (int j = 0; j < t->dim; ++j) {
            const double *Ej = E + (int64_t)j * t->n_vtx;
            double e = w[0] * Ej[vt[0]];
            for (int c = 1; c < nc; ++c) e = e + w[c] * Ej[vt[c]];
            if (Ep) Ep[j * n + p] = e;
            double vj = v[j * n + p] + qmdt * e;
            double xj = x[j * n + p] + vj * dt;
            xj = xj - floor(xj);
            if (xj == 1.0) xj = 0.0;
            v[j * n + p] = vj;
            x[j * n + p] = xj;
        }
        if (bin) {
            oloc q;
            if (locate_one(t, x, n, p, &q)) return -1;
            bin[p] = scheme == 0 ? q.leaf : t->leaf_pidt[(int64_t)q.leaf * nc + owner_corner(t, &q)];
        }
    }
    return 0;
}

/* ---------------------------------------------------------------- free streaming */
/* The particle-handling benchmark of the paper's results section (Sec. 6,
   setup): no field and no particle-grid interplay; every particle moves
   x <- x + v dt per axis, then
     boundary 0 (periodic):   x <- x - floor(x), 1.0 -> 0.0 (as in the push);
     boundary 1 (reflecting): below 0 the position is mirrored at 0 (x -> -x),
       at or above 1 at 1 (x -> 2 - x), and that velocity component changes
       sign; a particle mirrored exactly onto 1 is put at the largest double
       below 1.
   A move that a single reflection cannot bring back (|v dt| >= 1 towards a
   wall) is an error (-1).  `flops` artificial floating-point operations per
   particle move (the paper's 0 to 4096) are carried out and discarded.
   bin (nullable): new bin per particle for `scheme`. */
static volatile double orc_flop_sink;

int orc_free_stream(void *h, int64_t n, double *x, double *v, double dt, int boundary, int flops,
                    int32_t *bin, int scheme)
{
    otree *t = (otree *)h;
    int nc = 1 << t->dim;
    double sink = 0.0;
    for (int64_t p = 0; p < n; ++p) {
        for (int j = 0; j < t->dim; ++j) {
            double vj = v[j * n + p];
            double xj = x[j * n + p] + vj * dt;
            if (boundary == 0) {
                xj = xj - floor(xj);
                if (xj == 1.0) xj = 0.0;
            } else if (xj < 0.0) {
                xj = -xj;
                vj = -vj;
                if (!(xj < 1.0)) return -1;
            } else if (xj >= 1.0) {
                xj = 2.0 - xj;
                vj = -vj;
                if (xj < 0.0) return -1;
                if (xj == 1.0) xj = nextafter(1.0, 0.0);
            }
            if (!(xj >= 0.0 && xj < 1.0)) return -1;
            v[j * n + p] = vj;
            x[j * n + p] = xj;
        }
        double a = x[p];
        for (int f = 0; f < flops / 2; ++f) a = a * 0.5 + 0.25;
        sink += a;
        if (bin) {
            oloc q;
            if (locate_one(t, x, n, p, &q)) return -1;
            bin[p] = scheme == 0 ? q.leaf : t->leaf_pidt[(int64_t)q.leaf * nc + owner_corner(t, &q)];
        }
    }
    orc_flop_sink = sink;
    return 0;
}

/* ---------------------------------------------------------------- re-bin */
/* Stable re-bin.  new_bin: n bins in [0,n_bins).  old_start: n_bins+1 segment
   offsets of the input order, or NULL when the input is unsorted (then every
   particle counts as arriving).  Output: perm (out[j] = in[perm[j]]) and
   new_start (n_bins+1).  Within a bin: stayers in old order, then arrivals
   in old order. */
int orc_rebin(int64_t n, int64_t n_bins, const int32_t *new_bin, const int64_t *old_start,
              int64_t *perm, int64_t *new_start)
{
    int64_t *cnt_stay = (int64_t *)calloc((size_t)n_bins, sizeof(int64_t));
    int64_t *cnt_move = (int64_t *)calloc((size_t)n_bins, sizeof(int64_t));
    int32_t *old_bin = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    for (int64_t p = 0; p < n; ++p) old_bin[p] = -1;
    if (old_start) {
        if (old_start[0] != 0 || old_start[n_bins] != n) { free(cnt_stay); free(cnt_move); free(old_bin); return -1; }
        for (int64_t b = 0; b < n_bins; ++b)
            for (int64_t p = old_start[b]; p < old_start[b + 1]; ++p) old_bin[p] = (int32_t)b;
    }
    for (int64_t p = 0; p < n; ++p) {
        if (new_bin[p] < 0 || new_bin[p] >= n_bins) { free(cnt_stay); free(cnt_move); free(old_bin); return -1; }
        if (new_bin[p] == old_bin[p]) cnt_stay[new_bin[p]]++; else cnt_move[new_bin[p]]++;
    }
    int64_t *fill_stay = (int64_t *)malloc((size_t)n_bins * sizeof(int64_t));
    int64_t *fill_move = (int64_t *)malloc((size_t)n_bins * sizeof(int64_t));
    int64_t acc = 0;
    for (int64_t b = 0; b < n_bins; ++b) {
        new_start[b] = acc;
        fill_stay[b] = acc;
        fill_move[b] = acc + cnt_stay[b];
        acc += cnt_stay[b] + cnt_move[b];
    }
    new_start[n_bins] = acc;
    for (int64_t p = 0; p < n; ++p) {
        int32_t b = new_bin[p];
        if (b == old_bin[p]) perm[fill_stay[b]++] = p; else perm[fill_move[b]++] = p;
    }
    free(cnt_stay); free(cnt_move); free(old_bin); free(fill_stay); free(fill_move);
    return 0;
}

/* ---------------------------------------------------------------- deposit */
/* rho_v = sum_p q_p w_v(x_p) with Neumaier compensated summation in particle
   order.  q: per-particle charge or NULL (then q_uniform). */
int orc_deposit(void *h, int64_t n, const double *x, const double *q, double q_uniform, double *rho)
{
    otree *t = (otree *)h;
    int nc = 1 << t->dim;
    double *comp = (double *)calloc((size_t)t->n_vtx, sizeof(double));
    for (int64_t i = 0; i < t->n_vtx; ++i) rho[i] = 0.0;
    double w[8];
    for (int64_t p = 0; p < n; ++p) {
        oloc o;
        if (locate_one(t, x, n, p, &o)) { free(comp); return -1; }
        weights(t, &o, w);
        double qp = q ? q[p] : q_uniform;
        const int32_t *vt = t->leaf_vtx + (int64_t)o.leaf * nc;
        for (int c = 0; c < nc; ++c) {
            double term = qp * w[c];
            double s = rho[vt[c]];
            double tsum = s + term;
            if (fabs(s) >= fabs(term)) comp[vt[c]] += (s - tsum) + term;
            else comp[vt[c]] += (term - tsum) + s;
            rho[vt[c]] = tsum;
        }
    }
    for (int64_t i = 0; i < t->n_vtx; ++i) rho[i] += comp[i];
    free(comp);
    return 0;
}

/* ---------------------------------------------------------------- re-bin statistics */
/* Lifts per particle (paper Sec. 6.1; PIT, Sec. 5.1): a particle that leaves
   its leaf a is lifted to the parent cell until a cell covers it, then
   dropped into its new leaf b, so it is lifted level(a) - level(c) times, c
   the coarsest common ancestor of a and b.  The ancestor of a level-l cell
   with coordinates a at level m <= l has coordinates a / 3^(l-m); c is the
   finest level m <= min(level(a), level(b)) at which the two ancestors
   agree.  PIDT: the same in the dual tree.  Dual cells of a k = 3 tree nest
   (Sec. 4.1): the dual cell of the level-l vertex b covers, per axis, the
   finest vertices within (3^(L-l) - 1)/2 of b 3^(L-l), which on the lattice
   shifted by (3^L - 1)/2 is the aligned level-l block number
   (b + (3^l - 1)/2) mod 3^l; its ancestors are taken on those numbers.
   Tunnel distance: the periodic max-norm distance between the old and new
   bin's anchor (leaf lower corner, or vertex position) in finest units.
   out: particles, movers, lifts, max_tunnel, hist[n_hist] (particles by lift
   count, the last entry also counting larger ones); added to. */
static void bin_cell(const otree *t, int scheme, int64_t b, int *level, int64_t *a, int64_t *anchor)
{
    if (scheme == 0) {
        const onode *nd = &t->nodes[t->leaf_node[b]];
        *level = nd->level;
        for (int k = 0; k < t->dim; ++k) {
            a[k] = nd->a[k];
            anchor[k] = nd->a[k] * ipow3(t->L - nd->level);
        }
    } else {
        const int l = t->pidt_level[b];
        const int64_t nl = ipow3(l);
        *level = l;
        for (int k = 0; k < t->dim; ++k) {
            const int64_t bk = t->pidt_b[b * t->dim + k];
            a[k] = (bk + (nl - 1) / 2) % nl;
            anchor[k] = bk * ipow3(t->L - l);
        }
    }
}

int orc_rebin_stats(void *h, int scheme, int64_t n, const int64_t *old_start, const int32_t *new_bin,
                    int n_hist, int64_t *out)
{
    otree *t = (otree *)h;
    const int64_t n_bins = scheme == 0 ? t->n_leaves : t->n_pidt;
    if (old_start[0] != 0 || old_start[n_bins] != n) return -1;
    out[0] += n;
    for (int64_t b0 = 0; b0 < n_bins; ++b0) {
        for (int64_t p = old_start[b0]; p < old_start[b0 + 1]; ++p) {
            const int64_t b1 = new_bin[p];
            if (b1 < 0 || b1 >= n_bins) return -1;
            if (b1 == b0) { out[4] += 1; continue; }
            int l0, l1;
            int64_t a0[MAXD], a1[MAXD], A0[MAXD], A1[MAXD];
            bin_cell(t, scheme, b0, &l0, a0, A0);
            bin_cell(t, scheme, b1, &l1, a1, A1);
            int m = l0 < l1 ? l0 : l1;
            for (; m > 0; --m) {
                int same = 1;
                for (int k = 0; k < t->dim; ++k)
                    if (a0[k] / ipow3(l0 - m) != a1[k] / ipow3(l1 - m)) same = 0;
                if (same) break;
            }
            int64_t dist = 0;
            for (int k = 0; k < t->dim; ++k) {
                int64_t d = A0[k] > A1[k] ? A0[k] - A1[k] : A1[k] - A0[k];
                if (t->S - d < d) d = t->S - d;
                if (d > dist) dist = d;
            }
            const int lifts = l0 - m;
            out[1] += 1;
            out[2] += lifts;
            if (dist > out[3]) out[3] = dist;
            out[4 + (lifts < n_hist ? lifts : n_hist - 1)] += 1;
        }
    }
    return 0;
}
