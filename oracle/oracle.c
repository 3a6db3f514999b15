/*
 * oracle.c -- plain, slow FP64 CPU oracle for the Barnes-Hut gravity hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load this file's library.  It shares no code, header, table or
 * helper with the GPU library and must never be used as a fallback for it.
 *
 * What it computes (Iwasawa et al., "Implementation and Performance of FDPS"):
 *   - O-D: the exact quantity the tree approximates, softened FP64 direct summation with
 *     G = 1, equations (ParticleParticleNbody) and (ConversionNbody) of section
 *     "An example -- gravitational N-body problem".
 *   - O-T: a serial Barnes-Hut tree taken step by step: keys, sort, octree, multipole
 *     moments up to the quadrupole (section "Design concept of FDPS"), i-particle groups
 *     of the modified tree algorithm (section "Tree traverse and interaction
 *     calculation"), one shared interaction list per group built with a fixed opening
 *     angle (section "Exchange of particles and superparticles"), and the particle /
 *     superparticle force of equations (ParticleParticleNbody) and
 *     (ParticleSuperparticleNbody).
 *   - the exchange lists between domains, the short-range neighbour walk with the SPH
 *     density, the cutoff tree of TreePM, and the multisection domain decomposition with
 *     cost-weighted sampling (section "Domain decomposition"), each at its own section below.
 * Where the paper is silent (how keys and cells are formed, the opening test, group shape,
 * quadrupole formula) the oracle implements one fixed reading; each is stated at the
 * function that implements it.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no FMA contraction, so every
 * product and sum below is rounded exactly as written).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Threads of the OpenMP loops (for timing the oracle single-threaded); returns the previous
 * maximum. */
int or_set_threads(int n) {
    const int prev = omp_get_max_threads();
    if (n > 0) omp_set_num_threads(n);
    return prev;
}

#define OR_LEVELS 21            /* bits per axis of a key; deepest cell level */
#define OR_NONE 0xFFFFFFFFu

/* ------------------------------------------------------------------------------------ */
/* Neumaier-compensated summation (an exact-as-possible FP64 accumulator).               */
typedef struct { double s, c; } nsum;
static inline void nadd(nsum *a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}
static inline double nval(const nsum *a) { return a->s + a->c; }

/* ------------------------------------------------------------------------------------ */
/* O-D: direct summation.  For target i and every source j != i of the range [jb, je):
 *   a_i   += m_j (r_j - r_i) / (|r_j - r_i|^2 + eps_i^2)^{3/2}
 *   phi_i += -m_j / (|r_j - r_i|^2 + eps_i^2)^{1/2}
 * (equation ParticleParticleNbody with G = 1; the potential is the matching 1/r sum, the
 * self term excluded). */
void or_direct(int64_t jb, int64_t je, const double *x, const double *y, const double *z,
               const double *m, const double *eps, int64_t nt, const int64_t *tgt,
               double *ax, double *ay, double *az, double *pot) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nt; t++) {
        int64_t i = tgt[t];
        double e2 = eps[i] * eps[i];
        nsum sx = {0, 0}, sy = {0, 0}, sz = {0, 0}, sp = {0, 0};
        for (int64_t j = jb; j < je; j++) {
            if (j == i) continue;
            double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
            double r2 = dx * dx + dy * dy + dz * dz + e2;
            double rinv = 1.0 / sqrt(r2);
            double mr3 = m[j] * rinv * rinv * rinv;
            nadd(&sx, mr3 * dx);
            nadd(&sy, mr3 * dy);
            nadd(&sz, mr3 * dz);
            nadd(&sp, -m[j] * rinv);
        }
        ax[t] = nval(&sx); ay[t] = nval(&sy); az[t] = nval(&sz); pot[t] = nval(&sp);
    }
}

/* ------------------------------------------------------------------------------------ */
/* Root cube of one system.  Reading (the paper only says a tree is constructed): exact
 * per-axis minimum and maximum; L = largest extent; Lr = smallest power of two >= L
 * (Lr = 1 when L = 0); origin = the minimum corner.  out = {ox, oy, oz, Lr}. */
void or_root_cube(int64_t n, const double *x, const double *y, const double *z, double *out) {
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    const double *p[3] = {x, y, z};
    for (int a = 0; a < 3; a++) {
        if (n > 0) { lo[a] = p[a][0]; hi[a] = p[a][0]; }
        for (int64_t i = 1; i < n; i++) {
            if (p[a][i] < lo[a]) lo[a] = p[a][i];
            if (p[a][i] > hi[a]) hi[a] = p[a][i];
        }
    }
    double L = 0.0;
    for (int a = 0; a < 3; a++) if (hi[a] - lo[a] > L) L = hi[a] - lo[a];
    double Lr = 1.0;
    if (L > 0.0) {
        while (Lr < L) Lr *= 2.0;           /* exact: powers of two */
        while (Lr * 0.5 >= L) Lr *= 0.5;
    }
    out[0] = lo[0]; out[1] = lo[1]; out[2] = lo[2]; out[3] = Lr;
}

/* Integer grid coordinate on one axis: q = min(2^21 - 1, floor((x - o) * 2^21 / Lr)). */
static uint32_t grid_coord(double xv, double o, double Lr) {
    double s = 2097152.0 / Lr;              /* 2^21 / Lr: a power of two, exact */
    double t = (xv - o) * s;
    double f = floor(t);
    if (f < 0.0) f = 0.0;
    if (f > 2097151.0) f = 2097151.0;
    return (uint32_t)f;
}

/* Morton key: bit b of qx goes to key bit 3b+2, of qy to 3b+1, of qz to 3b (one bit at a
 * time, the plain definition of the interleave). */
uint64_t or_interleave(uint32_t qx, uint32_t qy, uint32_t qz) {
    uint64_t k = 0;
    for (int b = 0; b < OR_LEVELS; b++) {
        k |= (uint64_t)((qx >> b) & 1u) << (3 * b + 2);
        k |= (uint64_t)((qy >> b) & 1u) << (3 * b + 1);
        k |= (uint64_t)((qz >> b) & 1u) << (3 * b);
    }
    return k;
}

static void deinterleave(uint64_t k, uint32_t *qx, uint32_t *qy, uint32_t *qz) {
    uint32_t a = 0, b = 0, c = 0;
    for (int i = 0; i < OR_LEVELS; i++) {
        a |= (uint32_t)((k >> (3 * i + 2)) & 1u) << i;
        b |= (uint32_t)((k >> (3 * i + 1)) & 1u) << i;
        c |= (uint32_t)((k >> (3 * i)) & 1u) << i;
    }
    *qx = a; *qy = b; *qz = c;
}

void or_deinterleave(int64_t n, const uint64_t *k, uint32_t *q) {
    for (int64_t i = 0; i < n; i++) deinterleave(k[i], &q[3 * i], &q[3 * i + 1], &q[3 * i + 2]);
}

/* Keys of all particles of all systems (system s owns [off[s], off[s+1])).
 * cube receives {ox, oy, oz, Lr} per system. */
void or_keys(int64_t nsys, const int64_t *off, const double *x, const double *y,
             const double *z, double *cube, uint64_t *key) {
    for (int64_t s = 0; s < nsys; s++) {
        int64_t b = off[s], e = off[s + 1];
        double *c = cube + 4 * s;
        or_root_cube(e - b, x + b, y + b, z + b, c);
        for (int64_t i = b; i < e; i++)
            key[i] = or_interleave(grid_coord(x[i], c[0], c[3]), grid_coord(y[i], c[1], c[3]),
                                   grid_coord(z[i], c[2], c[3]));
    }
}

/* ------------------------------------------------------------------------------------ */
/* Sort by (system, key), ties by original index (a stable sort).  perm[r] = original index
 * of the particle at sorted rank r. */
typedef struct { int64_t sys; uint64_t key; int64_t idx; } sort_item;
static int cmp_item(const void *pa, const void *pb) {
    const sort_item *a = (const sort_item *)pa, *b = (const sort_item *)pb;
    if (a->sys != b->sys) return a->sys < b->sys ? -1 : 1;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
    return 0;
}

void or_sort(int64_t nsys, const int64_t *off, const uint64_t *key, uint32_t *perm) {
    int64_t n = off[nsys];
    sort_item *it = (sort_item *)malloc(sizeof(sort_item) * (size_t)(n > 0 ? n : 1));
    for (int64_t s = 0; s < nsys; s++)
        for (int64_t i = off[s]; i < off[s + 1]; i++) {
            it[i].sys = s; it[i].key = key[i]; it[i].idx = i;
        }
    qsort(it, (size_t)n, sizeof(sort_item), cmp_item);
    for (int64_t r = 0; r < n; r++) perm[r] = (uint32_t)it[r].idx;
    free(it);
}

/* ------------------------------------------------------------------------------------ */
/* Octree.  A cell is a run of sorted particles sharing the top 3*level key bits.  Reading:
 * the roots (one per system) are cells of level 0; a cell is split when it holds more than
 * n_leaf particles and its level is below 21; its non-empty octants become its children,
 * kept in ascending octant order; single-child cells are kept.  Cells are numbered in
 * breadth-first (level) order, which a FIFO queue over the roots produces directly. */
typedef struct {
    int64_t ncell, cap;
    int32_t *level;
    uint64_t *prefix;
    uint32_t *begin, *count, *first_child, *nchild, *parent;
} or_cells;

static void cells_push(or_cells *t, int32_t lv, uint64_t pre, uint32_t b, uint32_t c,
                       uint32_t par) {
    if (t->ncell == t->cap) {
        t->cap = t->cap ? 2 * t->cap : 64;
        t->level = realloc(t->level, sizeof(int32_t) * t->cap);
        t->prefix = realloc(t->prefix, sizeof(uint64_t) * t->cap);
        t->begin = realloc(t->begin, sizeof(uint32_t) * t->cap);
        t->count = realloc(t->count, sizeof(uint32_t) * t->cap);
        t->first_child = realloc(t->first_child, sizeof(uint32_t) * t->cap);
        t->nchild = realloc(t->nchild, sizeof(uint32_t) * t->cap);
        t->parent = realloc(t->parent, sizeof(uint32_t) * t->cap);
    }
    int64_t k = t->ncell++;
    t->level[k] = lv; t->prefix[k] = pre; t->begin[k] = b; t->count[k] = c;
    t->first_child[k] = OR_NONE; t->nchild[k] = 0; t->parent[k] = par;
}

/* skey: keys in sorted order.  Returns an opaque cell table. */
void *or_build_cells(int64_t nsys, const int64_t *off, const uint64_t *skey, int32_t n_leaf) {
    or_cells *t = (or_cells *)calloc(1, sizeof(or_cells));
    for (int64_t s = 0; s < nsys; s++)
        cells_push(t, 0, 0, (uint32_t)off[s], (uint32_t)(off[s + 1] - off[s]), OR_NONE);
    for (int64_t c = 0; c < t->ncell; c++) {     /* FIFO: t->ncell grows while we scan */
        int32_t lv = t->level[c];
        if (!((int64_t)t->count[c] > n_leaf && lv < OR_LEVELS)) continue;
        int sh = 3 * (OR_LEVELS - 1 - lv);      /* octant digit of a level lv+1 child */
        uint32_t b = t->begin[c], e = t->begin[c] + t->count[c];
        uint32_t first = (uint32_t)t->ncell, nch = 0;
        for (uint32_t oct = 0; oct < 8; oct++) {
            uint32_t cb = OR_NONE, cn = 0;
            for (uint32_t i = b; i < e; i++)
                if (((skey[i] >> sh) & 7u) == oct) { if (cb == OR_NONE) cb = i; cn++; }
            if (cn) { cells_push(t, lv + 1, (t->prefix[c] << 3) | oct, cb, cn, (uint32_t)c); nch++; }
        }
        t->first_child[c] = first;
        t->nchild[c] = nch;
    }
    return t;
}

int64_t or_cells_count(void *h) { return ((or_cells *)h)->ncell; }

/* System of every cell: roots are the first nsys cells and every parent precedes its
 * children in breadth-first order. */
void or_cells_system(void *h, int64_t nsys, uint32_t *csys) {
    or_cells *t = (or_cells *)h;
    for (int64_t c = 0; c < t->ncell; c++)
        csys[c] = c < nsys ? (uint32_t)c : csys[t->parent[c]];
}

void or_cells_export(void *h, int32_t *level, uint64_t *prefix, uint32_t *begin,
                     uint32_t *count, uint32_t *first_child, uint32_t *nchild, uint32_t *parent) {
    or_cells *t = (or_cells *)h;
    size_t n = (size_t)t->ncell;
    memcpy(level, t->level, n * sizeof(int32_t));
    memcpy(prefix, t->prefix, n * sizeof(uint64_t));
    memcpy(begin, t->begin, n * sizeof(uint32_t));
    memcpy(count, t->count, n * sizeof(uint32_t));
    memcpy(first_child, t->first_child, n * sizeof(uint32_t));
    memcpy(nchild, t->nchild, n * sizeof(uint32_t));
    memcpy(parent, t->parent, n * sizeof(uint32_t));
}

void or_cells_free(void *h) {
    or_cells *t = (or_cells *)h;
    if (!t) return;
    free(t->level); free(t->prefix); free(t->begin); free(t->count);
    free(t->first_child); free(t->nchild); free(t->parent); free(t);
}

/* ------------------------------------------------------------------------------------ */
/* Multipole moments of every cell, straight from its particle range (the definition):
 *   M = sum m,  X = sum m x / M,  Q_ab = sum m (3 d_a d_b - |d|^2 delta_ab),  d = x - X.
 * (The paper provides superparticles up to the quadrupole moment for 1/r; the traceless
 * form about the centre of mass is the reading used here, so the dipole vanishes.)
 * sx..sm are particle arrays in sorted order.  mom[10*c] = {M, X, Y, Z, Qxx, Qyy, Qzz,
 * Qxy, Qxz, Qyz}. */
void or_moments(int64_t ncell, const uint32_t *begin, const uint32_t *count,
                const double *sx, const double *sy, const double *sz, const double *sm,
                double *mom) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < ncell; c++) {
        uint32_t b = begin[c], e = begin[c] + count[c];
        nsum M = {0, 0}, MX = {0, 0}, MY = {0, 0}, MZ = {0, 0};
        for (uint32_t i = b; i < e; i++) {
            nadd(&M, sm[i]); nadd(&MX, sm[i] * sx[i]); nadd(&MY, sm[i] * sy[i]);
            nadd(&MZ, sm[i] * sz[i]);
        }
        double m = nval(&M);
        double X = 0, Y = 0, Z = 0;
        if (m > 0) { X = nval(&MX) / m; Y = nval(&MY) / m; Z = nval(&MZ) / m; }
        nsum q[6] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}};
        for (uint32_t i = b; i < e; i++) {
            double dx = sx[i] - X, dy = sy[i] - Y, dz = sz[i] - Z;
            double d2 = dx * dx + dy * dy + dz * dz;
            nadd(&q[0], sm[i] * (3.0 * dx * dx - d2));
            nadd(&q[1], sm[i] * (3.0 * dy * dy - d2));
            nadd(&q[2], sm[i] * (3.0 * dz * dz - d2));
            nadd(&q[3], sm[i] * (3.0 * dx * dy));
            nadd(&q[4], sm[i] * (3.0 * dx * dz));
            nadd(&q[5], sm[i] * (3.0 * dy * dz));
        }
        double *o = mom + 10 * c;
        o[0] = m; o[1] = X; o[2] = Y; o[3] = Z;
        for (int k = 0; k < 6; k++) o[4 + k] = nval(&q[k]);
    }
}

/* ------------------------------------------------------------------------------------ */
/* i-particle groups of the modified tree algorithm (Barnes 1990).  Reading of n_grp: the
 * largest number of particles that share one interaction list.  A group is a maximal cell
 * holding at most n_group particles; a leaf with more (possible only at level 21 or when
 * n_group < n_leaf) is cut into consecutive runs of n_group.  Depth-first order over
 * children in octant order lists the groups by ascending first particle.
 * Output per group: cell, begin, count.  Returns the number of groups. */
typedef struct { uint32_t *cell, *begin, *count; int64_t n, cap; } grp_buf;
static void grp_push(grp_buf *g, uint32_t c, uint32_t b, uint32_t n) {
    if (g->n == g->cap) {
        g->cap = g->cap ? 2 * g->cap : 64;
        g->cell = realloc(g->cell, sizeof(uint32_t) * g->cap);
        g->begin = realloc(g->begin, sizeof(uint32_t) * g->cap);
        g->count = realloc(g->count, sizeof(uint32_t) * g->cap);
    }
    g->cell[g->n] = c; g->begin[g->n] = b; g->count[g->n] = n; g->n++;
}
static void grp_visit(const or_cells *t, uint32_t c, int32_t ng, grp_buf *g) {
    uint32_t cnt = t->count[c];
    if (cnt == 0) return;
    if ((int64_t)cnt <= ng) { grp_push(g, c, t->begin[c], cnt); return; }
    if (t->nchild[c] == 0) {
        for (uint32_t b = 0; b < cnt; b += (uint32_t)ng)
            grp_push(g, c, t->begin[c] + b, (cnt - b) < (uint32_t)ng ? cnt - b : (uint32_t)ng);
        return;
    }
    for (uint32_t k = 0; k < t->nchild[c]; k++) grp_visit(t, t->first_child[c] + k, ng, g);
}

void *or_groups(void *h, int64_t nsys, int32_t n_group) {
    const or_cells *t = (const or_cells *)h;
    grp_buf *g = (grp_buf *)calloc(1, sizeof(grp_buf));
    for (int64_t s = 0; s < nsys; s++) grp_visit(t, (uint32_t)s, n_group, g);
    return g;
}
int64_t or_groups_count(void *gh) { return ((grp_buf *)gh)->n; }
void or_groups_export(void *gh, uint32_t *cell, uint32_t *begin, uint32_t *count) {
    grp_buf *g = (grp_buf *)gh;
    memcpy(cell, g->cell, sizeof(uint32_t) * g->n);
    memcpy(begin, g->begin, sizeof(uint32_t) * g->n);
    memcpy(count, g->count, sizeof(uint32_t) * g->n);
}
void or_groups_free(void *gh) {
    grp_buf *g = (grp_buf *)gh;
    if (!g) return;
    free(g->cell); free(g->begin); free(g->count); free(g);
}

/* Integer bounding box of each group's members in grid units (from their keys) and the
 * geometric centre of the group's cell: centre = o + (2*corner + 2^(21-l)) * Lr / 2^22,
 * with corner the cell's integer corner (one rounding, in the addition). */
void or_group_geometry(int64_t ng, const uint32_t *gcell, const uint32_t *gbegin,
                       const uint32_t *gcount, const int32_t *level, const uint64_t *prefix,
                       const uint64_t *skey, const uint32_t *csys, const double *cube,
                       uint32_t *qmin, uint32_t *qmax, double *centre) {
    for (int64_t g = 0; g < ng; g++) {
        uint32_t lo[3] = {OR_NONE, OR_NONE, OR_NONE}, hi[3] = {0, 0, 0};
        for (uint32_t i = gbegin[g]; i < gbegin[g] + gcount[g]; i++) {
            uint32_t q[3];
            deinterleave(skey[i], &q[0], &q[1], &q[2]);
            for (int a = 0; a < 3; a++) {
                if (q[a] < lo[a]) lo[a] = q[a];
                if (q[a] > hi[a]) hi[a] = q[a];
            }
        }
        uint32_t c = gcell[g];
        int32_t l = level[c];
        uint32_t cq[3];
        deinterleave(prefix[c] << (3 * (OR_LEVELS - l)), &cq[0], &cq[1], &cq[2]);
        const double *cb = cube + 4 * csys[c];
        for (int a = 0; a < 3; a++) {
            qmin[3 * g + a] = lo[a];
            qmax[3 * g + a] = hi[a];
            double half_grid = 2.0 * (double)cq[a] + (double)(1u << (OR_LEVELS - l));
            centre[3 * g + a] = cb[a] + half_grid * (cb[3] / 4194304.0);
        }
    }
}

/* ------------------------------------------------------------------------------------ */
/* Opening test (reading of "a fixed opening angle theta"): a cell of side S whose centre
 * lies at distance D from the group's box is used as a superparticle iff S^2 < theta^2 D^2;
 * otherwise it is opened (equality opens).  Everything is measured in half-grid units so
 * that S, D^2 and the box are exact integers:
 *   S = 2^(22-l),  centre C = 2*corner + 2^(21-l),  box [2 qmin, 2 qmax + 2],
 *   D^2 = sum_a max(0, Bmin_a - C_a, C_a - Bmax_a)^2,  theta^2 = theta * theta.
 * The box bounds every member, so the test is conservative for each i of the group, as
 * one shared list requires. */
static int accept_cell(int32_t l, uint64_t prefix, const int64_t *bq_lo, const int64_t *bq_hi,
                       double th2) {
    uint32_t cq[3];
    deinterleave(prefix << (3 * (OR_LEVELS - l)), &cq[0], &cq[1], &cq[2]);
    double D2 = 0.0;
    for (int a = 0; a < 3; a++) {
        int64_t C = 2 * (int64_t)cq[a] + ((int64_t)1 << (OR_LEVELS - l));
        int64_t bmin = 2 * bq_lo[a], bmax = 2 * bq_hi[a] + 2;
        int64_t d = 0;
        if (bmin - C > d) d = bmin - C;
        if (C - bmax > d) d = C - bmax;
        D2 += (double)(d * d);
    }
    double S = ldexp(1.0, 22 - l);
    return S * S < th2 * D2;
}

/* Group walk: depth first from the system's root, children in octant order.  An accepted
 * cell joins the superparticle (SPJ) list; an opened leaf contributes all its particles to
 * the particle (EPJ) list (section "Exchange of particles and superparticles";
 * equation geqL splits the sum this way). */
typedef struct { uint32_t *v; int64_t n, cap; } u32vec;
static void vpush(u32vec *a, uint32_t x) {
    if (a->n == a->cap) { a->cap = a->cap ? 2 * a->cap : 256; a->v = realloc(a->v, 4 * a->cap); }
    a->v[a->n++] = x;
}
static void walk_visit(const or_cells *t, uint32_t c, const int64_t *lo, const int64_t *hi,
                       double th2, u32vec *epj, u32vec *spj) {
    if (t->count[c] == 0) return;
    if (accept_cell(t->level[c], t->prefix[c], lo, hi, th2)) { vpush(spj, c); return; }
    if (t->nchild[c] == 0) {
        for (uint32_t i = t->begin[c]; i < t->begin[c] + t->count[c]; i++) vpush(epj, i);
        return;
    }
    for (uint32_t k = 0; k < t->nchild[c]; k++)
        walk_visit(t, t->first_child[c] + k, lo, hi, th2, epj, spj);
}

/* Walk the listed groups (gsel[k] for k < nsel) and return CSR lists:
 * counts[2k] = |EPJ|, counts[2k+1] = |SPJ|; the caller then asks for the flat arrays. */
typedef struct { int64_t nsel; u32vec *epj, *spj; } walk_res;

void *or_walk(void *h, int64_t nsel, const int64_t *gsel, const uint32_t *groot,
              const uint32_t *qmin, const uint32_t *qmax, double theta, int64_t *counts) {
    const or_cells *t = (const or_cells *)h;
    walk_res *w = (walk_res *)calloc(1, sizeof(walk_res));
    w->nsel = nsel;
    w->epj = (u32vec *)calloc((size_t)(nsel > 0 ? nsel : 1), sizeof(u32vec));
    w->spj = (u32vec *)calloc((size_t)(nsel > 0 ? nsel : 1), sizeof(u32vec));
    double th2 = theta * theta;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nsel; k++) {
        int64_t g = gsel[k];
        int64_t lo[3], hi[3];
        for (int a = 0; a < 3; a++) { lo[a] = qmin[3 * g + a]; hi[a] = qmax[3 * g + a]; }
        walk_visit(t, groot[g], lo, hi, th2, &w->epj[k], &w->spj[k]);
        counts[2 * k] = w->epj[k].n;
        counts[2 * k + 1] = w->spj[k].n;
    }
    return w;
}
/* Exchange lists (section "Exchange of particles and superparticles", long-range mode):
 * every domain -- one system of the set, with its own local tree -- sends every other
 * domain the particles and superparticles it needs, found by the usual traversal of the
 * sender's tree with the fixed opening angle theta.  Reading: the receiving domain is
 * represented by the exact bounding box of its particles (blo, bhi: 3 per system), mapped
 * into the sender's integer grid as q = floor((x - o) * 2^21 / Lr) per axis for the lower and
 * the upper corner (cube: o_x, o_y, o_z, Lr per system), clamped to [-2^24, 2^24] so that
 * half-grid distances stay exact in FP64 (the clamp only moves a distant box closer, which
 * opens more cells: the list stays sufficient).  The traversal is the group walk with that
 * box: accepted cells are superparticles, opened leaves give their particles.  Pairs are
 * ordered by sender, then receiver (receiver != sender); counts[2k] = |EPJ|,
 * counts[2k+1] = |SPJ| of pair k. */
static int64_t grid_signed(double xv, double o, double Lr) {
    double s = 2097152.0 / Lr;
    double f = floor((xv - o) * s);
    if (f < -16777216.0) f = -16777216.0;
    if (f > 16777216.0) f = 16777216.0;
    return (int64_t)f;
}

void *or_exchange(void *h, int64_t nsys, const double *cube, const double *blo,
                  const double *bhi, double theta, int64_t *counts) {
    const or_cells *t = (const or_cells *)h;
    const int64_t np = nsys * (nsys - 1);
    walk_res *w = (walk_res *)calloc(1, sizeof(walk_res));
    w->nsel = np;
    w->epj = (u32vec *)calloc((size_t)(np > 0 ? np : 1), sizeof(u32vec));
    w->spj = (u32vec *)calloc((size_t)(np > 0 ? np : 1), sizeof(u32vec));
    double th2 = theta * theta;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < np; k++) {
        const int64_t s = k / (nsys - 1), j = k % (nsys - 1), r = j < s ? j : j + 1;
        int64_t lo[3], hi[3];
        for (int a = 0; a < 3; a++) {
            lo[a] = grid_signed(blo[3 * r + a], cube[4 * s + a], cube[4 * s + 3]);
            hi[a] = grid_signed(bhi[3 * r + a], cube[4 * s + a], cube[4 * s + 3]);
        }
        walk_visit(t, (uint32_t)s, lo, hi, th2, &w->epj[k], &w->spj[k]);
        counts[2 * k] = w->epj[k].n;
        counts[2 * k + 1] = w->spj[k].n;
    }
    return w;
}

void or_walk_export(void *wh, uint32_t *epj, uint32_t *spj) {
    walk_res *w = (walk_res *)wh;
    int64_t oe = 0, os = 0;
    for (int64_t k = 0; k < w->nsel; k++) {
        if (w->epj[k].n) memcpy(epj + oe, w->epj[k].v, 4 * w->epj[k].n);
        if (w->spj[k].n) memcpy(spj + os, w->spj[k].v, 4 * w->spj[k].n);
        oe += w->epj[k].n; os += w->spj[k].n;
    }
}
void or_walk_free(void *wh) {
    walk_res *w = (walk_res *)wh;
    if (!w) return;
    for (int64_t k = 0; k < w->nsel; k++) { free(w->epj[k].v); free(w->spj[k].v); }
    free(w->epj); free(w->spj); free(w);
}

/* ------------------------------------------------------------------------------------ */
/* Force on the i-particles of the walked groups from their lists.
 * Particle part (equation ParticleParticleNbody, G = 1, self term excluded):
 *   a += m_j (r_j - r_i) / (|r_j - r_i|^2 + eps_i^2)^{3/2},  phi += -m_j / (...)^{1/2}.
 * Superparticle part (equation ParticleSuperparticleNbody read with the superparticle at
 * r'_j, extended to the quadrupole; r = r_i - X, R^2 = |r|^2 + eps_i^2):
 *   phi += -M/R - (1/2) r.Q.r / R^5
 *   a   += -M r / R^3 + Q r / R^5 - (5/2) (r.Q.r) r / R^7
 * quad = 0 keeps only the monopole (centre-of-mass) terms.
 * Inputs in sorted order; outputs acc[4*i] = {ax, ay, az, phi} at sorted position i. */
void or_force(void *wh, const int64_t *gsel, const uint32_t *gbegin, const uint32_t *gcount,
              const double *sx, const double *sy, const double *sz, const double *sm,
              const double *seps, const double *mom, int32_t quad, double *acc) {
    walk_res *w = (walk_res *)wh;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < w->nsel; k++) {
        int64_t g = gsel[k];
        for (uint32_t i = gbegin[g]; i < gbegin[g] + gcount[g]; i++) {
            double e2 = seps[i] * seps[i];
            nsum ax = {0, 0}, ay = {0, 0}, az = {0, 0}, ph = {0, 0};
            for (int64_t t = 0; t < w->epj[k].n; t++) {
                uint32_t j = w->epj[k].v[t];
                if (j == i) continue;
                double dx = sx[j] - sx[i], dy = sy[j] - sy[i], dz = sz[j] - sz[i];
                double r2 = dx * dx + dy * dy + dz * dz + e2;
                double rinv = 1.0 / sqrt(r2);
                double mr3 = sm[j] * rinv * rinv * rinv;
                nadd(&ax, mr3 * dx); nadd(&ay, mr3 * dy); nadd(&az, mr3 * dz);
                nadd(&ph, -sm[j] * rinv);
            }
            for (int64_t t = 0; t < w->spj[k].n; t++) {
                const double *o = mom + 10 * (size_t)w->spj[k].v[t];
                double rx = sx[i] - o[1], ry = sy[i] - o[2], rz = sz[i] - o[3];
                double R2 = rx * rx + ry * ry + rz * rz + e2;
                double Ri = 1.0 / sqrt(R2);
                double Ri2 = Ri * Ri;
                double Ri3 = Ri * Ri2;
                nadd(&ax, -o[0] * Ri3 * rx); nadd(&ay, -o[0] * Ri3 * ry); nadd(&az, -o[0] * Ri3 * rz);
                nadd(&ph, -o[0] * Ri);
                if (quad) {
                    double qx = o[4] * rx + o[7] * ry + o[8] * rz;
                    double qy = o[7] * rx + o[5] * ry + o[9] * rz;
                    double qz = o[8] * rx + o[9] * ry + o[6] * rz;
                    double rqr = rx * qx + ry * qy + rz * qz;
                    double Ri5 = Ri3 * Ri2, Ri7 = Ri5 * Ri2;
                    nadd(&ax, qx * Ri5 - 2.5 * rqr * rx * Ri7);
                    nadd(&ay, qy * Ri5 - 2.5 * rqr * ry * Ri7);
                    nadd(&az, qz * Ri5 - 2.5 * rqr * rz * Ri7);
                    nadd(&ph, -0.5 * rqr * Ri5);
                }
            }
            acc[4 * (size_t)i] = nval(&ax); acc[4 * (size_t)i + 1] = nval(&ay);
            acc[4 * (size_t)i + 2] = nval(&az); acc[4 * (size_t)i + 3] = nval(&ph);
        }
    }
}

/* ------------------------------------------------------------------------------------ */
/* Short-range neighbour lists and SPH density.  The same tree is traversed for short-range
 * interactions, with four kinds of cutoff length: fixed, j-dependent, i-dependent and
 * symmetric (section "Interaction calculation"); the paper's SPH application uses the
 * Wendland C6 kernel with a cutoff of 4.2 mean interparticle distances, about 300
 * neighbours (section "Giant impact simulation"), and models the list length by equation
 * nlist_short.  Readings:
 *   mode 0 fixed (a pair interacts if r < r_cut), 1 j-dependent "scatter" (r < h_j),
 *   2 i-dependent "gather" (r < h_i), 3 symmetric (r < max(h_i, h_j));
 *   candidate list of a group = the particles of every leaf the walk opens, where a cell is
 *   opened iff the distance between the group's integer box [2 qmin, 2 qmax + 2] and the
 *   cell's cube [C - 2^(21-l), C + 2^(21-l)] (half-grid units, exact integers) satisfies
 *   D^2 <= R^2, R = r * (2^22 / Lr) the search radius in half-grid units (an exact scaling of
 *   the physical radius r, one rounding in R * R); r = r_cut (fixed), the largest h of the
 *   group (gather), the largest h in the cell (scatter), the larger of the two (symmetric);
 *   rho_i = sum_j m_j W(|r_ij|, H) over pairs with |r_ij| < H, j = i included, H = r_cut
 *   (fixed), h_i (gather), h_j (scatter); symmetric: the mean of the gather and the scatter
 *   sums; n_i = number of j (i included) with |r_ij| < H, symmetric H = max(h_i, h_j);
 *   |r_ij|^2 = dx*dx + dy*dy + dz*dz rounded as written, compared with H*H.
 * Wendland C6 kernel (Dehnen & Aly 2012) in three dimensions, q = r / H < 1:
 *   W = 1365 / (64 pi H^3) (1 - q)^8 (1 + 8 q + 25 q^2 + 32 q^3). */
double or_wendland_c6(double r, double H) {
    double q = r / H;
    if (q >= 1.0) return 0.0;
    double u = 1.0 - q, u2 = u * u, u4 = u2 * u2, u8 = u4 * u4;
    const double pi = 3.14159265358979323846;
    return 1365.0 / (64.0 * pi * H * H * H) * u8 * (1.0 + 8.0 * q + 25.0 * q * q + 32.0 * q * q * q);
}

static double pair_r2(double dx, double dy, double dz) { return dx * dx + dy * dy + dz * dz; }

/* one pair's contribution: adds to rho and counts the neighbour */
static void sph_pair(int32_t mode, double r_cut, double r2, double mj, double hi, double hj,
                     nsum *rho, uint32_t *n) {
    double r = sqrt(r2);
    if (mode == 0) {
        if (r2 < r_cut * r_cut) { nadd(rho, mj * or_wendland_c6(r, r_cut)); (*n)++; }
    } else if (mode == 1) {
        if (r2 < hj * hj) { nadd(rho, mj * or_wendland_c6(r, hj)); (*n)++; }
    } else if (mode == 2) {
        if (r2 < hi * hi) { nadd(rho, mj * or_wendland_c6(r, hi)); (*n)++; }
    } else {
        double w = 0.0;
        if (r2 < hi * hi) w += or_wendland_c6(r, hi);
        if (r2 < hj * hj) w += or_wendland_c6(r, hj);
        if (w > 0.0) nadd(rho, 0.5 * mj * w);
        double H = hi > hj ? hi : hj;
        if (r2 < H * H) (*n)++;
    }
}

/* brute force over all pairs of each system (inputs in any order, per system contiguous) */
void or_density_brute(int64_t nsys, const int64_t *off, const double *x, const double *y,
                      const double *z, const double *m, const double *h, int32_t mode,
                      double r_cut, double *rho, uint32_t *nngb) {
    for (int64_t s = 0; s < nsys; s++) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = off[s]; i < off[s + 1]; i++) {
            nsum acc = {0, 0};
            uint32_t n = 0;
            double hi = h ? h[i] : r_cut;
            for (int64_t j = off[s]; j < off[s + 1]; j++) {
                double hj = h ? h[j] : r_cut;
                sph_pair(mode, r_cut, pair_r2(x[j] - x[i], y[j] - y[i], z[j] - z[i]), m[j], hi, hj,
                         &acc, &n);
            }
            rho[i] = nval(&acc);
            nngb[i] = n;
        }
    }
}

/* largest h of every cell's particles (sorted order) */
void or_cell_hmax(void *h, const double *sh, double *hmax) {
    const or_cells *t = (const or_cells *)h;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < t->ncell; c++) {
        double v = 0.0;
        for (uint32_t i = t->begin[c]; i < t->begin[c] + t->count[c]; i++) v = sh[i] > v ? sh[i] : v;
        hmax[c] = v;
    }
}

static void short_visit(const or_cells *t, uint32_t c, const int64_t *lo, const int64_t *hi,
                        int32_t mode, double rg, const double *hmax, double scale, u32vec *epj) {
    if (t->count[c] == 0) return;
    uint32_t cq[3];
    int32_t l = t->level[c];
    deinterleave(t->prefix[c] << (3 * (OR_LEVELS - l)), &cq[0], &cq[1], &cq[2]);
    double D2 = 0.0;
    int64_t half = (int64_t)1 << (OR_LEVELS - l);
    for (int a = 0; a < 3; a++) {
        int64_t C = 2 * (int64_t)cq[a] + half;
        int64_t bmin = 2 * lo[a], bmax = 2 * hi[a] + 2;
        int64_t d = 0;
        if (bmin - (C + half) > d) d = bmin - (C + half);
        if ((C - half) - bmax > d) d = (C - half) - bmax;
        D2 += (double)(d * d);
    }
    double r = mode == 1 ? hmax[c] : (mode == 3 && hmax[c] > rg ? hmax[c] : rg);
    double R = r * scale;
    if (D2 > R * R) return;
    if (t->nchild[c] == 0) {
        for (uint32_t i = t->begin[c]; i < t->begin[c] + t->count[c]; i++) vpush(epj, i);
        return;
    }
    for (uint32_t k = 0; k < t->nchild[c]; k++)
        short_visit(t, t->first_child[c] + k, lo, hi, mode, rg, hmax, scale, epj);
}

/* Candidate lists of all groups (counts[g] = length); rg[g] = the group's search radius for
 * modes 0, 2, 3 (r_cut, or its largest h); hmax per cell for modes 1, 3; cube per system. */
void *or_short_walk(void *h, int64_t ng, const uint32_t *groot, const uint32_t *qmin,
                    const uint32_t *qmax, int32_t mode, const double *rg, const double *hmax,
                    const double *cube, int64_t *counts) {
    const or_cells *t = (const or_cells *)h;
    walk_res *w = (walk_res *)calloc(1, sizeof(walk_res));
    w->nsel = ng;
    w->epj = (u32vec *)calloc((size_t)(ng > 0 ? ng : 1), sizeof(u32vec));
    w->spj = (u32vec *)calloc((size_t)(ng > 0 ? ng : 1), sizeof(u32vec));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t g = 0; g < ng; g++) {
        int64_t lo[3], hi[3];
        for (int a = 0; a < 3; a++) { lo[a] = qmin[3 * g + a]; hi[a] = qmax[3 * g + a]; }
        double scale = 4194304.0 / cube[4 * (size_t)groot[g] + 3];
        short_visit(t, groot[g], lo, hi, mode, rg ? rg[g] : 0.0, hmax, scale, &w->epj[g]);
        counts[g] = w->epj[g].n;
    }
    return w;
}

/* Density and neighbour count of every particle of every group from its candidate list
 * (inputs in sorted order, outputs at sorted positions). */
void or_density_lists(void *wh, const uint32_t *gbegin, const uint32_t *gcount, const double *sx,
                      const double *sy, const double *sz, const double *sm, const double *sh,
                      int32_t mode, double r_cut, double *rho, uint32_t *nngb) {
    walk_res *w = (walk_res *)wh;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t g = 0; g < w->nsel; g++) {
        for (uint32_t i = gbegin[g]; i < gbegin[g] + gcount[g]; i++) {
            nsum acc = {0, 0};
            uint32_t n = 0;
            double hi = sh ? sh[i] : r_cut;
            for (int64_t t = 0; t < w->epj[g].n; t++) {
                uint32_t j = w->epj[g].v[t];
                double hj = sh ? sh[j] : r_cut;
                sph_pair(mode, r_cut, pair_r2(sx[j] - sx[i], sy[j] - sy[i], sz[j] - sz[i]), sm[j], hi,
                         hj, &acc, &n);
            }
            rho[i] = nval(&acc);
            nngb[i] = n;
        }
    }
}

/* ------------------------------------------------------------------------------------ */
/* Tree part of TreePM (section "Cosmological simulation": a monopole-only tree kernel with
 * a cutoff of three mesh widths, theta 0.5, the long-range part on a mesh with the S2 cloud
 * profile of Hockney & Eastwood).  The tree part is Newton's force minus the force between
 * two S2 clouds of diameter r_cut (uniform-gradient spheres: density proportional to
 * r_cut/2 - r), i.e. 1/r^2 times g(xi), xi = 2 r / r_cut:
 *   g = 1 - (224 xi^3 - 224 xi^5 + 70 xi^6 + 48 xi^7 - 21 xi^8) / 140,           xi <= 1
 *   g = 1 - (12 - 224 xi^2 + 896 xi^3 - 840 xi^4 + 224 xi^5 + 70 xi^6 - 48 xi^7 + 7 xi^8) / 140,
 *                                                                                1 <= xi <= 2
 *   g = 0,                                                                       xi >= 2.
 * Readings: softening enters the Newtonian factor only, a = m (r_j - r_i) g(2 r / r_cut) /
 * (r^2 + eps_i^2)^{3/2} with r unsoftened; a superparticle is its monopole at the centre of
 * mass; the walk drops a cell whose cube lies farther than r_cut from the group's box (every
 * pair in it has g = 0; test as for the short-range walk, R = r_cut * 2^22 / Lr) and applies
 * the opening test to the others; no potential. */
double or_s2_cutoff(double xi) {
    if (xi >= 2.0) return 0.0;
    double x2 = xi * xi, x3 = x2 * xi, x4 = x2 * x2, x5 = x4 * xi, x6 = x3 * x3, x7 = x6 * xi,
           x8 = x4 * x4;
    if (xi <= 1.0) return 1.0 - (224.0 * x3 - 224.0 * x5 + 70.0 * x6 + 48.0 * x7 - 21.0 * x8) / 140.0;
    return 1.0 - (12.0 - 224.0 * x2 + 896.0 * x3 - 840.0 * x4 + 224.0 * x5 + 70.0 * x6 - 48.0 * x7 +
                  7.0 * x8) / 140.0;
}

/* all pairs of each system, caller's order, acc[3 i] */
void or_direct_cutoff(int64_t nsys, const int64_t *off, const double *x, const double *y,
                      const double *z, const double *m, const double *eps, double r_cut,
                      double *acc) {
    for (int64_t s = 0; s < nsys; s++) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = off[s]; i < off[s + 1]; i++) {
            nsum ax = {0, 0}, ay = {0, 0}, az = {0, 0};
            double e2 = eps[i] * eps[i];
            for (int64_t j = off[s]; j < off[s + 1]; j++) {
                if (j == i) continue;
                double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
                double r2 = dx * dx + dy * dy + dz * dz;
                double g = or_s2_cutoff(2.0 * sqrt(r2) / r_cut);
                if (g == 0.0) continue;
                double rinv = 1.0 / sqrt(r2 + e2);
                double f = m[j] * rinv * rinv * rinv * g;
                nadd(&ax, f * dx); nadd(&ay, f * dy); nadd(&az, f * dz);
            }
            acc[3 * i] = nval(&ax); acc[3 * i + 1] = nval(&ay); acc[3 * i + 2] = nval(&az);
        }
    }
}

static void cutoff_visit(const or_cells *t, uint32_t c, const int64_t *lo, const int64_t *hi,
                         double th2, double R2, u32vec *epj, u32vec *spj) {
    if (t->count[c] == 0) return;
    uint32_t cq[3];
    int32_t l = t->level[c];
    deinterleave(t->prefix[c] << (3 * (OR_LEVELS - l)), &cq[0], &cq[1], &cq[2]);
    double D2 = 0.0;
    int64_t half = (int64_t)1 << (OR_LEVELS - l);
    for (int a = 0; a < 3; a++) {
        int64_t C = 2 * (int64_t)cq[a] + half;
        int64_t bmin = 2 * lo[a], bmax = 2 * hi[a] + 2;
        int64_t d = 0;
        if (bmin - (C + half) > d) d = bmin - (C + half);
        if ((C - half) - bmax > d) d = (C - half) - bmax;
        D2 += (double)(d * d);
    }
    if (D2 > R2) return;
    if (accept_cell(l, t->prefix[c], lo, hi, th2)) { vpush(spj, c); return; }
    if (t->nchild[c] == 0) {
        for (uint32_t i = t->begin[c]; i < t->begin[c] + t->count[c]; i++) vpush(epj, i);
        return;
    }
    for (uint32_t k = 0; k < t->nchild[c]; k++)
        cutoff_visit(t, t->first_child[c] + k, lo, hi, th2, R2, epj, spj);
}

void *or_walk_cutoff(void *h, int64_t ng, const uint32_t *groot, const uint32_t *qmin,
                     const uint32_t *qmax, double theta, double r_cut, const double *cube,
                     int64_t *counts) {
    const or_cells *t = (const or_cells *)h;
    walk_res *w = (walk_res *)calloc(1, sizeof(walk_res));
    w->nsel = ng;
    w->epj = (u32vec *)calloc((size_t)(ng > 0 ? ng : 1), sizeof(u32vec));
    w->spj = (u32vec *)calloc((size_t)(ng > 0 ? ng : 1), sizeof(u32vec));
    double th2 = theta * theta;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t g = 0; g < ng; g++) {
        int64_t lo[3], hi[3];
        for (int a = 0; a < 3; a++) { lo[a] = qmin[3 * g + a]; hi[a] = qmax[3 * g + a]; }
        double R = r_cut * (4194304.0 / cube[4 * (size_t)groot[g] + 3]);
        cutoff_visit(t, groot[g], lo, hi, th2, R * R, &w->epj[g], &w->spj[g]);
        counts[2 * g] = w->epj[g].n;
        counts[2 * g + 1] = w->spj[g].n;
    }
    return w;
}

/* acceleration of every group member from its lists (sorted order, acc[3 i]) */
void or_force_cutoff(void *wh, const uint32_t *gbegin, const uint32_t *gcount, const double *sx,
                     const double *sy, const double *sz, const double *sm, const double *seps,
                     const double *mom, double r_cut, double *acc) {
    walk_res *w = (walk_res *)wh;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t g = 0; g < w->nsel; g++) {
        for (uint32_t i = gbegin[g]; i < gbegin[g] + gcount[g]; i++) {
            double e2 = seps[i] * seps[i];
            nsum ax = {0, 0}, ay = {0, 0}, az = {0, 0};
            for (int64_t t = 0; t < w->epj[g].n; t++) {
                uint32_t j = w->epj[g].v[t];
                if (j == i) continue;
                double dx = sx[j] - sx[i], dy = sy[j] - sy[i], dz = sz[j] - sz[i];
                double r2 = dx * dx + dy * dy + dz * dz;
                double gc = or_s2_cutoff(2.0 * sqrt(r2) / r_cut);
                double rinv = 1.0 / sqrt(r2 + e2);
                double f = sm[j] * rinv * rinv * rinv * gc;
                nadd(&ax, f * dx); nadd(&ay, f * dy); nadd(&az, f * dz);
            }
            for (int64_t t = 0; t < w->spj[g].n; t++) {
                const double *o = mom + 10 * (size_t)w->spj[g].v[t];
                double dx = o[1] - sx[i], dy = o[2] - sy[i], dz = o[3] - sz[i];
                double r2 = dx * dx + dy * dy + dz * dz;
                double gc = or_s2_cutoff(2.0 * sqrt(r2) / r_cut);
                double rinv = 1.0 / sqrt(r2 + e2);
                double f = o[0] * rinv * rinv * rinv * gc;
                nadd(&ax, f * dx); nadd(&ay, f * dy); nadd(&az, f * dz);
            }
            acc[3 * (size_t)i] = nval(&ax); acc[3 * (size_t)i + 1] = nval(&ay);
            acc[3 * (size_t)i + 2] = nval(&az);
        }
    }
}

/* ------------------------------------------------------------------------------------ */
/* Domain decomposition (section "Domain decomposition"): the multisection method with
 * the sampling method.  The domains are n_x n_y n_z boxes; the division is applied once
 * per axis -- n_x slabs in x, each slab cut into n_y columns in y, each column into n_z
 * domains in z -- so that the sample particles are equally divided.  The current domains
 * (the systems of the particle set) each draw a number of samples proportional to their
 * cost, so that every sample stands for the same amount of work.
 * Readings (the paper does not fix them):
 *   - samples are drawn with replacement, uniformly over the domain's particles: sample s
 *     of a domain with n_p particles starting at off_p is particle
 *     off_p + floor(r * n_p / 2^64), r = SplitMix64 output number s for the seed;
 *   - a division sorts the samples of a segment by coordinate (ties by sample number) and
 *     cuts them into runs of equal count, run i being the sorted ranks
 *     [floor(i K / n), floor((i + 1) K / n)); each cut lies at the midpoint of the two
 *     samples on either side of it, the outer faces are -inf and +inf;
 *   - a particle belongs to the domain whose box holds it, lower faces closed and upper
 *     faces open. */

/* SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014): a Weyl sequence with increment 0x9E3779B97F4A7C15 followed by a 64-bit
 * finaliser.  Output number ctr (0-based) of the generator seeded with seed. */
uint64_t or_splitmix64(uint64_t seed, uint64_t ctr) {
    uint64_t z = seed + (ctr + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* particle index of every sample: k[p] samples of current domain p (particles
 * [off[p], off[p+1])), numbered consecutively over the domains in order */
void or_dd_sample(int64_t nsys, const int64_t *off, const int64_t *k, uint64_t seed,
                  uint32_t *idx) {
    uint64_t s = 0;
    for (int64_t p = 0; p < nsys; p++) {
        uint64_t np = (uint64_t)(off[p + 1] - off[p]);
        for (int64_t j = 0; j < k[p]; j++, s++) {
            unsigned __int128 prod = (unsigned __int128)or_splitmix64(seed, s) * np;
            idx[s] = (uint32_t)(off[p] + (int64_t)(uint64_t)(prod >> 64));
        }
    }
}

typedef struct { double v; uint32_t s; } dd_item;

static int dd_cmp(const void *a, const void *b) {
    const dd_item *x = (const dd_item *)a, *y = (const dd_item *)b;
    if (x->v < y->v) return -1;
    if (x->v > y->v) return 1;
    return (x->s > y->s) - (x->s < y->s);
}

/* Divide the samples listed in items[0..K) (sorted here in place by coordinate v, ties by
 * sample number) into n runs of equal count: run i of the sorted ranks is
 * [floor(i K / n), floor((i + 1) K / n)).  b[0..n] receives the faces (b[0] = -inf,
 * b[n] = +inf, b[i] = midpoint of the samples at ranks floor(i K / n) - 1 and floor(i K / n))
 * and run[t] the run of the t-th sorted sample. */
static void dd_divide(dd_item *items, int64_t K, int n, double *b, int *run) {
    qsort(items, (size_t)K, sizeof(dd_item), dd_cmp);
    b[0] = -INFINITY;
    b[n] = INFINITY;
    for (int i = 1; i < n; i++) {
        int64_t r = (int64_t)i * K / n;
        b[i] = (items[r - 1].v + items[r].v) * 0.5;
    }
    for (int i = 0; i < n; i++)
        for (int64_t t = (int64_t)i * K / n; t < (int64_t)(i + 1) * K / n; t++) run[t] = i;
}

/* The multisection of K samples (coordinates sx, sy, sz; sample number = position) into
 * nx x ny x nz domains.  Needs K >= nx ny nz so that every run holds a sample.  Outputs the
 * faces bx[nx+1], by[nx][ny+1], bz[nx][ny][nz+1] and the domain (ix ny + iy) nz + iz of
 * every sample.  Returns 0, or -1 when K is too small. */
int or_dd_multisection(int64_t K, const double *sx, const double *sy, const double *sz, int nx,
                       int ny, int nz, double *bx, double *by, double *bz, uint32_t *cell) {
    if (K < (int64_t)nx * ny * nz) return -1;
    dd_item *it = (dd_item *)malloc(sizeof(dd_item) * (size_t)(K > 0 ? K : 1));
    dd_item *sub = (dd_item *)malloc(sizeof(dd_item) * (size_t)(K > 0 ? K : 1));
    int *run = (int *)malloc(sizeof(int) * (size_t)(K > 0 ? K : 1));
    int *ix = (int *)malloc(sizeof(int) * (size_t)(K > 0 ? K : 1));
    int *iy = (int *)malloc(sizeof(int) * (size_t)(K > 0 ? K : 1));
    /* x: all samples */
    for (int64_t s = 0; s < K; s++) { it[s].v = sx[s]; it[s].s = (uint32_t)s; }
    dd_divide(it, K, nx, bx, run);
    for (int64_t t = 0; t < K; t++) ix[it[t].s] = run[t];
    /* y: the samples of each slab */
    for (int a = 0; a < nx; a++) {
        int64_t m = 0;
        for (int64_t s = 0; s < K; s++)
            if (ix[s] == a) { sub[m].v = sy[s]; sub[m].s = (uint32_t)s; m++; }
        dd_divide(sub, m, ny, by + (size_t)a * (ny + 1), run);
        for (int64_t t = 0; t < m; t++) iy[sub[t].s] = run[t];
    }
    /* z: the samples of each column */
    for (int a = 0; a < nx; a++)
        for (int c = 0; c < ny; c++) {
            int64_t m = 0;
            for (int64_t s = 0; s < K; s++)
                if (ix[s] == a && iy[s] == c) { sub[m].v = sz[s]; sub[m].s = (uint32_t)s; m++; }
            int col = a * ny + c;
            dd_divide(sub, m, nz, bz + (size_t)col * (nz + 1), run);
            for (int64_t t = 0; t < m; t++) cell[sub[t].s] = (uint32_t)(col * nz + run[t]);
        }
    free(it); free(sub); free(run); free(ix); free(iy);
    return 0;
}

/* number of faces b[1..n-1] at or below v: the run of [b[i], b[i+1]) that holds v */
static int dd_run_of(const double *b, int n, double v) {
    int i = 0;
    for (int j = 1; j < n; j++)
        if (b[j] <= v) i = j;
    return i;
}

/* destination domain of every particle: the box of the multisection that holds it */
void or_dd_assign(int64_t n, const double *x, const double *y, const double *z, int nx, int ny,
                  int nz, const double *bx, const double *by, const double *bz, uint32_t *dest) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        int a = dd_run_of(bx, nx, x[i]);
        int c = dd_run_of(by + (size_t)a * (ny + 1), ny, y[i]);
        int col = a * ny + c;
        int e = dd_run_of(bz + (size_t)col * (nz + 1), nz, z[i]);
        dest[i] = (uint32_t)(col * nz + e);
    }
}
