/*
 * og_oracle.c -- CPU oracle for the occupancy-grid ray sampler.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or helper with the
 * HIP library.
 *
 * What it computes (Kato & Tarashima, "Plug-and-Play Acceleration of
 * Occupancy Grid-based NeRF Rendering using VDB Grid and Hierarchical Ray
 * Traversal", 2024): for every camera ray, the fixed-step sample points that
 * fall in occupied voxels of a binary occupancy grid (Sec. 3, Alg. 1 and
 * Alg. 2 of the supplementary material), optionally over several nested
 * cascade grids where the finest grid that contains a point decides its
 * occupancy (Sec. 3, last paragraph).
 *
 * The paper does not spell out the floating-point definition of "the voxel a
 * point belongs to", so this file fixes one (every decision in IEEE binary32,
 * one rounding per operation, no fused multiply-add):
 *
 *   voxel size        h_a   = fl((A_a - B_a) / R)           box [B, A], res R
 *   plane m           P_a(m) = fl(B_a + fl(float(m) * h_a))  m = 0..R
 *   reciprocal        r_a   = fl(1 / d_a)
 *   crossing          T_a(m) = fl(fl(P_a(m) - o_a) * r_a)
 *   zero axis         d_a == 0 or r_a infinite: the coordinate never changes
 *   ownership of t    d_a > 0: c_a = #{m : T_a(m) < t} - 1
 *                     d_a < 0: c_a = R - #{m : T_a(m) < t}
 *                     zero axis: c_a = -1 if o_a < P_a(0),
 *                                else #{m in 1..R : P_a(m) <= o_a}
 *                     i.e. a voxel owns the half-open parameter range
 *                     (entry, exit]; a point on a face belongs to the voxel
 *                     the ray leaves (the "<=" tests of Alg. 1).
 *   level of t        the smallest cascade index whose voxel is inside
 *   lattice           constant:  t_n = fl(t_min + fl(float(n) * dt))
 *                     growing:   t_0 = t_min,
 *                                t_{n+1} = fl(t_n + max(fl(t_n * c), dt_min))
 *   samples           { n >= 0 : t_n <= t_max and occupied(t_n) },
 *                     emitted as (t_n, t_{n+1}, voxel id) in increasing n;
 *                     voxel id = ((level * R + i) * R + j) * R + k.
 *   A ray with a non-finite origin or direction, or t_min > t_max, has none.
 *
 * Three independent ways of reaching that sample set:
 *   method 0  brute force: test every lattice point by the ownership rule;
 *   method 1/2  dense-grid DDA over voxels, driven as in Alg. 1 (branch) or
 *             Alg. 2 (skip);
 *   method 3/4  a VDB tree (root table -> internal node -> 8^3 leaf, with
 *             uniform blocks pruned into tiles, Sec. 3) and a level-adaptive
 *             DDA that steps over a whole tile at once (HDDA, Sec. 2.3),
 *             driven as in Alg. 1 or Alg. 2;
 *   method 5/6  the same tree and DDA, where inside a leaf the cell is the
 *             aligned 4^3 sub-block holding the voxel when it is uniform (all
 *             empty or all occupied), else the voxel: empty space is passed by
 *             powers of two down to single voxels (Fig. 1), driven as in
 *             Alg. 1 or Alg. 2.
 * Every way also reports how many cells a ray's walk visits (orc_cells).
 *
 * Readings of the algorithms (where the printed text is ambiguous):
 *   - Alg. 2's inner "repeat ... until" loop is read as "repeat until the
 *     voxel is occupied", and each repeat resumes where the previous cell
 *     ended (not from t_min); if no occupied cell is left the ray ends.
 *   - Both algorithms stop emitting at t_max: only t_n <= t_max are samples,
 *     while t1 = t_{n+1} is not clipped.
 *   - When the analyzer runs past the grid it returns nothing and the ray
 *     ends.
 *
 * Plain code on purpose: linear plane counts, byte-per-voxel grids, no
 * blocking or fusion.  Build: gcc -O2 -ffp-contract=off -fopenmp (no
 * -ffast-math; x86-64 SSE arithmetic rounds every binary32 operation once).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_LEVELS 8

typedef struct {
    int32_t L;            /* number of cascade levels, finest first */
    int32_t R;            /* voxels per axis, same for every level */
    const float *box;     /* [L][6]: min x,y,z then max x,y,z */
    const uint8_t *occ;   /* [L][R][R][R], x slowest, z fastest; nonzero = occupied */
} orc_grid;

typedef struct {
    int32_t kind;         /* 0 constant step, 1 growing (cone) step */
    float dt;             /* constant step */
    float cone;           /* growing step: dt_n = max(t_n * cone, dt_min) */
    float dt_min;
} orc_step;

/* ------------------------------------------------------------------ */
/* The oracle's own VDB tree: plain arrays, one byte per voxel in leaves. */

typedef struct {
    int32_t L, R, ilog2;  /* internal node = 2^ilog2 leaf blocks per axis */
    int32_t D;            /* voxels per axis covered by one root cell = 8 << ilog2 */
    int32_t NR;           /* root cells per axis = ceil(R / D) */
    int32_t S;            /* leaf slots per internal node per axis = 1 << ilog2 */
    int8_t *root_kind;    /* [L][NR^3]: 0 empty tile, 1 full tile, 2 node */
    int32_t *root_node;   /* [L][NR^3]: node index when kind == 2 */
    int32_t n_nodes;
    int8_t *slot_kind;    /* [n_nodes][S^3]: 0 empty tile, 1 full tile, 2 leaf */
    int32_t *slot_leaf;   /* [n_nodes][S^3]: leaf index when kind == 2 */
    int32_t n_leaves;
    uint8_t *leaf_vox;    /* [n_leaves][8][8][8] */
    int64_t n_slot_full, n_slot_empty, n_root_full, n_root_empty;
} orc_vdb;

/* ------------------------------------------------------------------ */
/* Canonical binary32 geometry (see the header comment). */

static float voxel_size(const float *box, int R, int a)
{
    return (box[3 + a] - box[a]) / (float)R;
}

static float plane_pos(const float *box, int R, int a, int m)
{
    float h = voxel_size(box, R, a);
    float mh = (float)m * h;
    return box[a] + mh;
}

typedef struct {
    int L, R;
    const float *box;
    const uint8_t *occ;
    float o[3], d[3], r[3];
    int zero[3];
    float *T;             /* [L][3][R+1] crossing parameters T_a(m) */
    float *P;             /* [L][3][R+1] plane positions P_a(m) */
} ray_ctx;

static float *T_of(const ray_ctx *x, int lev, int a) { return x->T + ((size_t)lev * 3 + a) * (x->R + 1); }
static float *P_of(const ray_ctx *x, int lev, int a) { return x->P + ((size_t)lev * 3 + a) * (x->R + 1); }

static int ray_init(ray_ctx *x, const orc_grid *g, const float *o, const float *d)
{
    x->L = g->L;
    x->R = g->R;
    x->box = g->box;
    x->occ = g->occ;
    for (int a = 0; a < 3; ++a) {
        if (!isfinite(o[a]) || !isfinite(d[a])) return 0;
        x->o[a] = o[a];
        x->d[a] = d[a];
        x->r[a] = 1.0f / d[a];
        x->zero[a] = (d[a] == 0.0f) || isinf(x->r[a]);
    }
    size_t n = (size_t)g->L * 3 * (g->R + 1);
    x->T = (float *)malloc(n * sizeof(float));
    x->P = (float *)malloc(n * sizeof(float));
    for (int lev = 0; lev < g->L; ++lev)
        for (int a = 0; a < 3; ++a) {
            float *T = T_of(x, lev, a), *P = P_of(x, lev, a);
            for (int m = 0; m <= g->R; ++m) {
                P[m] = plane_pos(g->box + 6 * lev, g->R, a, m);
                float diff = P[m] - x->o[a];
                T[m] = diff * x->r[a];
            }
        }
    return 1;
}

static void ray_free(ray_ctx *x)
{
    free(x->T);
    free(x->P);
}

/* Number of planes m in 0..R with T(m) < t (inclusive = 0) or T(m) <= t
 * (inclusive = 1).  A plain linear count. */
static int count_planes(const float *T, int R, float t, int inclusive)
{
    int k = 0;
    for (int m = 0; m <= R; ++m)
        if (inclusive ? (T[m] <= t) : (T[m] < t)) ++k;
    return k;
}

/* Voxel coordinate on axis a that owns parameter t (inclusive = 0), or that
 * owns the parameters just above t (inclusive = 1).  May be outside 0..R-1. */
static int axis_cell(const ray_ctx *x, int lev, int a, float t, int inclusive)
{
    int R = x->R;
    if (x->zero[a]) {
        const float *P = P_of(x, lev, a);
        if (x->o[a] < P[0]) return -1;
        int c = 0;
        for (int m = 1; m <= R; ++m)
            if (P[m] <= x->o[a]) ++c;
        return c;
    }
    int k = count_planes(T_of(x, lev, a), R, t, inclusive);
    return x->d[a] > 0.0f ? k - 1 : R - k;
}

static int inside(int R, const int *c)
{
    return c[0] >= 0 && c[0] < R && c[1] >= 0 && c[1] < R && c[2] >= 0 && c[2] < R;
}

/* Level and voxel owning t: the finest level whose voxel is inside. */
static int locate(const ray_ctx *x, float t, int *lev_out, int *c)
{
    for (int lev = 0; lev < x->L; ++lev) {
        for (int a = 0; a < 3; ++a) c[a] = axis_cell(x, lev, a, t, 0);
        if (inside(x->R, c)) {
            *lev_out = lev;
            return 1;
        }
    }
    return 0;
}

/* Debug id ((lev*R + i)*R + j)*R + k, formed in 64 bits; callers ask for
 * ids only on grids whose ids fit in int32 (n_levels * R^3 <= 2^31). */
static int32_t voxel_id(int R, int lev, const int *c)
{
    return (int32_t)((((int64_t)lev * R + c[0]) * R + c[1]) * R + c[2]);
}

static int occupied(const ray_ctx *x, int lev, const int *c)
{
    size_t R = (size_t)x->R;
    return x->occ[(((size_t)lev * R + c[0]) * R + c[1]) * R + c[2]] != 0;
}

/* ------------------------------------------------------------------ */
/* Lattice of sample parameters. */

typedef struct {
    const orc_step *s;
    float tmin;
    int64_t n;
    float t, tnext;
} lattice;

static float lattice_const(const orc_step *s, float tmin, int64_t n)
{
    float nd = (float)n * s->dt;
    return tmin + nd;
}

static float cone_next(const orc_step *s, float t)
{
    float grow = t * s->cone;
    float dt = grow > s->dt_min ? grow : s->dt_min;
    return t + dt;
}

static void lat_init(lattice *q, const orc_step *s, float tmin)
{
    q->s = s;
    q->tmin = tmin;
    q->n = 0;
    q->t = tmin;
    q->tnext = s->kind == 0 ? lattice_const(s, tmin, 1) : cone_next(s, tmin);
}

static void lat_advance(lattice *q)
{
    q->n += 1;
    q->t = q->tnext;
    q->tnext = q->s->kind == 0 ? lattice_const(q->s, q->tmin, q->n + 1) : cone_next(q->s, q->t);
}

/* ------------------------------------------------------------------ */
/* Sample sink. */

typedef struct {
    int64_t count, cap;
    float *t0, *t1;
    int32_t *vox;
} sink;

static void emit(sink *k, float t0, float t1, int32_t vox)
{
    if (k->count < k->cap) {
        if (k->t0) k->t0[k->count] = t0;
        if (k->t1) k->t1[k->count] = t1;
        if (k->vox) k->vox[k->count] = vox;
    }
    k->count += 1;
}

/* ------------------------------------------------------------------ */
/* Method 0: brute force over the lattice. */

static void brute_force(const ray_ctx *x, const orc_step *s, float tmin, float tmax, sink *out)
{
    lattice q;
    for (lat_init(&q, s, tmin); q.t <= tmax; lat_advance(&q)) {
        int lev, c[3];
        if (locate(x, q.t, &lev, c) && occupied(x, lev, c))
            emit(out, q.t, q.tnext, voxel_id(x->R, lev, c));
    }
}

/* ------------------------------------------------------------------ */
/* Which level owns which stretch of the ray.  Level l contains exactly the
 * parameters in (E_l, X_l]; the owner of a parameter is the finest level
 * that contains it.  Between two consecutive breakpoints the owner is
 * constant, so the ray splits into segments (p, q] with one owner each. */

typedef struct {
    float a, b;
    int lev;
} segment;

static int level_span(const ray_ctx *x, int lev, float *E, float *X)
{
    float e = -INFINITY, xx = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (x->zero[a]) {
            int c = axis_cell(x, lev, a, 0.0f, 0);
            if (c < 0 || c >= x->R) return 0;
            continue;
        }
        const float *T = T_of(x, lev, a);
        float lo = T[0] < T[x->R] ? T[0] : T[x->R];
        float hi = T[0] < T[x->R] ? T[x->R] : T[0];
        if (lo > e) e = lo;
        if (hi < xx) xx = hi;
    }
    *E = e;
    *X = xx;
    return e < xx;
}

static int cmp_float(const void *p, const void *q)
{
    float a = *(const float *)p, b = *(const float *)q;
    return (a > b) - (a < b);
}

static int ray_segments(const ray_ctx *x, segment *seg)
{
    float E[ORC_MAX_LEVELS], X[ORC_MAX_LEVELS], bp[2 * ORC_MAX_LEVELS];
    int hit[ORC_MAX_LEVELS], nb = 0, ns = 0;
    for (int lev = 0; lev < x->L; ++lev) {
        hit[lev] = level_span(x, lev, &E[lev], &X[lev]);
        if (hit[lev]) {
            bp[nb++] = E[lev];
            bp[nb++] = X[lev];
        }
    }
    qsort(bp, nb, sizeof(float), cmp_float);
    for (int i = 0; i + 1 < nb; ++i) {
        float p = bp[i], q = bp[i + 1];
        if (!(p < q)) continue;
        for (int lev = 0; lev < x->L; ++lev)
            if (hit[lev] && E[lev] <= p && X[lev] >= q) {
                seg[ns].a = p;
                seg[ns].b = q;
                seg[ns].lev = lev;
                ++ns;
                break;
            }
    }
    return ns;
}

/* ------------------------------------------------------------------ */
/* Analyzers: enumerate consecutive cells of one level inside one segment,
 * each with its parameter interval (t0, t1] and its occupancy. */

typedef struct {
    const ray_ctx *x;
    const orc_vdb *vdb;   /* NULL: dense voxel DDA; else level-adaptive HDDA */
    int sub;              /* HDDA only: leaf voxels merge into uniform 4^3 sub-blocks */
    int lev;
    int c[3];
    float seg_a, seg_b;
    float t_cur;          /* lower end of the next cell's interval (HDDA) */
    int live;
} analyzer;

/* Lower and upper crossing of the voxel on axis a (zero axis: unbounded). */
static void axis_bounds(const ray_ctx *x, int lev, int a, int lo_m, int hi_m, float *lo, float *hi)
{
    if (x->zero[a]) {
        *lo = -INFINITY;
        *hi = INFINITY;
        return;
    }
    const float *T = T_of(x, lev, a);
    if (x->d[a] > 0.0f) {
        *lo = T[lo_m];
        *hi = T[hi_m];
    } else {
        *lo = T[hi_m];
        *hi = T[lo_m];
    }
}

static void analyzer_start(analyzer *z, const ray_ctx *x, const orc_vdb *vdb, int sub, const segment *s,
                           float tmin)
{
    z->x = x;
    z->vdb = vdb;
    z->sub = sub;
    z->lev = s->lev;
    z->seg_a = s->a;
    z->seg_b = s->b;
    z->live = 1;
    /* Start at the voxel owning t_min if t_min lies after the segment start,
     * else at the voxel owning the parameters just after the start. */
    int after = tmin > s->a;
    float ts = after ? tmin : s->a;
    for (int a = 0; a < 3; ++a) z->c[a] = axis_cell(x, s->lev, a, ts, !after);
    z->t_cur = after ? nextafterf(tmin, -INFINITY) : s->a;
    if (!inside(x->R, z->c)) z->live = 0;
}

/* 1 if the aligned cube of e^3 voxels at (b0, b1, b2) inside leaf `leaf`
 * holds one value throughout. */
static int leaf_cube_uniform(const orc_vdb *v, int32_t leaf, int b0, int b1, int b2, int e)
{
    const uint8_t *L = v->leaf_vox + (size_t)leaf * 512;
    uint8_t first = L[(b0 * 8 + b1) * 8 + b2];
    for (int i = b0; i < b0 + e; ++i)
        for (int j = b1; j < b1 + e; ++j)
            for (int k = b2; k < b2 + e; ++k)
                if (L[(i * 8 + j) * 8 + k] != first) return 0;
    return 1;
}

/* The VDB cell holding voxel c: its edge length in voxels and occupancy.
 * With sub, a leaf voxel's cell is the aligned 4^3 sub-block of its leaf
 * holding it when that is uniform, else the voxel itself. */
static void vdb_lookup(const orc_vdb *v, int lev, const int *c, int sub, int *D, int *occ_out)
{
    int rc[3], sl[3], lc[3];
    for (int a = 0; a < 3; ++a) {
        rc[a] = c[a] / v->D;
        sl[a] = (c[a] / 8) % v->S;
        lc[a] = c[a] % 8;
    }
    size_t ri = (size_t)lev * v->NR * v->NR * v->NR + ((size_t)rc[0] * v->NR + rc[1]) * v->NR + rc[2];
    if (v->root_kind[ri] != 2) {
        *D = v->D;
        *occ_out = v->root_kind[ri];
        return;
    }
    size_t si = (size_t)v->root_node[ri] * v->S * v->S * v->S + ((size_t)sl[0] * v->S + sl[1]) * v->S + sl[2];
    if (v->slot_kind[si] != 2) {
        *D = 8;
        *occ_out = v->slot_kind[si];
        return;
    }
    const int32_t leaf = v->slot_leaf[si];
    *D = 1;
    *occ_out = v->leaf_vox[(size_t)leaf * 512 + (lc[0] * 8 + lc[1]) * 8 + lc[2]] != 0;
    if (sub && leaf_cube_uniform(v, leaf, lc[0] / 4 * 4, lc[1] / 4 * 4, lc[2] / 4 * 4, 4)) *D = 4;
}

/* Next cell: returns 0 when the segment is exhausted. */
static int analyzer_next(analyzer *z, int *cell, float *t0, float *t1, int *occ_out)
{
    if (!z->live) return 0;
    const ray_ctx *x = z->x;
    int R = x->R;
    if (z->vdb == NULL) {
        /* Voxel DDA: the cell interval is (max lower crossing, min upper crossing]. */
        float lo = -INFINITY, hi = INFINITY;
        int step_axis = -1;
        for (int a = 0; a < 3; ++a) {
            float l, h;
            axis_bounds(x, z->lev, a, z->c[a], z->c[a] + 1, &l, &h);
            if (l > lo) lo = l;
            if (h < hi) {
                hi = h;
                step_axis = a;
            }
        }
        for (int a = 0; a < 3; ++a) cell[a] = z->c[a];
        *t0 = lo > z->seg_a ? lo : z->seg_a;
        *t1 = hi < z->seg_b ? hi : z->seg_b;
        *occ_out = occupied(x, z->lev, z->c);
        if (hi >= z->seg_b || step_axis < 0) {
            z->live = 0;
        } else {
            z->c[step_axis] += x->d[step_axis] > 0.0f ? 1 : -1;
            if (!inside(R, z->c)) z->live = 0;
        }
        return 1;
    }
    /* Level-adaptive DDA: the cell is the largest uniform VDB cell (root
     * tile, internal tile or voxel) that holds the current voxel. */
    int D, occ;
    vdb_lookup(z->vdb, z->lev, z->c, z->sub, &D, &occ);
    float exit_t = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (x->zero[a]) continue;
        int base = (z->c[a] / D) * D;
        int m = x->d[a] > 0.0f ? base + D : base;
        /* crossing of a plane possibly beyond the grid (tiles that stick out) */
        float P = plane_pos(x->box + 6 * z->lev, R, a, m);
        float diff = P - x->o[a];
        float T = diff * x->r[a];
        if (T < exit_t) exit_t = T;
    }
    for (int a = 0; a < 3; ++a) cell[a] = z->c[a];
    *t0 = z->t_cur;
    *t1 = exit_t < z->seg_b ? exit_t : z->seg_b;
    *occ_out = occ;
    if (exit_t >= z->seg_b) {
        z->live = 0;
    } else {
        /* the voxel that owns the parameters just after the cell's exit */
        for (int a = 0; a < 3; ++a)
            if (!x->zero[a]) z->c[a] = axis_cell(x, z->lev, a, exit_t, 1);
        z->t_cur = exit_t;
        if (!inside(R, z->c)) z->live = 0;
    }
    return 1;
}

/* ------------------------------------------------------------------ */
/* Alg. 1 (branch) and Alg. 2 (skip) drivers, over the ray's segments. */

static int32_t sample_voxel_id(const ray_ctx *x, const analyzer *z, const int *cell, float t)
{
    if (z->vdb == NULL) return voxel_id(x->R, z->lev, cell);
    /* a tile covers many voxels: name the voxel that owns t itself */
    int c[3];
    for (int a = 0; a < 3; ++a) c[a] = axis_cell(x, z->lev, a, t, 0);
    return voxel_id(x->R, z->lev, c);
}

/* The samples a cell holds: the lattice points in its parameter interval
 * (t0, t1] (a voxel owns (entry, exit], the reading of Alg. 1's tests), none
 * beyond tmax.  The lattice only moves forward, as the cells of a ray come
 * in increasing t. */
static void emit_cell(lattice *q, float t0, float t1, float tmax, const ray_ctx *x, const analyzer *z,
                      const int *cell, sink *out)
{
    while (q->t <= t0) lat_advance(q);
    for (; q->t <= t1 && q->t <= tmax; lat_advance(q)) emit(out, q->t, q->tnext, sample_voxel_id(x, z, cell, q->t));
}

/* The next cell the loop looks at: with skip = 0 the next cell along the ray
 * whatever it holds (Alg. 1 visits every cell and tests it); with skip = 1
 * the next occupied one, passing all empty cells before it (Alg. 2).  0 when
 * the segment has no such cell left.  *visited counts every cell the
 * analyzer returns, occupied or not. */
static int next_cell(analyzer *z, int skip, int *cell, float *t0, float *t1, int *occ, int64_t *visited)
{
    do {
        if (!analyzer_next(z, cell, t0, t1, occ)) return 0;
        *visited += 1;
    } while (skip && !*occ);
    return 1;
}

/* All samples of a ray: each segment's cells in ray order, every occupied
 * cell giving the lattice points it holds.  Both loop structures find the
 * same occupied cells, so they give the same samples. */
static void march(const ray_ctx *x, const orc_vdb *vdb, int sub, int skip, const orc_step *s, float tmin,
                  float tmax, sink *out, int64_t *visited)
{
    segment seg[2 * ORC_MAX_LEVELS];
    int ns = ray_segments(x, seg);
    lattice q;
    lat_init(&q, s, tmin);
    for (int si = 0; si < ns && q.t <= tmax; ++si) {
        if (seg[si].b < q.t) continue;  /* holds no lattice point still ahead */
        analyzer z;
        analyzer_start(&z, x, vdb, sub, &seg[si], tmin);
        int cell[3], occ;
        float t0, t1;
        while (q.t <= tmax && next_cell(&z, skip, cell, &t0, &t1, &occ, visited)) {
            if (t0 >= tmax) break;  /* a cell starting at or past tmax holds no sample */
            if (occ) emit_cell(&q, t0, t1, tmax, x, &z, cell, out);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Public entry points (ctypes). */

static int64_t ray_run(const orc_grid *g, const orc_vdb *vdb, const orc_step *s, const float *o, const float *d,
                       float tmin, float tmax, int32_t method, float *t0, float *t1, int32_t *vox, int64_t cap,
                       int64_t *visited)
{
    sink out = {0, cap, t0, t1, vox};
    if (!(tmin <= tmax)) return 0;
    ray_ctx x;
    if (!ray_init(&x, g, o, d)) return 0;
    switch (method) {
    case 0: brute_force(&x, s, tmin, tmax, &out); break;
    case 1: march(&x, NULL, 0, 0, s, tmin, tmax, &out, visited); break;
    case 2: march(&x, NULL, 0, 1, s, tmin, tmax, &out, visited); break;
    case 3: march(&x, vdb, 0, 0, s, tmin, tmax, &out, visited); break;
    case 4: march(&x, vdb, 0, 1, s, tmin, tmax, &out, visited); break;
    case 5: march(&x, vdb, 1, 0, s, tmin, tmax, &out, visited); break;
    case 6: march(&x, vdb, 1, 1, s, tmin, tmax, &out, visited); break;
    default: out.count = -1;
    }
    ray_free(&x);
    return out.count;
}

int64_t orc_ray(const orc_grid *g, const orc_vdb *vdb, const orc_step *s, const float *o, const float *d,
                float tmin, float tmax, int32_t method, float *t0, float *t1, int32_t *vox, int64_t cap)
{
    int64_t visited = 0;
    return ray_run(g, vdb, s, o, d, tmin, tmax, method, t0, t1, vox, cap, &visited);
}

static int bad_method(const orc_vdb *vdb, int32_t method)
{
    return method < 0 || method > 6 || (method >= 3 && vdb == NULL);
}

/* counts[i] = number of samples of ray i.  Returns 0, or -1 on a bad method. */
int32_t orc_count(const orc_grid *g, const orc_vdb *vdb, const orc_step *s, const float *o, const float *d,
                  int64_t n, float tmin, float tmax, int32_t method, int64_t *counts, int32_t nthreads)
{
    if (bad_method(vdb, method)) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 256)
#endif
    for (int64_t i = 0; i < n; ++i)
        counts[i] = orc_ray(g, vdb, s, o + 3 * i, d + 3 * i, tmin, tmax, method, NULL, NULL, NULL, 0);
    return 0;
}

/* cells[i] = number of cells ray i's walk visits (occupied or not) before it
 * ends, for the DDA methods 1..6 (brute force visits no cells).  Returns 0,
 * or -1 on a bad method. */
int32_t orc_cells(const orc_grid *g, const orc_vdb *vdb, const orc_step *s, const float *o, const float *d,
                  int64_t n, float tmin, float tmax, int32_t method, int64_t *cells, int32_t nthreads)
{
    if (bad_method(vdb, method) || method == 0) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 256)
#endif
    for (int64_t i = 0; i < n; ++i) {
        int64_t visited = 0;
        ray_run(g, vdb, s, o + 3 * i, d + 3 * i, tmin, tmax, method, NULL, NULL, NULL, 0, &visited);
        cells[i] = visited;
    }
    return 0;
}

/* Writes ray i's samples at offsets[i] .. offsets[i+1]-1 (offsets from the
 * counts of the same method).  Returns the number of rays whose count did
 * not match their offsets span. */
int64_t orc_fill(const orc_grid *g, const orc_vdb *vdb, const orc_step *s, const float *o, const float *d,
                 int64_t n, float tmin, float tmax, int32_t method, const int64_t *offsets, int32_t *ray_ids,
                 float *t0, float *t1, int32_t *vox, int32_t nthreads)
{
    int64_t bad = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : bad)
#endif
    for (int64_t i = 0; i < n; ++i) {
        int64_t b = offsets[i], cap = offsets[i + 1] - offsets[i];
        int64_t c = orc_ray(g, vdb, s, o + 3 * i, d + 3 * i, tmin, tmax, method, t0 ? t0 + b : NULL,
                            t1 ? t1 + b : NULL, vox ? vox + b : NULL, cap);
        if (c != cap) bad += 1;
        if (ray_ids)
            for (int64_t k = 0; k < cap; ++k) ray_ids[b + k] = (int32_t)i;
    }
    return bad;
}

/* ------------------------------------------------------------------ */
/* VDB build: for every 8^3 block decide all-empty / all-occupied / mixed;
 * all-uniform blocks become tiles (Sec. 3: uniform regions are pruned and
 * kept as tiles), mixed blocks become leaves; one level up the same rule
 * turns an internal node whose slots are all empty (all full) tiles into a
 * root tile.  Voxels outside the grid (when R is not a multiple of the
 * internal node size) count as empty. */

orc_vdb *orc_vdb_build(const orc_grid *g, int32_t ilog2)
{
    if (g->R <= 0 || ilog2 < 1 || ilog2 > 5 || g->L < 1 || g->L > ORC_MAX_LEVELS) return NULL;
    orc_vdb *v = (orc_vdb *)calloc(1, sizeof(orc_vdb));
    int R = g->R;
    v->L = g->L;
    v->R = R;
    v->ilog2 = ilog2;
    v->S = 1 << ilog2;
    v->D = 8 * v->S;
    v->NR = (R + v->D - 1) / v->D;
    size_t nroot = (size_t)g->L * v->NR * v->NR * v->NR;
    size_t nslot = (size_t)v->S * v->S * v->S;
    v->root_kind = (int8_t *)calloc(nroot, 1);
    v->root_node = (int32_t *)calloc(nroot, sizeof(int32_t));
    v->slot_kind = (int8_t *)calloc(nroot * nslot, 1);
    v->slot_leaf = (int32_t *)calloc(nroot * nslot, sizeof(int32_t));
    v->leaf_vox = (uint8_t *)calloc(nroot * nslot * 512, 1);
    for (int lev = 0; lev < g->L; ++lev)
        for (int rx = 0; rx < v->NR; ++rx)
            for (int ry = 0; ry < v->NR; ++ry)
                for (int rz = 0; rz < v->NR; ++rz) {
                    size_t ri = (size_t)lev * v->NR * v->NR * v->NR + ((size_t)rx * v->NR + ry) * v->NR + rz;
                    int node = v->n_nodes;
                    int n_empty = 0, n_full = 0;
                    int8_t kinds[32 * 32 * 32];
                    uint8_t blk[512];
                    for (int sx = 0; sx < v->S; ++sx)
                        for (int sy = 0; sy < v->S; ++sy)
                            for (int sz = 0; sz < v->S; ++sz) {
                                int ones = 0;
                                for (int i = 0; i < 8; ++i)
                                    for (int j = 0; j < 8; ++j)
                                        for (int k = 0; k < 8; ++k) {
                                            int x = rx * v->D + sx * 8 + i;
                                            int y = ry * v->D + sy * 8 + j;
                                            int z = rz * v->D + sz * 8 + k;
                                            int on = 0;
                                            if (x < R && y < R && z < R)
                                                on = g->occ[(((size_t)lev * R + x) * R + y) * R + z] != 0;
                                            blk[(i * 8 + j) * 8 + k] = (uint8_t)on;
                                            ones += on;
                                        }
                                int s = (sx * v->S + sy) * v->S + sz;
                                size_t si = (size_t)node * nslot + s;
                                if (ones == 0) {
                                    kinds[s] = 0;
                                    n_empty++;
                                } else if (ones == 512) {
                                    kinds[s] = 1;
                                    n_full++;
                                } else {
                                    kinds[s] = 2;
                                    v->slot_leaf[si] = v->n_leaves;
                                    memcpy(v->leaf_vox + (size_t)v->n_leaves * 512, blk, 512);
                                    v->n_leaves++;
                                }
                                v->slot_kind[si] = kinds[s];
                            }
                    if (n_empty == (int)nslot || n_full == (int)nslot) {
                        v->root_kind[ri] = n_full == (int)nslot ? 1 : 0;
                        if (v->root_kind[ri]) v->n_root_full++;
                        else v->n_root_empty++;
                    } else {
                        v->root_kind[ri] = 2;
                        v->root_node[ri] = node;
                        v->n_nodes++;
                        v->n_slot_empty += n_empty;
                        v->n_slot_full += n_full;
                    }
                }
    return v;
}

/* stats: n_nodes, n_leaves, slot full tiles, slot empty tiles, root full tiles, root empty tiles */
void orc_vdb_stats(const orc_vdb *v, int64_t *out)
{
    out[0] = v->n_nodes;
    out[1] = v->n_leaves;
    out[2] = v->n_slot_full;
    out[3] = v->n_slot_empty;
    out[4] = v->n_root_full;
    out[5] = v->n_root_empty;
}

void orc_vdb_free(orc_vdb *v)
{
    if (!v) return;
    free(v->root_kind);
    free(v->root_node);
    free(v->slot_kind);
    free(v->slot_leaf);
    free(v->leaf_vox);
    free(v);
}

/* The binary32 values the definition is built from, for pinning tests:
 * out[0..R] = P_a(m), out[R+1..2R+1] = T_a(m). */
void orc_planes(const float *box, int32_t R, int32_t a, float o, float d, float *out)
{
    float r = 1.0f / d;
    for (int m = 0; m <= R; ++m) {
        out[m] = plane_pos(box, R, a, m);
        float diff = out[m] - o;
        out[R + 1 + m] = diff * r;
    }
}

/* The lattice t_0..t_{n-1}. */
void orc_lattice(const orc_step *s, float tmin, int64_t n, float *out)
{
    lattice q;
    lat_init(&q, s, tmin);
    for (int64_t i = 0; i < n; ++i, lat_advance(&q)) out[i] = q.t;
}
