/*
 * sdf.c -- plain FP64 reference of ray / point-cloud intersection through the
 * implicit surface of Eq. 1 (paper, Section 2.2.1 "Intersections").
 *
 * TEST INFRASTRUCTURE.  Only tests/, __graft_entry__.smoke() and bench.py's
 * cpu_baseline leg may call this code.  It shares no code with the HIP path.
 *
 * Definition (with the readings where the paper is silent marked R):
 *   - f(x) = (x - p(x)) . n(x), p and n the weighted averages of the positions
 *     and normals of the points near x (Eq. 1).  R: weights
 *     w = (1 - |x - q|^2 / h^2)^4 for |x - q| < h, 0 beyond; n(x) is the
 *     normalised weighted sum of the (oriented, normalised) point normals;
 *     f is undefined where no point lies within h or the normals cancel.
 *   - The point set of a subvoxel is the points whose centre lies in that
 *     finest cell ("leaf").  R: a point's leaf is floor((q - origin) / leaf)
 *     taken in FP32 arithmetic, exactly as the GPU assigns it, so that both
 *     sides agree on this integer decision.
 *   - For every occupied leaf the ray passes through, the centre c of the
 *     axis-aligned box around the leaf's points is projected onto the ray,
 *     t_c = (c - o) . d; the line segment is [t_c - D/2, t_c + D/2] with D the
 *     leaf's diagonal, clipped to the query's range [t_lo, t_hi].
 *   - From the segment's near end the march evaluates f at s_i and moves on
 *     by |f(s_i)|.  An intersection is found at s_i when |f(s_i)| <= eps, or
 *     between s_{i-1} and s_i when the two values differ in sign (R: at the
 *     zero of the linear interpolation).  R: where f is undefined the march
 *     moves on by h / 2 and no sign is compared across such a sample; a leaf
 *     is given up after max_steps evaluations or when s_i passes the
 *     segment's far end.
 *   - R: the ray's intersection is the one of smallest t over all the leaves
 *     the ray crosses within [0, t_hi]; the normal is n at the final sample.
 * Brute force: every leaf is tested against the ray by a slab test; the
 * neighbours of x are found through a sorted list of cells of edge >= h
 * (every point within h of x lies in the 27 cells around x's).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    const float* xyz;          /* [n_pts*3] */
    const float* nrm;          /* [n_pts*3] any non-zero length */
    int64_t n_pts;
    float origin[3];           /* the scene's FP32 grid origin */
    float leaf;                /* the scene's FP32 finest edge */
    const float* o;            /* [n_rays*3] ray origins */
    const float* d;            /* [n_rays*3] ray directions (renormalised in FP64) */
    const float* trange;       /* [n_rays*2] (t_lo, t_hi), or NULL for (0, inf) */
    int64_t n_rays;
    double h;                  /* neighbourhood radius */
    double eps;                /* |f| at or below this is an intersection */
    int32_t max_steps;         /* evaluations per leaf segment */
    int32_t n_threads;
    double diam_scale;         /* segment length / leaf diagonal (1 for the definition) */
    double cross_margin;       /* a leaf counts as crossed when its overlap with the ray is >= -margin */
    double* t;                 /* [n_rays] intersection distance, +inf none */
    double* point;             /* [n_rays*3] */
    double* normal;            /* [n_rays*3] n at the intersection */
    int32_t* leaf_cell;        /* [n_rays*3] cell of the leaf whose march found it, -1 none */
    const double* o64;         /* optional FP64 origins, directions and ranges (used instead of o, d, */
    const double* d64;         /* trange when given): the state of rays that have already reflected */
    const double* trange64;
} OracleSdfArgs;

typedef struct {
    int64_t key;
    int64_t idx;
} KeyIdx;

static int cmp_keyidx(const void* a, const void* b)
{
    const KeyIdx* x = a;
    const KeyIdx* y = b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

typedef struct {
    const OracleSdfArgs* a;
    /* FP64 points */
    double *px, *py, *pz, *nx, *ny, *nz;
    /* neighbour cells: points sorted by cell key */
    double cell, clo[3];
    int64_t cdim[3];
    KeyIdx* cells;
    /* occupied leaves */
    int64_t n_leaves;
    int64_t* leaf_lin;         /* linear leaf index */
    int32_t* leaf_c;           /* [n_leaves*3] leaf cell */
    double* leaf_ctr;          /* [n_leaves*3] centre of the box around its points */
    int64_t lo, hi;            /* rays of a worker */
} Sdf;

/* first entry with key >= k */
static int64_t lower_bound(const KeyIdx* v, int64_t n, int64_t k)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t m = lo + (hi - lo) / 2;
        if (v[m].key < k) lo = m + 1;
        else hi = m;
    }
    return lo;
}

/* f(x) of Eq. 1.  Returns 1 with f and the unit normal n(x), 0 where f is
 * undefined.  p(x) - x is accumulated relative to x (the same quantity). */
static int sdf_eval(const Sdf* S, const double* x, double* f, double* n)
{
    const double h = S->a->h, h2 = h * h;
    int64_t cc[3];
    for (int a = 0; a < 3; ++a) cc[a] = (int64_t)floor((x[a] - S->clo[a]) / S->cell);
    double sw = 0.0, sp[3] = {0.0, 0.0, 0.0}, sn[3] = {0.0, 0.0, 0.0};
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int64_t c[3] = {cc[0] + dx, cc[1] + dy, cc[2] + dz};
                if (c[0] < 0 || c[1] < 0 || c[2] < 0 || c[0] >= S->cdim[0] || c[1] >= S->cdim[1] ||
                    c[2] >= S->cdim[2])
                    continue;
                int64_t k = c[0] + S->cdim[0] * (c[1] + S->cdim[1] * c[2]);
                for (int64_t e = lower_bound(S->cells, S->a->n_pts, k); e < S->a->n_pts && S->cells[e].key == k;
                     ++e) {
                    int64_t q = S->cells[e].idx;
                    double ex = S->px[q] - x[0], ey = S->py[q] - x[1], ez = S->pz[q] - x[2];
                    double d2 = ex * ex + ey * ey + ez * ez;
                    if (!(d2 < h2)) continue;
                    double w = 1.0 - d2 / h2;
                    w = w * w;
                    w = w * w;
                    sw += w;
                    sp[0] += w * ex; sp[1] += w * ey; sp[2] += w * ez;
                    sn[0] += w * S->nx[q]; sn[1] += w * S->ny[q]; sn[2] += w * S->nz[q];
                }
            }
    double ln = sqrt(sn[0] * sn[0] + sn[1] * sn[1] + sn[2] * sn[2]);
    if (!(sw > 0.0) || !(ln > 0.0)) return 0;
    for (int a = 0; a < 3; ++a) n[a] = sn[a] / ln;
    /* (x - p) . n with p - x = sp / sw */
    *f = -(sp[0] * n[0] + sp[1] * n[1] + sp[2] * n[2]) / sw;
    return 1;
}

/* Interval of t over which the ray o + t d lies in the box [lo, hi]; returns
 * 0 when the ray never does.  Zero direction components test the slab. */
static int slab(const double* o, const double* d, const double* lo, const double* hi, double m, double* t0,
                double* t1)
{
    double a0 = -INFINITY, a1 = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] != 0.0) {
            double ta = (lo[a] - o[a]) / d[a], tb = (hi[a] - o[a]) / d[a];
            if (ta > tb) { double s = ta; ta = tb; tb = s; }
            if (ta > a0) a0 = ta;
            if (tb < a1) a1 = tb;
        } else if (o[a] < lo[a] - m || o[a] > hi[a] + m) {
            return 0;
        }
    }
    *t0 = a0;
    *t1 = a1;
    return 1;
}

/* The march over one leaf's segment [ta, tb].  Returns 1 with the hit. */
static int march(const Sdf* S, const double* o, const double* d, double ta, double tb, double* th, double* nh)
{
    const OracleSdfArgs* a = S->a;
    double t = ta, fp = 0.0, tp = 0.0;
    int have_prev = 0;
    for (int i = 0; i < a->max_steps && t <= tb; ++i) {
        double x[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
        double f, n[3];
        if (!sdf_eval(S, x, &f, n)) {
            have_prev = 0;
            t += 0.5 * a->h;
            continue;
        }
        if (fabs(f) <= a->eps) {
            *th = t;
            memcpy(nh, n, sizeof n);
            return 1;
        }
        if (have_prev && ((f < 0.0) != (fp < 0.0))) {
            *th = tp + (t - tp) * fp / (fp - f);
            memcpy(nh, n, sizeof n);
            return 1;
        }
        have_prev = 1;
        fp = f;
        tp = t;
        t += fabs(f);
    }
    return 0;
}

static void sdf_ray(const Sdf* S, int64_t r)
{
    const OracleSdfArgs* a = S->a;
    double o[3], d[3];
    for (int k = 0; k < 3; ++k) {
        o[k] = a->o64 ? a->o64[3 * r + k] : (double)a->o[3 * r + k];
        d[k] = a->d64 ? a->d64[3 * r + k] : (double)a->d[3 * r + k];
    }
    double dl = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    d[0] /= dl; d[1] /= dl; d[2] /= dl;
    double t_lo = a->trange64 ? a->trange64[2 * r] : (a->trange ? a->trange[2 * r] : 0.0);
    double t_hi = a->trange64 ? a->trange64[2 * r + 1] : (a->trange ? a->trange[2 * r + 1] : INFINITY);
    const double L = a->leaf, D = a->diam_scale * sqrt(3.0) * L, m = a->cross_margin;
    double best = INFINITY, bn[3] = {0.0, 0.0, 0.0};
    int64_t bl = -1, bi = -1;
    for (int64_t l = 0; l < S->n_leaves; ++l) {
        double lo[3], hi[3], t0, t1;
        for (int k = 0; k < 3; ++k) {
            lo[k] = (double)a->origin[k] + (double)S->leaf_c[3 * l + k] * L;
            hi[k] = lo[k] + L;
        }
        if (!slab(o, d, lo, hi, m, &t0, &t1)) continue;
        /* crossed within [0, t_hi] */
        double u0 = t0 > 0.0 ? t0 : 0.0, u1 = t1 < t_hi ? t1 : t_hi;
        if (u0 - u1 > m) continue;
        const double* c = S->leaf_ctr + 3 * l;
        double tc = (c[0] - o[0]) * d[0] + (c[1] - o[1]) * d[1] + (c[2] - o[2]) * d[2];
        double ta = tc - 0.5 * D, tb = tc + 0.5 * D;
        if (ta < t_lo) ta = t_lo;
        if (tb > t_hi) tb = t_hi;
        if (!(ta <= tb)) continue;
        double th, nh[3];
        if (march(S, o, d, ta, tb, &th, nh) && (th < best || (th == best && S->leaf_lin[l] < bl))) {
            best = th;
            memcpy(bn, nh, sizeof nh);
            bl = S->leaf_lin[l];
            bi = l;
        }
    }
    a->t[r] = best;
    for (int k = 0; k < 3; ++k) {
        a->point[3 * r + k] = bl >= 0 ? o[k] + best * d[k] : NAN;
        a->normal[3 * r + k] = bn[k];
    }
    for (int k = 0; k < 3; ++k) a->leaf_cell[3 * r + k] = bl >= 0 ? S->leaf_c[3 * bi + k] : -1;
}

static void* sdf_worker(void* p)
{
    const Sdf* S = p;
    for (int64_t r = S->lo; r < S->hi; ++r) sdf_ray(S, r);
    return NULL;
}

int oracle_sdf_intersect(OracleSdfArgs* a)
{
    if (!a || a->n_pts < 0 || a->n_rays < 0 || !(a->h > 0.0) || !(a->eps >= 0.0) || a->max_steps < 0 ||
        !(a->leaf > 0.0f) || !(a->diam_scale > 0.0) || (a->n_rays > 0 && ((!a->o && !a->o64) || (!a->d && !a->d64) || !a->t || !a->point || !a->normal ||
                            !a->leaf_cell)) ||
        (a->n_pts > 0 && (!a->xyz || !a->nrm)))
        return -1;
    Sdf S;
    memset(&S, 0, sizeof S);
    S.a = a;
    int64_t n = a->n_pts;
    size_t nb = (size_t)(n > 0 ? n : 1) * sizeof(double);
    S.px = malloc(nb); S.py = malloc(nb); S.pz = malloc(nb);
    S.nx = malloc(nb); S.ny = malloc(nb); S.nz = malloc(nb);
    S.cells = malloc((size_t)(n > 0 ? n : 1) * sizeof(KeyIdx));
    KeyIdx* lk = malloc((size_t)(n > 0 ? n : 1) * sizeof(KeyIdx));
    S.leaf_lin = malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    S.leaf_c = malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(int32_t));
    S.leaf_ctr = malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(double));
    int status = (!S.px || !S.py || !S.pz || !S.nx || !S.ny || !S.nz || !S.cells || !lk || !S.leaf_lin ||
                  !S.leaf_c || !S.leaf_ctr) ? -2 : 0;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t q = 0; q < n && !status; ++q) {
        S.px[q] = a->xyz[3 * q]; S.py[q] = a->xyz[3 * q + 1]; S.pz[q] = a->xyz[3 * q + 2];
        double nx = a->nrm[3 * q], ny = a->nrm[3 * q + 1], nz = a->nrm[3 * q + 2];
        double len = sqrt(nx * nx + ny * ny + nz * nz);
        if (!(len > 0.0) || !isfinite(len)) { status = -1; break; }
        S.nx[q] = nx / len; S.ny[q] = ny / len; S.nz[q] = nz / len;
        double p[3] = {S.px[q], S.py[q], S.pz[q]};
        for (int k = 0; k < 3; ++k) {
            if (p[k] < lo[k]) lo[k] = p[k];
            if (p[k] > hi[k]) hi[k] = p[k];
        }
    }
    /* neighbour cells of edge h: every point within h of x lies in the 27 cells around x's */
    S.cell = a->h;
    for (int k = 0; k < 3 && !status; ++k) {
        S.clo[k] = n > 0 ? lo[k] - a->h : 0.0;
        S.cdim[k] = n > 0 ? (int64_t)floor((hi[k] + a->h - S.clo[k]) / S.cell) + 2 : 1;
    }
    if (!status && (double)S.cdim[0] * (double)S.cdim[1] * (double)S.cdim[2] > 9e18) status = -1;
    for (int64_t q = 0; q < n && !status; ++q) {
        double p[3] = {S.px[q], S.py[q], S.pz[q]};
        int64_t c[3];
        for (int k = 0; k < 3; ++k) c[k] = (int64_t)floor((p[k] - S.clo[k]) / S.cell);
        S.cells[q].key = c[0] + S.cdim[0] * (c[1] + S.cdim[1] * c[2]);
        S.cells[q].idx = q;
    }
    if (!status) qsort(S.cells, (size_t)n, sizeof(KeyIdx), cmp_keyidx);
    /* leaves: the point's cell taken in FP32, as the kernels do */
    int32_t* pc = malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(int32_t));
    if (!pc) status = -2;
    int64_t gd[3] = {1, 1, 1};
    if (!status) {
        const float inv = 1.0f / a->leaf;
        for (int64_t q = 0; q < n; ++q)
            for (int k = 0; k < 3; ++k) {
                float u = a->xyz[3 * q + k] - a->origin[k];
                float v = u * inv;
                pc[3 * q + k] = (int32_t)floorf(v);
            }
        int32_t mn[3] = {0, 0, 0}, mx[3] = {0, 0, 0};
        for (int64_t q = 0; q < n; ++q)
            for (int k = 0; k < 3; ++k) {
                if (q == 0 || pc[3 * q + k] < mn[k]) mn[k] = pc[3 * q + k];
                if (q == 0 || pc[3 * q + k] > mx[k]) mx[k] = pc[3 * q + k];
            }
        if (n > 0 && (mn[0] < 0 || mn[1] < 0 || mn[2] < 0)) status = -1;
        for (int k = 0; k < 3; ++k) gd[k] = (int64_t)mx[k] + 1;
        for (int64_t q = 0; q < n && !status; ++q) {
            lk[q].key = pc[3 * q] + gd[0] * (pc[3 * q + 1] + gd[1] * (int64_t)pc[3 * q + 2]);
            lk[q].idx = q;
        }
        if (!status) qsort(lk, (size_t)n, sizeof(KeyIdx), cmp_keyidx);
        for (int64_t e = 0; e < n && !status;) {
            int64_t f = e;
            double blo[3] = {INFINITY, INFINITY, INFINITY}, bhi[3] = {-INFINITY, -INFINITY, -INFINITY};
            while (f < n && lk[f].key == lk[e].key) {
                int64_t q = lk[f].idx;
                double p[3] = {S.px[q], S.py[q], S.pz[q]};
                for (int k = 0; k < 3; ++k) {
                    if (p[k] < blo[k]) blo[k] = p[k];
                    if (p[k] > bhi[k]) bhi[k] = p[k];
                }
                ++f;
            }
            int64_t l = S.n_leaves++;
            int64_t q = lk[e].idx;
            S.leaf_lin[l] = lk[e].key;
            for (int k = 0; k < 3; ++k) {
                S.leaf_c[3 * l + k] = pc[3 * q + k];
                S.leaf_ctr[3 * l + k] = 0.5 * (blo[k] + bhi[k]);
            }
            e = f;
        }
    }
    free(pc);
    free(lk);
    if (!status) {
        int nt = a->n_threads > 0 ? a->n_threads : 1;
        if (nt > a->n_rays) nt = (int)(a->n_rays > 0 ? a->n_rays : 1);
        Sdf* W = calloc((size_t)nt, sizeof(Sdf));
        pthread_t* T = calloc((size_t)nt, sizeof(pthread_t));
        if (!W || !T) status = -2;
        if (!status) {
            for (int k = 0; k < nt; ++k) {
                W[k] = S;
                W[k].lo = a->n_rays * k / nt;
                W[k].hi = a->n_rays * (k + 1) / nt;
            }
            for (int k = 1; k < nt; ++k) pthread_create(&T[k], NULL, sdf_worker, &W[k]);
            sdf_worker(&W[0]);
            for (int k = 1; k < nt; ++k) pthread_join(T[k], NULL);
        }
        free(W);
        free(T);
    }
    free(S.px); free(S.py); free(S.pz); free(S.nx); free(S.ny); free(S.nz);
    free(S.cells); free(S.leaf_lin); free(S.leaf_c); free(S.leaf_ctr);
    return status;
}
