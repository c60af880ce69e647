/*
 * oracle.c -- plain FP64 brute-force reference for coarse-path ray launching.
 *
 * TEST INFRASTRUCTURE.  Only tests/, __graft_entry__.smoke() and bench.py's
 * cpu_baseline leg may call this library.  It shares no code with the HIP
 * path and is never used by it.
 *
 * What it computes (paper, Section 2.2 "Coarse Path Tracing", read with the
 * uniform ray launching of the Introduction): from each TX, rays leave in the
 * directions given by the caller (renormalised in FP64); every ray is tested against EVERY point of
 * the cloud (no acceleration structure), reflects specularly at the nearest
 * hit up to K times (Section 2.2.3, propagation phase: rays are traced until
 * they hit nothing or reach the interaction limit), and is tested against
 * every RX sphere on every segment.  Receptions are emitted as records; the
 * label sequence of each record is the coarse path of Section 2.2.3 (labels
 * in interaction order), deduplicated in oracle/__init__.py.
 *
 * Readings where the paper is silent (Section 2.2.1 uses an SDF over nearby
 * points; the launching here uses point-wise surfels instead):
 *   - each point is a two-sided disk: centre p, unit normal n (the input
 *     normal normalised in FP64), radius r_s;
 *   - a ray o + t d hits point m iff |d.n| > 1e-12, t = ((p-o).n)/(d.n) > t_eps,
 *     m is not the point the ray just left, and |o + t d - p| <= r_s;
 *   - the nearest hit wins; equal t is broken by the smaller point index;
 *   - reflection uses the hit point's own normal: d' = d - 2 (d.n) n,
 *     renormalised;
 *   - a segment [0, t_end] (t_end = hit distance or +inf) is received by RX r
 *     iff s = (rx - o).d lies in (0, t_end] and the closest approach
 *     |o + s d - rx| <= rho(L + s), rho(u) = sigma * u * alpha / sqrt(3),
 *     alpha = sqrt(8 pi / (sqrt(3) N)) the ideal angular spacing of N rays;
 *     L is the polyline length already travelled.  RX spheres are
 *     transparent.
 *
 * Besides the exact answer, the parity mode lists for every segment the set
 * of answers that an FP32 implementation may legitimately give (near ties and
 * surfels whose thresholds lie inside an error band), and flags receptions
 * whose thresholds lie inside a band.  The bands are inputs.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAXACC 64
#define ORACLE_DEN_SKIP 1e-12
#define ORACLE_MAXN 8           /* most reflections of a refined path */

typedef struct {
    /* scene */
    const float* xyz;          /* [n_pts*3] */
    const float* nrm;          /* [n_pts*3] */
    const uint32_t* label;     /* [n_pts]   */
    int64_t n_pts;
    /* antennas and rays */
    const float* tx;           /* [n_tx*3] */
    int32_t n_tx;
    const float* rx;           /* [n_rx*3] */
    int32_t n_rx;
    const float* dirs;         /* [n_rays*3], shared by every TX */
    int64_t n_rays;            /* rays per TX */
    const int64_t* sel;        /* global ray ids g = tx*n_rays + j to trace; NULL: all */
    int64_t n_sel;
    /* method parameters */
    int32_t K;                 /* maximum number of reflections */
    double r_s;                /* surfel radius */
    double t_eps;              /* self-intersection distance */
    double sigma;              /* reception sphere scale */
    double alpha;              /* angular ray spacing; <= 0: ideal spacing of n_rays */
    /* parity bands (parity != 0) */
    int32_t parity;
    double tie_rel;            /* relative window on hit distance (1e-4) */
    double err_abs;            /* absolute position error per segment of the compared implementation */
    double err_dir;            /* direction error per segment of the compared implementation */
    double edge_rel;           /* relative band on r_s, t_eps and rho */
    double den_amb;            /* |d.n| at or below this is ambiguous */
    int32_t n_threads;
    /* per traced ray and segment b = 0..K: index r*(K+1) + b */
    int64_t* hit_id;           /* -1: no hit */
    double* hit_t;             /* +inf: no hit */
    int32_t* acc_n;            /* size of the acceptable set (parity) */
    int64_t* acc_id;           /* [.. * ORACLE_MAXACC], -1 stands for "no hit" */
    double* acc_tc;            /* nearest clear hit of the segment (+inf: none), for oracle_accepts */
    double* seg_o;             /* optional [.. * 3] segment origin */
    double* seg_d;             /* optional [.. * 3] segment direction */
    /* per traced ray and reflection k = 0..K-1: index r*K + k */
    int64_t* seq;              /* label of the k-th interaction, -1 */
    double* pts;               /* [.. * 3] k-th interaction point */
    /* reception records, in traced-ray order */
    int64_t rec_cap;
    int64_t n_rec;             /* out: number of records (may exceed rec_cap) */
    int64_t* rec_sel;          /* index into the traced rays */
    int64_t* rec_g;            /* global ray id */
    int32_t* rec_tx;
    int32_t* rec_rx;
    int32_t* rec_b;            /* number of reflections before reception */
    double* rec_lpoly;         /* L + |rx - o| */
    double* rec_lunf;          /* L + s */
    int32_t* rec_flags;        /* bit0 received, bit1 ambiguous */
    const struct OracleGrid* grid;  /* NULL: brute force; else the uniform-grid DDA (parity mode off) */
} OracleArgs;

/* A uniform grid of cubic cells over the points, each cell listing every
 * point whose disk's bounding sphere meets it (the cell box padded by a
 * rounding margin): a superset of the points a ray can hit inside the cell. */
typedef struct OracleGrid {
    double lo[3];
    double cell;
    int64_t dims[3];
    int64_t* begin;            /* [cells + 1] CSR offsets */
    int64_t* items;            /* point ids */
} OracleGrid;

/* ------------------------------------------------------------------------ */
/* ray directions                                                            */
/* ------------------------------------------------------------------------ */

/* Uniformly spaced directions on the unit sphere (Fibonacci lattice):
 * z_j = 1 - (2j+1)/N, phi_j = 2 pi frac(j (3 - sqrt 5)/2), computed in FP64
 * and rounded to FP32.  The fractional part is taken before the multiply by
 * 2 pi so that large j keeps its angular resolution. */
int oracle_fibonacci(int64_t n, float* out)
{
    if (n <= 0 || !out) return -1;
    const double g = (3.0 - sqrt(5.0)) / 2.0;
    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t j = 0; j < n; ++j) {
        double z = 1.0 - (double)(2 * j + 1) / (double)n;
        double r = sqrt(fmax(0.0, 1.0 - z * z));
        double jg = (double)j * g;
        double f = jg - floor(jg);
        double phi = two_pi * f;
        out[3 * j + 0] = (float)(r * cos(phi));
        out[3 * j + 1] = (float)(r * sin(phi));
        out[3 * j + 2] = (float)z;
    }
    return 0;
}

/* Ideal angular spacing of N directions on the sphere: hexagonal cells of
 * area (sqrt 3 / 2) a^2 tile the 4 pi steradians. */
double oracle_ray_spacing(int64_t n)
{
    return sqrt(8.0 * M_PI / (sqrt(3.0) * (double)n));
}

/* ------------------------------------------------------------------------ */
/* brute force                                                               */
/* ------------------------------------------------------------------------ */

typedef struct {
    double *px, *py, *pz, *nx, *ny, *nz;
} Pts64;

typedef struct {
    int64_t n, cap;
    int64_t *sel, *g;
    int32_t *tx, *rx, *b, *flags;
    double *lp, *lu;
} RecBuf;

static int rec_push(RecBuf* r, int64_t sel, int64_t g, int32_t tx, int32_t rx, int32_t b,
                    double lp, double lu, int32_t flags)
{
    if (r->n == r->cap) {
        int64_t c = r->cap ? 2 * r->cap : 256;
#define GROW(f, T) do { void* q = realloc(r->f, (size_t)c * sizeof(T)); if (!q) return -1; r->f = (T*)q; } while (0)
        GROW(sel, int64_t); GROW(g, int64_t); GROW(tx, int32_t); GROW(rx, int32_t);
        GROW(b, int32_t); GROW(flags, int32_t); GROW(lp, double); GROW(lu, double);
#undef GROW
        r->cap = c;
    }
    int64_t i = r->n++;
    r->sel[i] = sel; r->g[i] = g; r->tx[i] = tx; r->rx[i] = rx; r->b[i] = b;
    r->lp[i] = lp; r->lu[i] = lu; r->flags[i] = flags;
    return 0;
}

static void rec_free(RecBuf* r)
{
    free(r->sel); free(r->g); free(r->tx); free(r->rx); free(r->b); free(r->flags);
    free(r->lp); free(r->lu);
}

typedef struct {
    const OracleArgs* a;
    const Pts64* P;
    double alpha;
    int64_t lo, hi;            /* traced-ray range */
    RecBuf rec;
    int status;
} Work;

static inline double dot3(const double* u, const double* v) { return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]; }

/* Parity bands of one surfel for the segment o + t d (segment index b,
 * bb = b + 1).  A surfel is ambiguous when one of its thresholds (disk edge,
 * t_eps, grazing incidence) lies within the error band of the compared
 * implementation; it is a candidate when it is a hit by the definition.
 * Returns 0 when the surfel is clearly not a hit under any band (then the
 * outputs are unset). */
static int surfel_class(const OracleArgs* a, const double* p, const double* n, const double* o,
                        const double* d, double bb, double* t_out, double* band_out, int* cand, int* amb)
{
    double den = d[0] * n[0] + d[1] * n[1] + d[2] * n[2];
    if (fabs(den) <= ORACLE_DEN_SKIP) return 0;
    double wx = p[0] - o[0], wy = p[1] - o[1], wz = p[2] - o[2];
    double t = (wx * n[0] + wy * n[1] + wz * n[2]) / den;
    double qx = o[0] + t * d[0] - p[0];
    double qy = o[1] + t * d[1] - p[1];
    double qz = o[2] + t * d[2] - p[2];
    double dist = sqrt(qx * qx + qy * qy + qz * qz);
    /* position error of the compared ray at this distance, projected into
     * the disk plane (grows as 1/|den| at grazing incidence) */
    double band = bb * (a->err_abs + fabs(t) * a->err_dir) * (1.0 + 1.0 / fabs(den));
    double band_r = band + a->edge_rel * a->r_s;
    double band_t = band + a->edge_rel * a->t_eps;
    if (dist > a->r_s + band_r) return 0;          /* clearly outside the disk */
    if (t <= a->t_eps - band_t) return 0;          /* clearly behind / too close */
    *cand = (t > a->t_eps) && (dist <= a->r_s);
    *amb = (fabs(den) <= a->den_amb) || (fabs(dist - a->r_s) <= band_r) || (fabs(t - a->t_eps) <= band_t);
    *t_out = t;
    *band_out = band;
    return 1;
}

/* One segment: the exact nearest hit (definition), and in parity mode the
 * set of answers compatible with the error bands. */
static void nearest_hit(const OracleArgs* a, const Pts64* P, const double* o, const double* d,
                        int64_t last, int32_t b, int64_t* best_out, double* tb_out,
                        int32_t* acc_n, int64_t* acc_id, double* acc_tc, double* acc_tlo, double* acc_thi)
{
    const double rs2 = a->r_s * a->r_s;
    int64_t best = -1;
    double tb = INFINITY;
    for (int64_t m = 0; m < a->n_pts; ++m) {
        if (m == last) continue;
        double den = d[0] * P->nx[m] + d[1] * P->ny[m] + d[2] * P->nz[m];
        if (fabs(den) <= ORACLE_DEN_SKIP) continue;
        double wx = P->px[m] - o[0], wy = P->py[m] - o[1], wz = P->pz[m] - o[2];
        double t = (wx * P->nx[m] + wy * P->ny[m] + wz * P->nz[m]) / den;
        if (!(t > a->t_eps)) continue;
        double qx = o[0] + t * d[0] - P->px[m];
        double qy = o[1] + t * d[1] - P->py[m];
        double qz = o[2] + t * d[2] - P->pz[m];
        double dist2 = qx * qx + qy * qy + qz * qz;
        if (dist2 <= rs2 && (t < tb || (t == tb && m < best))) {
            tb = t;
            best = m;
        }
    }
    *best_out = best;
    *tb_out = tb;
    if (!a->parity) return;

    /* Parity mode: the acceptable set, its extent in t and the nearest clear
     * hit.  Only the first ORACLE_MAXACC members are stored; membership of any
     * other point is decided by oracle_accepts with the same tc. */
    const double bb = (double)(b + 1);
    double tc = INFINITY;
    for (int64_t m = 0; m < a->n_pts; ++m) {
        if (m == last) continue;
        const double pm[3] = {P->px[m], P->py[m], P->pz[m]}, nm[3] = {P->nx[m], P->ny[m], P->nz[m]};
        double t, band;
        int cand, amb;
        if (!surfel_class(a, pm, nm, o, d, bb, &t, &band, &cand, &amb)) continue;
        if (cand && !amb && t < tc) tc = t;
    }
    int32_t na = 0;
    double t_lo = INFINITY, t_hi = -INFINITY;
    /* "no hit" is acceptable when no clear hit exists; it is stored first,
     * so a set larger than the array never drops it */
    if (tc == INFINITY) { acc_id[na++] = -1; t_hi = INFINITY; }
    for (int64_t m = 0; m < a->n_pts; ++m) {
        if (m == last) continue;
        const double pm[3] = {P->px[m], P->py[m], P->pz[m]}, nm[3] = {P->nx[m], P->ny[m], P->nz[m]};
        double t, band;
        int cand, amb;
        if (!surfel_class(a, pm, nm, o, d, bb, &t, &band, &cand, &amb)) continue;
        if (t <= tc * (1.0 + a->tie_rel) + band && (cand || amb)) {
            if (na < ORACLE_MAXACC) acc_id[na] = m;
            ++na;
            if (t < t_lo) t_lo = t;
            if (t > t_hi) t_hi = t;
        }
    }
    *acc_n = na;
    *acc_tc = tc;
    *acc_tlo = t_lo;
    *acc_thi = t_hi;
}

/* The hit test of point m (same formula as the brute force). */
static inline int surfel_hit(const OracleArgs* a, const Pts64* P, const double* o, const double* d, int64_t m,
                             double* t_out)
{
    double den = d[0] * P->nx[m] + d[1] * P->ny[m] + d[2] * P->nz[m];
    if (fabs(den) <= ORACLE_DEN_SKIP) return 0;
    double wx = P->px[m] - o[0], wy = P->py[m] - o[1], wz = P->pz[m] - o[2];
    double t = (wx * P->nx[m] + wy * P->ny[m] + wz * P->nz[m]) / den;
    if (!(t > a->t_eps)) return 0;
    double qx = o[0] + t * d[0] - P->px[m];
    double qy = o[1] + t * d[1] - P->py[m];
    double qz = o[2] + t * d[2] - P->pz[m];
    if (!(qx * qx + qy * qy + qz * qz <= a->r_s * a->r_s)) return 0;
    *t_out = t;
    return 1;
}

/* Nearest hit by a 3D DDA over the grid (Amanatides and Woo): cells in ray
 * order, every listed point tested, stop once the best hit lies before the
 * current cell's exit.  Same (t, index) minimum as the brute force because
 * every point a ray meets inside a cell is listed in that cell. */
static void nearest_hit_grid(const OracleArgs* a, const Pts64* P, const OracleGrid* G, const double* o,
                             const double* d, int64_t last, int64_t* best_out, double* tb_out)
{
    int64_t best = -1;
    double tb = INFINITY;
    double t0 = 0.0, t1 = INFINITY;
    for (int ax = 0; ax < 3; ++ax) {
        double lo = G->lo[ax], hi = G->lo[ax] + (double)G->dims[ax] * G->cell;
        if (d[ax] != 0.0) {
            double ta = (lo - o[ax]) / d[ax], tc = (hi - o[ax]) / d[ax];
            t0 = fmax(t0, fmin(ta, tc));
            t1 = fmin(t1, fmax(ta, tc));
        } else if (o[ax] < lo || o[ax] > hi) {
            t1 = -1.0;
        }
    }
    if (t0 <= t1) {
        int64_t c[3], step[3];
        double tmax[3], tdelta[3];
        for (int ax = 0; ax < 3; ++ax) {
            double x = o[ax] + t0 * d[ax];
            int64_t ci = (int64_t)floor((x - G->lo[ax]) / G->cell);
            if (ci < 0) ci = 0;
            if (ci >= G->dims[ax]) ci = G->dims[ax] - 1;
            c[ax] = ci;
            if (d[ax] > 0.0) {
                step[ax] = 1;
                tmax[ax] = (G->lo[ax] + (double)(ci + 1) * G->cell - o[ax]) / d[ax];
                tdelta[ax] = G->cell / d[ax];
            } else if (d[ax] < 0.0) {
                step[ax] = -1;
                tmax[ax] = (G->lo[ax] + (double)ci * G->cell - o[ax]) / d[ax];
                tdelta[ax] = -G->cell / d[ax];
            } else {
                step[ax] = 0;
                tmax[ax] = INFINITY;
                tdelta[ax] = INFINITY;
            }
        }
        for (;;) {
            int64_t cell = c[0] + G->dims[0] * (c[1] + G->dims[1] * c[2]);
            for (int64_t e = G->begin[cell]; e < G->begin[cell + 1]; ++e) {
                int64_t m = G->items[e];
                double t;
                if (m == last || !surfel_hit(a, P, o, d, m, &t)) continue;
                if (t < tb || (t == tb && m < best)) {
                    tb = t;
                    best = m;
                }
            }
            int ax = tmax[0] <= tmax[1] ? (tmax[0] <= tmax[2] ? 0 : 2) : (tmax[1] <= tmax[2] ? 1 : 2);
            if (best >= 0 && tb < tmax[ax]) break;
            c[ax] += step[ax];
            if (c[ax] < 0 || c[ax] >= G->dims[ax]) break;
            tmax[ax] += tdelta[ax];
        }
    }
    *best_out = best;
    *tb_out = tb;
}

/* Build the grid of cubic cells of edge `cell` over n points with disks of
 * radius r_s.  Returns NULL when out of memory or on bad arguments. */
OracleGrid* oracle_grid_build(const float* xyz, int64_t n, double r_s, double cell)
{
    if (n < 0 || (n > 0 && !xyz) || !(r_s > 0.0) || !(cell > 0.0)) return NULL;
    OracleGrid* G = calloc(1, sizeof(OracleGrid));
    if (!G) return NULL;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < n; ++i)
        for (int ax = 0; ax < 3; ++ax) {
            lo[ax] = fmin(lo[ax], (double)xyz[3 * i + ax]);
            hi[ax] = fmax(hi[ax], (double)xyz[3 * i + ax]);
        }
    if (n == 0)
        for (int ax = 0; ax < 3; ++ax) lo[ax] = hi[ax] = 0.0;
    double scale = 0.0;
    for (int ax = 0; ax < 3; ++ax) scale = fmax(scale, fmax(fabs(lo[ax]), fabs(hi[ax])));
    const double pad = 1e-9 * fmax(scale, cell) + 1e-12;   /* covers the DDA's rounding */
    int64_t total = 1;
    for (int ax = 0; ax < 3; ++ax) {
        G->lo[ax] = lo[ax] - r_s - 2.0 * pad;
        G->dims[ax] = (int64_t)ceil((hi[ax] + r_s + 2.0 * pad - G->lo[ax]) / cell) + 1;
        total *= G->dims[ax];
    }
    G->cell = cell;
    G->begin = calloc((size_t)total + 1, sizeof(int64_t));
    if (!G->begin) { free(G); return NULL; }
    for (int pass = 0; pass < 2; ++pass) {
        for (int64_t i = 0; i < n; ++i) {
            int64_t a0[3], a1[3];
            for (int ax = 0; ax < 3; ++ax) {
                double x = (double)xyz[3 * i + ax];
                a0[ax] = (int64_t)floor((x - r_s - pad - G->lo[ax]) / cell);
                a1[ax] = (int64_t)floor((x + r_s + pad - G->lo[ax]) / cell);
                if (a0[ax] < 0) a0[ax] = 0;
                if (a1[ax] >= G->dims[ax]) a1[ax] = G->dims[ax] - 1;
            }
            for (int64_t z = a0[2]; z <= a1[2]; ++z)
                for (int64_t y = a0[1]; y <= a1[1]; ++y)
                    for (int64_t x = a0[0]; x <= a1[0]; ++x) {
                        int64_t cidx = x + G->dims[0] * (y + G->dims[1] * z);
                        if (pass == 0) G->begin[cidx + 1]++;
                        else G->items[G->begin[cidx]++] = i;
                    }
        }
        if (pass == 0) {
            for (int64_t k = 0; k < total; ++k) G->begin[k + 1] += G->begin[k];
            G->items = malloc((size_t)(G->begin[total] > 0 ? G->begin[total] : 1) * sizeof(int64_t));
            if (!G->items) { free(G->begin); free(G); return NULL; }
        } else {
            for (int64_t k = total; k > 0; --k) G->begin[k] = G->begin[k - 1];
            G->begin[0] = 0;
        }
    }
    return G;
}

void oracle_grid_free(OracleGrid* G)
{
    if (!G) return;
    free(G->begin);
    free(G->items);
    free(G);
}

static void trace_range(Work* w)
{
    const OracleArgs* a = w->a;
    const Pts64* P = w->P;
    const int32_t K = a->K;
    const double inv_sqrt3 = 1.0 / sqrt(3.0);
    for (int64_t r = w->lo; r < w->hi; ++r) {
        int64_t g = a->sel ? a->sel[r] : r;
        int32_t i = (int32_t)(g / a->n_rays);
        int64_t j = g % a->n_rays;
        double o[3] = {a->tx[3 * i], a->tx[3 * i + 1], a->tx[3 * i + 2]};
        double d[3] = {a->dirs[3 * j], a->dirs[3 * j + 1], a->dirs[3 * j + 2]};
        {   /* launch directions are FP32 approximations of unit vectors:
             * renormalise so that ray parameters are lengths */
            double inv = 1.0 / sqrt(dot3(d, d));
            d[0] *= inv; d[1] *= inv; d[2] *= inv;
        }
        double L = 0.0;
        int64_t last = -1;
        for (int32_t k = 0; k < K; ++k) {
            if (a->seq) a->seq[r * K + k] = -1;
            if (a->pts) a->pts[(r * K + k) * 3] = a->pts[(r * K + k) * 3 + 1] = a->pts[(r * K + k) * 3 + 2] = NAN;
        }
        for (int32_t b = 0; b <= K; ++b) {
            int64_t s_idx = r * (K + 1) + b;
            if (a->hit_id) a->hit_id[s_idx] = -2;     /* -2: segment not traced */
            if (a->hit_t) a->hit_t[s_idx] = NAN;
            if (a->acc_n) a->acc_n[s_idx] = 0;
        }
        for (int32_t b = 0; b <= K; ++b) {
            int64_t s_idx = r * (K + 1) + b;
            int64_t best;
            double tb;
            int32_t na = 1;
            int64_t acc[ORACLE_MAXACC];
            double tc = INFINITY, t_lo = INFINITY, t_hi = -INFINITY;
            if (a->grid && !a->parity) nearest_hit_grid(a, P, a->grid, o, d, last, &best, &tb);
            else nearest_hit(a, P, o, d, last, b, &best, &tb, &na, acc, &tc, &t_lo, &t_hi);
            if (a->hit_id) a->hit_id[s_idx] = best;
            if (a->hit_t) a->hit_t[s_idx] = tb;
            if (a->seg_o) { a->seg_o[3 * s_idx] = o[0]; a->seg_o[3 * s_idx + 1] = o[1]; a->seg_o[3 * s_idx + 2] = o[2]; }
            if (a->seg_d) { a->seg_d[3 * s_idx] = d[0]; a->seg_d[3 * s_idx + 1] = d[1]; a->seg_d[3 * s_idx + 2] = d[2]; }
            if (a->parity) {
                if (t_lo > tb) t_lo = tb;
                if (t_hi < tb) t_hi = tb;
                if (a->acc_n) a->acc_n[s_idx] = na;
                if (a->acc_tc) a->acc_tc[s_idx] = tc;
                for (int32_t q = 0; q < na && q < ORACLE_MAXACC; ++q)
                    if (a->acc_id) a->acc_id[s_idx * ORACLE_MAXACC + q] = acc[q];
            }
            /* reception on [0, tb] */
            const double bb = (double)(b + 1);
            for (int32_t q = 0; q < a->n_rx; ++q) {
                const double rxp[3] = {a->rx[3 * q], a->rx[3 * q + 1], a->rx[3 * q + 2]};
                double v[3] = {rxp[0] - o[0], rxp[1] - o[1], rxp[2] - o[2]};
                double s = dot3(v, d);
                double c[3] = {o[0] + s * d[0] - rxp[0], o[1] + s * d[1] - rxp[1], o[2] + s * d[2] - rxp[2]};
                double dist = sqrt(dot3(c, c));
                double rho = a->sigma * (L + s) * w->alpha * inv_sqrt3;
                int received = (s > 0.0) && (s <= tb) && (dist <= rho);
                int amb = 0;
                if (a->parity) {
                    double band = bb * (a->err_abs + fabs(s) * a->err_dir);
                    if (fabs(s) <= band) amb = 1;
                    if (isfinite(tb) && fabs(s - tb) <= a->tie_rel * tb + band) amb = 1;
                    if (fabs(dist - rho) <= a->edge_rel * fabs(rho) + band) amb = 1;
                    if (na > 1 && s >= t_lo * (1.0 - a->tie_rel) - band &&
                        (s <= t_hi * (1.0 + a->tie_rel) + band || !isfinite(t_hi))) amb = 1;
                    if (s <= -band || dist > rho + a->edge_rel * fabs(rho) + band) amb = 0;   /* clearly out */
                    if (s > t_hi * (1.0 + a->tie_rel) + band) amb = 0;                         /* clearly past */
                }
                if (received || amb) {
                    double lp = L + sqrt(dot3(v, v));
                    if (rec_push(&w->rec, r, g, i, q, b, lp, L + s, (received ? 1 : 0) | (amb ? 2 : 0))) {
                        w->status = -2;
                        return;
                    }
                }
            }
            if (best < 0 || b == K) break;
            /* specular reflection at the hit point */
            double n[3] = {P->nx[best], P->ny[best], P->nz[best]};
            double qp[3] = {o[0] + tb * d[0], o[1] + tb * d[1], o[2] + tb * d[2]};
            if (a->seq) a->seq[r * K + b] = (int64_t)a->label[best];
            if (a->pts) { a->pts[(r * K + b) * 3] = qp[0]; a->pts[(r * K + b) * 3 + 1] = qp[1]; a->pts[(r * K + b) * 3 + 2] = qp[2]; }
            L += tb;
            double dn = dot3(d, n);
            double e[3] = {d[0] - 2.0 * dn * n[0], d[1] - 2.0 * dn * n[1], d[2] - 2.0 * dn * n[2]};
            double inv = 1.0 / sqrt(dot3(e, e));
            d[0] = e[0] * inv; d[1] = e[1] * inv; d[2] = e[2] * inv;
            o[0] = qp[0]; o[1] = qp[1]; o[2] = qp[2];
            last = best;
        }
    }
}

static void* worker(void* p)
{
    trace_range((Work*)p);
    return NULL;
}

/* Returns 0 on success, -1 on bad arguments, -2 out of host memory,
 * -3 if the records did not fit (n_rec holds the number needed). */
int oracle_launch(OracleArgs* a)
{
    if (!a || a->n_pts < 0 || (a->n_pts > 0 && (!a->xyz || !a->nrm || !a->label)) || a->n_tx < 1 ||
        !a->tx || a->n_rx < 0 || (a->n_rx > 0 && !a->rx) || a->n_rays < 1 || !a->dirs || a->K < 0 ||
        !(a->r_s > 0.0))
        return -1;
    int64_t n_trace = a->sel ? a->n_sel : (int64_t)a->n_tx * a->n_rays;
    Pts64 P;
    size_t nb = (size_t)(a->n_pts > 0 ? a->n_pts : 1) * sizeof(double);
    P.px = malloc(nb); P.py = malloc(nb); P.pz = malloc(nb);
    P.nx = malloc(nb); P.ny = malloc(nb); P.nz = malloc(nb);
    if (!P.px || !P.py || !P.pz || !P.nx || !P.ny || !P.nz) return -2;
    for (int64_t m = 0; m < a->n_pts; ++m) {
        P.px[m] = a->xyz[3 * m]; P.py[m] = a->xyz[3 * m + 1]; P.pz[m] = a->xyz[3 * m + 2];
        double nx = a->nrm[3 * m], ny = a->nrm[3 * m + 1], nz = a->nrm[3 * m + 2];
        double len = sqrt(nx * nx + ny * ny + nz * nz);
        if (!(len > 0.0) || !isfinite(len)) {
            free(P.px); free(P.py); free(P.pz); free(P.nx); free(P.ny); free(P.nz);
            return -1;
        }
        P.nx[m] = nx / len; P.ny[m] = ny / len; P.nz[m] = nz / len;
    }
    double alpha = a->alpha > 0.0 ? a->alpha : oracle_ray_spacing(a->n_rays);
    int nt = a->n_threads > 0 ? a->n_threads : 1;
    if (nt > n_trace) nt = (int)(n_trace > 0 ? n_trace : 1);
    Work* W = calloc((size_t)nt, sizeof(Work));
    pthread_t* T = calloc((size_t)nt, sizeof(pthread_t));
    int status = 0;
    if (!W || !T) status = -2;
    for (int k = 0; k < nt && !status; ++k) {
        W[k].a = a; W[k].P = &P; W[k].alpha = alpha;
        W[k].lo = n_trace * k / nt; W[k].hi = n_trace * (k + 1) / nt;
    }
    if (!status) {
        for (int k = 1; k < nt; ++k) pthread_create(&T[k], NULL, worker, &W[k]);
        worker(&W[0]);
        for (int k = 1; k < nt; ++k) pthread_join(T[k], NULL);
        int64_t total = 0;
        for (int k = 0; k < nt; ++k) {
            if (W[k].status) status = W[k].status;
            total += W[k].rec.n;
        }
        a->n_rec = total;
        if (!status && total > a->rec_cap) status = -3;
        if (!status) {
            int64_t at = 0;
            for (int k = 0; k < nt; ++k) {
                RecBuf* r = &W[k].rec;
                for (int64_t q = 0; q < r->n; ++q, ++at) {
                    if (a->rec_sel) a->rec_sel[at] = r->sel[q];
                    if (a->rec_g) a->rec_g[at] = r->g[q];
                    if (a->rec_tx) a->rec_tx[at] = r->tx[q];
                    if (a->rec_rx) a->rec_rx[at] = r->rx[q];
                    if (a->rec_b) a->rec_b[at] = r->b[q];
                    if (a->rec_lpoly) a->rec_lpoly[at] = r->lp[q];
                    if (a->rec_lunf) a->rec_lunf[at] = r->lu[q];
                    if (a->rec_flags) a->rec_flags[at] = r->flags[q];
                }
            }
        }
    }
    for (int k = 0; W && k < nt; ++k) rec_free(&W[k].rec);
    free(W); free(T);
    free(P.px); free(P.py); free(P.pz); free(P.nx); free(P.ny); free(P.nz);
    return status;
}

/* Membership of point m in the acceptable set of one segment (parity mode):
 * the segment starts at o with unit direction d (FP64, as the oracle traced
 * it), has index b, left point `last` and nearest clear hit tc (acc_tc).
 * The same test as the set nearest_hit builds, for sets too large to store.
 * Returns 1 or 0, -1 on bad arguments. */
int oracle_accepts(const OracleArgs* a, const double* o, const double* d, int32_t b, int64_t last,
                   double tc, int64_t m)
{
    if (!a || !o || !d || m < -1 || m >= a->n_pts || b < 0) return -1;
    if (m == -1) return tc == INFINITY;
    if (m == last) return 0;
    double n[3] = {a->nrm[3 * m], a->nrm[3 * m + 1], a->nrm[3 * m + 2]};
    double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    if (!(len > 0.0) || !isfinite(len)) return -1;
    n[0] /= len; n[1] /= len; n[2] /= len;
    const double p[3] = {a->xyz[3 * m], a->xyz[3 * m + 1], a->xyz[3 * m + 2]};
    double t, band;
    int cand, amb;
    if (!surfel_class(a, p, n, o, d, (double)(b + 1), &t, &band, &cand, &amb)) return 0;
    return t <= tc * (1.0 + a->tie_rel) + band && (cand || amb);
}

/* ------------------------------------------------------------------------ */
/* visibility rays of the cone tracer (Section 2.2.2 and Section 2.2.4)      */
/* ------------------------------------------------------------------------ */

/*
 * A ray from o towards an intersectable entity's reception point p checks
 * that the entity is visible: nothing of the point cloud may be hit before
 * the ray enters the entity's subvoxel (the box [box_lo, box_hi]).  Hits use
 * the surfel disks of the launcher (same test as nearest_hit: t > t_eps,
 * |o + t u - p_m| <= r_s, u = (p - o)/|p - o|).  Per ray the answer is
 * 1 visible, 0 blocked; in parity mode 2 marks a decision that the FP32 error
 * bands can flip (a surfel that is a hit or ambiguous under the bands lies
 * within the band of t_in, or the nearest clear hit does).  t_out receives
 * t_in (the box entry distance along u, 0 when o is inside the box).
 */
typedef struct {
    const OracleArgs* a;
    const Pts64* P;
    const double *o, *p, *box;
    int64_t lo, hi;
    int32_t* state;
    double* t_out;
} VisWork;

static double box_entry(const double* o, const double* u, const double* lo, const double* hi)
{
    double t0 = 0.0, t1 = INFINITY;
    for (int ax = 0; ax < 3; ++ax) {
        if (u[ax] != 0.0) {
            double ta = (lo[ax] - o[ax]) / u[ax], tb = (hi[ax] - o[ax]) / u[ax];
            if (ta > tb) { double t = ta; ta = tb; tb = t; }
            if (ta > t0) t0 = ta;
            if (tb < t1) t1 = tb;
        } else if (o[ax] < lo[ax] || o[ax] > hi[ax]) {
            return INFINITY;
        }
    }
    return t0 <= t1 ? t0 : INFINITY;
}

static void* vis_worker(void* arg)
{
    VisWork* w = (VisWork*)arg;
    const OracleArgs* a = w->a;
    const Pts64* P = w->P;
    for (int64_t r = w->lo; r < w->hi; ++r) {
        const double* o = w->o + 3 * r;
        const double* p = w->p + 3 * r;
        double u[3] = {p[0] - o[0], p[1] - o[1], p[2] - o[2]};
        double len = sqrt(dot3(u, u));
        if (!(len > 0.0)) { w->state[r] = 1; if (w->t_out) w->t_out[r] = 0.0; continue; }
        u[0] /= len; u[1] /= len; u[2] /= len;
        const double t_in = box_entry(o, u, w->box + 6 * r, w->box + 6 * r + 3);
        if (w->t_out) w->t_out[r] = t_in;
        double t_clear = INFINITY, t_soft = INFINITY, band_at = 0.0;
        for (int64_t m = 0; m < a->n_pts; ++m) {
            const double pm[3] = {P->px[m], P->py[m], P->pz[m]}, nm[3] = {P->nx[m], P->ny[m], P->nz[m]};
            if (!a->parity) {
                double t;
                if (surfel_hit(a, P, o, u, m, &t) && t < t_clear) t_clear = t;
                continue;
            }
            double t, band;
            int cand, amb;
            if (!surfel_class(a, pm, nm, o, u, 1.0, &t, &band, &cand, &amb)) continue;
            if (cand && !amb && t < t_clear) { t_clear = t; }
            if ((cand || amb) && t < t_soft) { t_soft = t; band_at = band; }
        }
        if (!a->parity) { w->state[r] = t_clear >= t_in ? 1 : 0; continue; }
        /* the compared implementation's t_in and t moves by the same bands */
        const double band = (a->err_abs + fabs(t_in) * a->err_dir) + band_at + a->tie_rel * t_in;
        if (t_soft >= t_in + band) w->state[r] = 1;           /* clearly nothing before the box */
        else if (t_clear < t_in - band) w->state[r] = 0;      /* clearly blocked */
        else w->state[r] = 2;
    }
    return NULL;
}

int oracle_visibility(const OracleArgs* a, int64_t n, const double* o, const double* p, const double* box,
                      int32_t* state, double* t_out)
{
    if (!a || n < 0 || (n > 0 && (!o || !p || !box || !state)) || a->n_pts < 0 ||
        (a->n_pts > 0 && (!a->xyz || !a->nrm)) || !(a->r_s > 0.0))
        return -1;
    Pts64 P;
    size_t nb = (size_t)(a->n_pts > 0 ? a->n_pts : 1) * sizeof(double);
    P.px = malloc(nb); P.py = malloc(nb); P.pz = malloc(nb);
    P.nx = malloc(nb); P.ny = malloc(nb); P.nz = malloc(nb);
    int status = (!P.px || !P.py || !P.pz || !P.nx || !P.ny || !P.nz) ? -2 : 0;
    for (int64_t m = 0; m < a->n_pts && !status; ++m) {
        P.px[m] = a->xyz[3 * m]; P.py[m] = a->xyz[3 * m + 1]; P.pz[m] = a->xyz[3 * m + 2];
        double nx = a->nrm[3 * m], ny = a->nrm[3 * m + 1], nz = a->nrm[3 * m + 2];
        double len = sqrt(nx * nx + ny * ny + nz * nz);
        if (!(len > 0.0) || !isfinite(len)) status = -1;
        else { P.nx[m] = nx / len; P.ny[m] = ny / len; P.nz[m] = nz / len; }
    }
    if (!status && n > 0) {
        int nt = a->n_threads > 0 ? a->n_threads : 1;
        if (nt > n) nt = (int)n;
        VisWork* W = calloc((size_t)nt, sizeof(VisWork));
        pthread_t* T = calloc((size_t)nt, sizeof(pthread_t));
        if (!W || !T) status = -2;
        for (int k = 0; k < nt && !status; ++k) {
            W[k] = (VisWork){a, &P, o, p, box, n * k / nt, n * (k + 1) / nt, state, t_out};
        }
        if (!status) {
            for (int k = 1; k < nt; ++k) pthread_create(&T[k], NULL, vis_worker, &W[k]);
            vis_worker(&W[0]);
            for (int k = 1; k < nt; ++k) pthread_join(T[k], NULL);
        }
        free(W); free(T);
    }
    free(P.px); free(P.py); free(P.pz); free(P.nx); free(P.ny); free(P.nz);
    return status;
}

/* ------------------------------------------------------------------------ */
/* path refinement (Section 2.3, Eq. 2)                                      */
/* ------------------------------------------------------------------------ */

/*
 * Each coarse path (TX, interaction points q_1..q_N, RX) is refined into an
 * exact path by minimising its length f = sum_k |I_k - I_{k+1}| (Eq. 2),
 * I_0 = TX, I_{N+1} = RX.  An interaction point I_k = c_k + r_k u_k + s_k v_k
 * moves in the tangent plane of the surface at its current position c_k
 * (u_k, v_k orthonormal to the normal n_k there); r_k u_k + s_k v_k is the
 * projection of the step onto that plane, so no explicit basis is needed.
 * One iteration:
 *   1. G_k = (I_k - I_{k-1})/|I_k - I_{k-1}| + (I_k - I_{k+1})/|I_k - I_{k+1}|,
 *      the derivative of the local length f_k with respect to I_k;
 *      g_k = G_k - (G_k . n_k) n_k = (df_k/dr_k) u_k + (df_k/ds_k) v_k;
 *   2. stop (converged) when |(g_1 .. g_N)| < delta;
 *   3. every point takes the gradient step R_k = c_k - a_k g_k at once;
 *   4. for k = 1..N a ray is traced from the (new) I_{k-1} towards R_k; its
 *      nearest hit gives the new c_k and n_k (the hit surfel's normal); a
 *      ray that hits nothing ends the refinement (invalid path).
 * After rho iterations without convergence the path is invalid.  With
 * smooth_h > 0 the normal n_k is the weighted average of the normals of the
 * points within smooth_h of c_k (the smooth surface normal of Eq. 1) instead
 * of the hit surfel's own.  The step
 * size is not given in the paper: a_k = eta / (1/|c_k - I_{k-1}| +
 * 1/|c_k - I_{k+1}|) scales the step by the inverse of the largest curvature
 * of f_k in the tangent plane.  The initial c_k are found the same way as in
 * step 4, tracing towards the coarse points q_k.  A converged path is valid
 * if both neighbours of every interaction lie on the same side of its
 * surface (a reflection, not a crossing) and the last segment to the RX is
 * not blocked (the segments before it end at nearest hits by construction).
 *
 * Diffraction (edge_of[p*K + k] >= 0): the point is D_k = a + t_k w on its
 * edge's segment [a, b] (w = (b - a)/|b - a|, Section 2.3), starting at the
 * projection of the coarse point; the derivative of f_k along the edge is
 * G_k . w, and t_k steps by a_k (G_k . w) with the same a_k.  No ray is
 * traced to a diffraction point.  A ray leaving a diffraction point starts
 * r_s further along its direction (the surfels of the edge's own faces meet
 * the edge), and a segment arriving at one is blocked only by a hit more
 * than r_s before it.  A step taking t_k off [0, |b - a|] ends the path
 * (off the edge).  A converged path also needs both neighbours of every
 * diffraction point outside the edge's wedge ((I - D) . n1 > 0 or
 * (I - D) . n2 > 0 with the faces' outward normals) and every segment
 * arriving at a diffraction point unblocked.
 */

#define ORACLE_REF_VALID 0
#define ORACLE_REF_NOT_CONVERGED 1
#define ORACLE_REF_MISS 2
#define ORACLE_REF_WRONG_SIDE 3
#define ORACLE_REF_OCCLUDED 4
#define ORACLE_REF_DEGENERATE 5
#define ORACLE_REF_OFF_EDGE 6

typedef struct {
    const float* xyz;          /* [n_pts*3] */
    const float* nrm;          /* [n_pts*3] */
    const uint32_t* label;     /* [n_pts] */
    int64_t n_pts;
    double r_s, t_eps;
    int64_t n_paths;
    int32_t K;                 /* stride of the per-path point arrays */
    const double* tx;          /* [n_paths*3] TX of each path */
    const double* rx;          /* [n_paths*3] RX of each path */
    const int32_t* n_refl;     /* [n_paths] N */
    const double* pts;         /* [n_paths*K*3] coarse interaction points */
    int32_t max_iters;         /* rho */
    double grad_tol;           /* delta */
    double step;               /* eta */
    double smooth_h;           /* > 0: surface normal = weighted average of normals within this radius */
    int32_t n_threads;
    int32_t* status;           /* ORACLE_REF_* */
    int32_t* iters;            /* gradient steps taken */
    double* grad;              /* final |g| */
    double* length;            /* f of the final points */
    double* out_pts;           /* [n_paths*K*3], NaN past N */
    int64_t* out_id;           /* [n_paths*K] surfel of each interaction, -1 past N */
    int64_t* out_label;        /* [n_paths*K], -1 past N */
    /* diffraction edges; edge_of NULL: every interaction is a reflection */
    const int32_t* edge_of;    /* [n_paths*K]: edge of interaction k, -1 for a reflection */
    int32_t n_edges;
    const double* edge_seg;    /* [n_edges*6]: end points a, b */
    const double* edge_nrm;    /* [n_edges*6]: outward normals n1, n2 of the two faces */
    const int64_t* edge_label; /* [n_edges] */
} OracleRefineArgs;

typedef struct {
    const OracleRefineArgs* a;
    const Pts64* P;
    int64_t lo, hi;
} RefWork;

static double dist3(const double* p, const double* q)
{
    double e[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
    return sqrt(dot3(e, e));
}

/* Surface normal at c as the weighted average of the nearby points' normals
 * (the n(x) of Eq. 1): weights (1 - |c - p|^2 / h^2)^4 for |c - p| < h (the
 * paper gives no kernel; this one is smooth and vanishes at h), each normal
 * oriented to agree with the hit surfel's normal `nh`.  Replaces nh unless
 * no point lies within h. */
static void smooth_normal(const Pts64* P, int64_t n_pts, double h, const double* c, double* nh)
{
    const double h2 = h * h;
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t q = 0; q < n_pts; ++q) {
        double dx = P->px[q] - c[0], dy = P->py[q] - c[1], dz = P->pz[q] - c[2];
        double d2 = dx * dx + dy * dy + dz * dz;
        if (!(d2 < h2)) continue;
        double w = 1.0 - d2 / h2;
        w = w * w;
        w = w * w;
        double sg = (P->nx[q] * nh[0] + P->ny[q] * nh[1] + P->nz[q] * nh[2]) < 0.0 ? -w : w;
        s[0] += sg * P->nx[q];
        s[1] += sg * P->ny[q];
        s[2] += sg * P->nz[q];
    }
    double l = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
    if (l > 0.0) { nh[0] = s[0] / l; nh[1] = s[1] / l; nh[2] = s[2] / l; }
}

/* Nearest hit of the ray from o towards target (excluding surfel `last`),
 * the ray starting `skip` along its direction.  Returns 1 with the hit
 * point, normal and surfel (t_out: its distance from o), 0 on a miss, -1 if
 * the target coincides with o. */
static int trace_towards(const OracleArgs* A, const Pts64* P, const double* o, const double* target, int64_t last,
                         double skip, double* c, double* n, int64_t* m, double* t_out)
{
    double d[3] = {target[0] - o[0], target[1] - o[1], target[2] - o[2]};
    double len = sqrt(dot3(d, d));
    if (!(len > 0.0)) return -1;
    d[0] /= len; d[1] /= len; d[2] /= len;
    const double os[3] = {o[0] + skip * d[0], o[1] + skip * d[1], o[2] + skip * d[2]};
    int64_t best;
    double tb;
    int32_t na;
    int64_t acc[ORACLE_MAXACC];
    double tc, t_lo, t_hi;
    nearest_hit(A, P, os, d, last, 0, &best, &tb, &na, acc, &tc, &t_lo, &t_hi);
    if (t_out) *t_out = skip + tb;
    if (best < 0) return 0;
    c[0] = os[0] + tb * d[0]; c[1] = os[1] + tb * d[1]; c[2] = os[2] + tb * d[2];
    n[0] = P->nx[best]; n[1] = P->ny[best]; n[2] = P->nz[best];
    *m = best;
    return 1;
}

static void refine_one(const OracleRefineArgs* a, const OracleArgs* A, const Pts64* P, int64_t p)
{
    const int32_t K = a->K;
    const int32_t N = a->n_refl[p];
    const double* T = a->tx + 3 * p;
    const double* R = a->rx + 3 * p;
    double c[ORACLE_MAXN][3], n[ORACLE_MAXN][3], g[ORACLE_MAXN][3], tgt[ORACLE_MAXN][3];
    /* diffraction points: edge, its start a, unit direction w, length, parameter t */
    int32_t E[ORACLE_MAXN];
    double ea[ORACLE_MAXN][3], ew[ORACLE_MAXN][3], el[ORACLE_MAXN], tp[ORACLE_MAXN];
    int64_t m[ORACLE_MAXN];
    int32_t status = ORACLE_REF_VALID, it = 0;
    double gnorm = 0.0;
    const double clear = a->r_s;
    for (int32_t k = 0; k < K; ++k) {
        a->out_id[p * K + k] = -1;
        a->out_label[p * K + k] = -1;
        a->out_pts[(p * K + k) * 3] = a->out_pts[(p * K + k) * 3 + 1] = a->out_pts[(p * K + k) * 3 + 2] = NAN;
    }
    for (int32_t k = 0; k < N; ++k) {
        for (int j = 0; j < 3; ++j) tgt[k][j] = a->pts[(p * K + k) * 3 + j];
        E[k] = a->edge_of ? a->edge_of[p * K + k] : -1;
        m[k] = -1;
        if (E[k] >= 0) {
            const double* sg = a->edge_seg + 6 * (int64_t)E[k];
            double d[3] = {sg[3] - sg[0], sg[4] - sg[1], sg[5] - sg[2]};
            el[k] = sqrt(dot3(d, d));
            for (int j = 0; j < 3; ++j) { ea[k][j] = sg[j]; ew[k][j] = d[j] / el[k]; }
            double q[3] = {tgt[k][0] - ea[k][0], tgt[k][1] - ea[k][1], tgt[k][2] - ea[k][2]};
            tp[k] = dot3(q, ew[k]);   /* the coarse point's projection onto the edge */
        }
    }
    /* I(k) for k = 0..N+1 */
#define IPT(k) ((k) == 0 ? T : ((k) == N + 1 ? R : c[(k) - 1]))
#define DIFF(k) ((k) >= 1 && (k) <= N && E[(k) - 1] >= 0)
    for (;;) {
        /* the interaction points: diffraction points on their edges, reflection points traced
           towards the targets (the coarse points first, then the gradient steps) */
        int64_t last = -1;
        double skip = 0.0;
        for (int32_t k = 0; k < N && status == ORACLE_REF_VALID; ++k) {
            if (E[k] >= 0) {
                for (int j = 0; j < 3; ++j) c[k][j] = ea[k][j] + tp[k] * ew[k][j];
                last = -1;
                skip = clear;
                continue;
            }
            int r = trace_towards(A, P, IPT(k), tgt[k], last, skip, c[k], n[k], &m[k], NULL);
            if (r > 0 && a->smooth_h > 0.0) smooth_normal(P, a->n_pts, a->smooth_h, c[k], n[k]);
            if (r < 0) status = ORACLE_REF_DEGENERATE;
            else if (r == 0) status = ORACLE_REF_MISS;
            last = m[k];
            skip = 0.0;
        }
        if (status != ORACLE_REF_VALID) break;
        /* gradient of the path length: tangent planes of reflections, edge directions of diffractions */
        double gg = 0.0;
        for (int32_t k = 1; k <= N; ++k) {
            const double* I = IPT(k);
            const double* Ip = IPT(k - 1);
            const double* In = IPT(k + 1);
            double lp = dist3(I, Ip), ln = dist3(I, In);
            if (!(lp > 0.0) || !(ln > 0.0)) { status = ORACLE_REF_DEGENERATE; break; }
            double G[3];
            for (int j = 0; j < 3; ++j) G[j] = (I[j] - Ip[j]) / lp + (I[j] - In[j]) / ln;
            if (E[k - 1] >= 0) {
                double gw = dot3(G, ew[k - 1]);
                for (int j = 0; j < 3; ++j) g[k - 1][j] = gw * ew[k - 1][j];
                gg += gw * gw;
            } else {
                double gn = dot3(G, n[k - 1]);
                for (int j = 0; j < 3; ++j) g[k - 1][j] = G[j] - gn * n[k - 1][j];
                gg += dot3(g[k - 1], g[k - 1]);
            }
        }
        if (status != ORACLE_REF_VALID) break;
        gnorm = sqrt(gg);
        if (gnorm < a->grad_tol) break;
        if (it == a->max_iters) { status = ORACLE_REF_NOT_CONVERGED; break; }
        /* simultaneous gradient step of every point */
        int off = 0;
        for (int32_t k = 1; k <= N; ++k) {
            const double* I = IPT(k);
            double step = a->step / (1.0 / dist3(I, IPT(k - 1)) + 1.0 / dist3(I, IPT(k + 1)));
            if (E[k - 1] >= 0) {
                tp[k - 1] -= step * dot3(g[k - 1], ew[k - 1]);
                if (!(tp[k - 1] >= 0.0 && tp[k - 1] <= el[k - 1])) off = 1;
            } else {
                for (int j = 0; j < 3; ++j) tgt[k - 1][j] = I[j] - step * g[k - 1][j];
            }
        }
        if (off) { status = ORACLE_REF_OFF_EDGE; break; }
        ++it;
    }
    if (status == ORACLE_REF_VALID) {
        /* a reflection keeps both neighbours on one side of the surface; a diffraction has
           both outside the edge's wedge */
        for (int32_t k = 1; k <= N && status == ORACLE_REF_VALID; ++k) {
            const double* I = IPT(k);
            if (E[k - 1] >= 0) {
                const double* nn = a->edge_nrm + 6 * (int64_t)E[k - 1];
                for (int side = 0; side < 2; ++side) {
                    const double* X = IPT(side ? k + 1 : k - 1);
                    double v[3] = {X[0] - I[0], X[1] - I[1], X[2] - I[2]};
                    if (!(dot3(v, nn) > 0.0 || dot3(v, nn + 3) > 0.0)) status = ORACLE_REF_WRONG_SIDE;
                }
                continue;
            }
            double sp = 0.0, sn = 0.0;
            for (int j = 0; j < 3; ++j) {
                sp += (IPT(k - 1)[j] - I[j]) * n[k - 1][j];
                sn += (IPT(k + 1)[j] - I[j]) * n[k - 1][j];
            }
            if (!(sp * sn > 0.0)) status = ORACLE_REF_WRONG_SIDE;
        }
    }
    /* segments not ending at a nearest hit: those arriving at a diffraction point (blocked by a
       hit more than r_s before it) and the last one, to the RX */
    for (int32_t k = 1; k <= N + 1 && status == ORACLE_REF_VALID; ++k) {
        if (k <= N && E[k - 1] < 0) continue;
        const int prev_diff = DIFF(k - 1);
        double cc[3], nn[3], tb;
        int64_t mm;
        const double len = dist3(IPT(k - 1), IPT(k));
        int r = trace_towards(A, P, IPT(k - 1), IPT(k), (k >= 2 && !prev_diff) ? m[k - 2] : -1,
                              prev_diff ? clear : 0.0, cc, nn, &mm, &tb);
        if (r < 0) status = ORACLE_REF_DEGENERATE;
        else if (r > 0 && tb < (k <= N ? len - clear : len)) status = ORACLE_REF_OCCLUDED;
    }
    double f = 0.0;
    int finite = (status != ORACLE_REF_MISS && status != ORACLE_REF_DEGENERATE);
    for (int32_t k = 0; k <= N && finite; ++k) f += dist3(IPT(k), IPT(k + 1));
    a->length[p] = finite ? f : NAN;
    a->status[p] = status;
    a->iters[p] = it;
    a->grad[p] = finite ? gnorm : NAN;
    if (finite)
        for (int32_t k = 0; k < N; ++k) {
            a->out_id[p * K + k] = E[k] >= 0 ? -2 - (int64_t)E[k] : m[k];
            a->out_label[p * K + k] = E[k] >= 0 ? a->edge_label[E[k]] : (int64_t)a->label[m[k]];
            for (int j = 0; j < 3; ++j) a->out_pts[(p * K + k) * 3 + j] = c[k][j];
        }
#undef DIFF
#undef IPT
}

static void* refine_worker(void* q)
{
    RefWork* w = (RefWork*)q;
    OracleArgs A;
    memset(&A, 0, sizeof(A));
    A.n_pts = w->a->n_pts;
    A.r_s = w->a->r_s;
    A.t_eps = w->a->t_eps;
    for (int64_t p = w->lo; p < w->hi; ++p) refine_one(w->a, &A, w->P, p);
    return NULL;
}

/* Returns 0, -1 on bad arguments, -2 out of host memory. */
int oracle_refine(OracleRefineArgs* a)
{
    if (!a || a->n_pts < 0 || (a->n_pts > 0 && (!a->xyz || !a->nrm || !a->label)) || a->n_paths < 0 ||
        a->K < 0 || a->K > ORACLE_MAXN || !(a->r_s > 0.0) || a->max_iters < 0 || !(a->step > 0.0))
        return -1;
    for (int64_t p = 0; p < a->n_paths; ++p)
        if (a->n_refl[p] < 0 || a->n_refl[p] > a->K) return -1;
    if (a->edge_of) {
        if (a->n_edges < 0 || (a->n_edges > 0 && (!a->edge_seg || !a->edge_nrm || !a->edge_label))) return -1;
        for (int64_t q = 0; q < a->n_paths * a->K; ++q)
            if (a->edge_of[q] < -1 || a->edge_of[q] >= a->n_edges) return -1;
        for (int32_t e = 0; e < a->n_edges; ++e) {
            const double* sg = a->edge_seg + 6 * (int64_t)e;
            double d[3] = {sg[3] - sg[0], sg[4] - sg[1], sg[5] - sg[2]};
            if (!(dot3(d, d) > 0.0)) return -1;
        }
    }
    Pts64 P;
    size_t nb = (size_t)(a->n_pts > 0 ? a->n_pts : 1) * sizeof(double);
    P.px = malloc(nb); P.py = malloc(nb); P.pz = malloc(nb);
    P.nx = malloc(nb); P.ny = malloc(nb); P.nz = malloc(nb);
    int status = (!P.px || !P.py || !P.pz || !P.nx || !P.ny || !P.nz) ? -2 : 0;
    for (int64_t q = 0; q < a->n_pts && !status; ++q) {
        P.px[q] = a->xyz[3 * q]; P.py[q] = a->xyz[3 * q + 1]; P.pz[q] = a->xyz[3 * q + 2];
        double nx = a->nrm[3 * q], ny = a->nrm[3 * q + 1], nz = a->nrm[3 * q + 2];
        double len = sqrt(nx * nx + ny * ny + nz * nz);
        if (!(len > 0.0) || !isfinite(len)) status = -1;
        else { P.nx[q] = nx / len; P.ny[q] = ny / len; P.nz[q] = nz / len; }
    }
    int nt = a->n_threads > 0 ? a->n_threads : 1;
    if (nt > a->n_paths) nt = (int)(a->n_paths > 0 ? a->n_paths : 1);
    RefWork* W = calloc((size_t)nt, sizeof(RefWork));
    pthread_t* T = calloc((size_t)nt, sizeof(pthread_t));
    if (!status && (!W || !T)) status = -2;
    if (!status) {
        for (int k = 0; k < nt; ++k) {
            W[k].a = a; W[k].P = &P;
            W[k].lo = a->n_paths * k / nt; W[k].hi = a->n_paths * (k + 1) / nt;
        }
        for (int k = 1; k < nt; ++k) pthread_create(&T[k], NULL, refine_worker, &W[k]);
        refine_worker(&W[0]);
        for (int k = 1; k < nt; ++k) pthread_join(T[k], NULL);
    }
    free(W); free(T);
    free(P.px); free(P.py); free(P.pz); free(P.nx); free(P.ny); free(P.nz);
    return status;
}
