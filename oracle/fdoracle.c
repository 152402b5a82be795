/*
 * fdoracle.c -- plain, untiled FP64 reference of the acoustic finite-difference
 * sweep (forward, adjoint, gradient).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this file; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code with the HIP library.
 *
 * What it computes (paper: Sec. 6.3.1, Fig. "acoustic_devito"; the damped
 * leapfrog of the second-order-in-time acoustic wave equation
 *     m u_tt + damp u_t - Lap(u) = source,   m = 1/v^2):
 *
 *   u^{n+1}(i) = ((dt*damp - 2m) u^{n-1} + 4m u^n + 2 dt^2 L_h u^n) / (dt*damp + 2m)
 *
 * with L_h the star Laplacian of space order so = 2M,
 *   L_h u(i) = sum_a [ c_0 u(i) + sum_{k=1..M} c_k (u(i - k e_a) + u(i + k e_a)) ] / h_a^2,
 * u == 0 outside the grid (the paper's never-written ghost cells, Sec. 6.3.1
 * loop bounds), the closed-form central-difference weights
 *   c_k = 2 (-1)^{k+1} (M!)^2 / (k^2 (M-k)! (M+k)!),   c_0 = -2 sum_k c_k,
 * whose so=8 values scaled by 2 dt^2/h^2 are the constants the paper prints.
 *
 * Readings of what the paper leaves open (source/receiver/sponge are only named
 * there, not defined):
 *   * point source injection in the step that produces u^{n+1}:
 *       u^{n+1}(s) += 2 dt^2 w[n][s] / (dt*damp(s) + 2 m(s))
 *   * receivers sample the new level on grid nodes: d[n][r] = u^{n+1}(r)
 *   * a point off the grid (a position in grid-index units, p_a in [0, n_a - 1])
 *     acts through multilinear interpolation: P is the row of weights
 *     w_c = prod_a (c_a ? f_a : 1 - f_a) over the 2^d nodes c of the cell that
 *     holds it (f_a the fractional part; on the last node of an axis the cell
 *     below is used).  A receiver records P u^{n+1}; a source adds
 *     A^{-1} 2 dt^2 P^T w, i.e. w_c 2 dt^2 w / (dt*damp(c) + 2 m(c)) at each node
 *     (the definitions above are the special case of a single node, weight 1).
 *   * or, per point set, Kaiser-windowed sinc interpolation of half-width r
 *     (Hicks 2002; 1 <= r <= 8): along each axis the 2r nodes i0-r+1 .. i0+r
 *     around x = i0 + f (i0 = floor x) weigh
 *       s(d) = sinc(d) I0(b sqrt(1 - (d/r)^2)) / I0(b),   d = node - x,
 *     sinc(d) = sin(pi d)/(pi d) (exactly 1 at d = 0, 0 at other integers), the
 *     point's weight at a node is the product over the axes, and nodes outside
 *     the grid drop out (the field is zero there).  b(r) is the window shape
 *     that minimises the largest error of interpolating cos(k x + phase) for
 *     k h <= pi/2 (four points per wavelength), found by a search in steps of
 *     0.1.  P and P^T use the same weights, as above.
 *   * separable sponge: damp(i) = sum_a d0_a (delta_a / L)^2, delta_a the number
 *     of cells into the outer L-cell layer (0 in the interior and at its inner
 *     edge), d0_a = 1.5 ln(1000) / (vref L h_a).  damp carries the units of m
 *     (s/m^2): it is the usual 1/s damping rate 1.5 vref ln(1000) / (L h) divided
 *     by vref^2, a fixed constant, so damp does not depend on the model v.
 *
 * Adjoint: writing step k as  A u^k - B u^{k-1} - C u^{k-2} = 2 dt^2 P_s^T w^{k-1}
 * with A = diag(2m + dt damp), B = 4m + 2 dt^2 L_h (symmetric), C = diag(dt damp - 2m),
 * the transposed system is solved backward in time:
 *   lambda^k = A^{-1} (B lambda^{k+1} + C lambda^{k+2} + P_r^T y[k-1]),  k = nt..1,
 * lambda^{nt+1} = lambda^{nt+2} = 0, and (F^T y)[k-1][s] = 2 dt^2 lambda^k(s).
 * Born (linearised) modelling: differentiating the step with respect to m
 * (dA = 2 dm, dB = 4 dm, dC = -2 dm) gives the perturbation wavefield
 *   A du^k = B du^{k-1} + C du^{k-2} - 2 dm (u^k - 2u^{k-1} + u^{k-2}),
 * du^0 = du^{-1} = 0, and the perturbed traces dd[n] = P_r du^{n+1}; for a
 * velocity perturbation dv, dm = -2 dv / v^3.
 * Gradient of J = 1/2 sum (d - d_obs)^2 (plain sum):
 *   dJ/dm(x) = -2 sum_{k=1..nt} lambda^k(x) (u^k - 2u^{k-1} + u^{k-2})(x),
 *   dJ/dv = dJ/dm * (-2 / v^3).
 *
 * Layout: dense C order, axis ndim-1 contiguous; grids of dimension 1 and 2
 * are handled as 3-D grids with leading unit extents and only the present axes
 * take part in the Laplacian.  The outer loop carries one OpenMP parallel-for,
 * as the paper's untiled "normal" control does (Sec. 6.5, transformation types).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXM 8
#define OR_PI 3.14159265358979323846

typedef struct or_problem {
    int32_t ndim;        /* 1, 2 or 3 */
    int32_t so;          /* space order: even, 2..16 */
    int64_t n[3];        /* extents of the ndim axes, last contiguous */
    double h[3];         /* spacing per axis (m) */
    int64_t nt;          /* time steps */
    double dt;           /* time step (s) */
    int32_t sponge;      /* sponge width L in cells (0: none) */
    int32_t pad0;
    double vref;         /* velocity setting the sponge strength (m/s) */
    const double *v;     /* velocity, N^d (m/s) */
    int32_t ns;          /* number of sources */
    int32_t nr;          /* number of receivers */
    const int32_t *src;  /* [ns][ndim] grid indices (used when spos is NULL) */
    const int32_t *rec;  /* [nr][ndim] grid indices (used when rpos is NULL) */
    const double *spos;  /* [ns][ndim] positions in grid-index units, or NULL */
    const double *rpos;  /* [nr][ndim] positions in grid-index units, or NULL */
    int32_t ssinc;       /* sources: 0 multilinear, r in 1..8 windowed sinc of half-width r */
    int32_t rsinc;       /* receivers: the same */
} or_problem;

/* The nodes a point acts on and their interpolation weights (at most 16^3). */
#define OR_MAXPT 4096
typedef struct stencil_pt {
    int n;
    int64_t idx[OR_MAXPT];
    double w[OR_MAXPT];
} stencil_pt;

typedef struct geom {
    int64_t n[3];   /* extents as 3-D (leading unit axes for ndim < 3) */
    double h[3];
    int first;      /* first present axis: 3 - ndim */
    int64_t npts;
} geom;

static int make_geom(const or_problem *p, geom *g)
{
    if (!p || p->ndim < 1 || p->ndim > 3) return -1;
    g->first = 3 - p->ndim;
    g->npts = 1;
    for (int a = 0; a < 3; ++a) {
        if (a < g->first) { g->n[a] = 1; g->h[a] = 1.0; }
        else {
            g->n[a] = p->n[a - g->first];
            g->h[a] = p->h[a - g->first];
            if (g->n[a] < 1 || !(g->h[a] > 0)) return -1;
        }
        g->npts *= g->n[a];
    }
    return 0;
}

/* Central second-derivative weights of order 2M (closed form), c[0..M]. */
int or_weights(int so, double *c)
{
    if (so < 2 || so > 2 * OR_MAXM || (so & 1)) return -1;
    int M = so / 2;
    double sum = 0.0;
    for (int k = 1; k <= M; ++k) {
        double r = 1.0; /* (M!)^2 / ((M-k)! (M+k)!) as a product of k ratios */
        for (int j = 1; j <= k; ++j) r *= (double)(M - k + j) / (double)(M + j);
        c[k] = 2.0 * ((k & 1) ? 1.0 : -1.0) * r / ((double)k * (double)k);
        sum += c[k];
    }
    c[0] = -2.0 * sum;
    return 0;
}

static double at3(const geom *g, const double *u, int64_t i0, int64_t i1, int64_t i2)
{
    if (i0 < 0 || i0 >= g->n[0] || i1 < 0 || i1 >= g->n[1] || i2 < 0 || i2 >= g->n[2]) return 0.0;
    return u[(i0 * g->n[1] + i1) * g->n[2] + i2];
}

/* L_h u at one point: the definition, axis by axis, u = 0 outside the grid. */
static double lap_point(const geom *g, const double *c, int M, const double *u,
                        int64_t i0, int64_t i1, int64_t i2)
{
    double total = 0.0;
    int64_t ii[3] = {i0, i1, i2};
    for (int a = g->first; a < 3; ++a) {
        double s = c[0] * at3(g, u, i0, i1, i2);
        for (int k = 1; k <= M; ++k) {
            int64_t lo[3] = {ii[0], ii[1], ii[2]}, hi[3] = {ii[0], ii[1], ii[2]};
            lo[a] -= k;
            hi[a] += k;
            s += c[k] * (at3(g, u, lo[0], lo[1], lo[2]) + at3(g, u, hi[0], hi[1], hi[2]));
        }
        total += s / (g->h[a] * g->h[a]);
    }
    return total;
}

static int laplacian_g(const geom *g, int so, const double *u, double *out)
{
    double c[OR_MAXM + 1];
    if (or_weights(so, c)) return -1;
    int M = so / 2;
#pragma omp parallel for schedule(static)
    for (int64_t i0 = 0; i0 < g->n[0]; ++i0)
        for (int64_t i1 = 0; i1 < g->n[1]; ++i1)
            for (int64_t i2 = 0; i2 < g->n[2]; ++i2)
                out[(i0 * g->n[1] + i1) * g->n[2] + i2] = lap_point(g, c, M, u, i0, i1, i2);
    return 0;
}

/* Star Laplacian of order so on a dense ndim grid (zero outside). */
int or_laplacian(int ndim, const int64_t *n, const double *h, int so, const double *u, double *out)
{
    or_problem p;
    memset(&p, 0, sizeof p);
    p.ndim = ndim;
    for (int a = 0; a < ndim; ++a) { p.n[a] = n[a]; p.h[a] = h[a]; }
    geom g;
    if (make_geom(&p, &g)) return -1;
    return laplacian_g(&g, so, u, out);
}

/* Separable sponge profile along one axis (reading stated in the header). */
static double sponge_1d(int64_t i, int64_t n, int L, double h, double vref)
{
    if (L <= 0) return 0.0;
    double delta = 0.0;
    if (i < L) delta = (double)(L - i);
    else if (i > n - 1 - L) delta = (double)(i - (n - 1 - L));
    double d0 = 1.5 * log(1000.0) / (vref * (double)L * h);
    double r = delta / (double)L;
    return d0 * r * r;
}

static void damp_g(const or_problem *p, const geom *g, double *damp)
{
#pragma omp parallel for schedule(static)
    for (int64_t i0 = 0; i0 < g->n[0]; ++i0)
        for (int64_t i1 = 0; i1 < g->n[1]; ++i1)
            for (int64_t i2 = 0; i2 < g->n[2]; ++i2) {
                int64_t ii[3] = {i0, i1, i2};
                double d = 0.0;
                for (int a = g->first; a < 3; ++a)
                    d += sponge_1d(ii[a], g->n[a], p->sponge, g->h[a], p->vref);
                damp[(i0 * g->n[1] + i1) * g->n[2] + i2] = d;
            }
}

int or_damp(const or_problem *p, double *damp)
{
    geom g;
    if (make_geom(p, &g)) return -1;
    damp_g(p, &g, damp);
    return 0;
}

static int64_t point_index(const or_problem *p, const geom *g, const int32_t *idx)
{
    int64_t ii[3] = {0, 0, 0};
    for (int a = 0; a < p->ndim; ++a) {
        int64_t v = idx[a];
        if (v < 0 || v >= p->n[a]) return -1;
        ii[a + g->first] = v;
    }
    return (ii[0] * g->n[1] + ii[1]) * g->n[2] + ii[2];
}

/* One step of the recurrence  A u_new = B u_cur + C u_prev  (no source), with
 * the paper's numerator/denominator form.  Used by forward and adjoint alike,
 * since B is symmetric and A, C are diagonal. */
static void leapfrog_step(const geom *g, const double *c, int M, double dt,
                          const double *m, const double *damp,
                          const double *u_cur, const double *u_prev, double *u_new)
{
    double dt2 = dt * dt;
#pragma omp parallel for schedule(static)
    for (int64_t i0 = 0; i0 < g->n[0]; ++i0)
        for (int64_t i1 = 0; i1 < g->n[1]; ++i1)
            for (int64_t i2 = 0; i2 < g->n[2]; ++i2) {
                int64_t i = (i0 * g->n[1] + i1) * g->n[2] + i2;
                double tcse = dt * damp[i];
                double lap = lap_point(g, c, M, u_cur, i0, i1, i2);
                u_new[i] = ((tcse - 2.0 * m[i]) * u_prev[i] + 4.0 * m[i] * u_cur[i] + 2.0 * dt2 * lap)
                           / (tcse + 2.0 * m[i]);
            }
}

/* Multilinear interpolation of a position: the nodes of its cell with nonzero
 * weight.  -1 if a coordinate is not finite or lies outside [0, n_a - 1]. */
static int point_stencil(const or_problem *p, const geom *g, const double *pos, stencil_pt *out)
{
    int64_t base[3] = {0, 0, 0};
    double f[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < p->ndim; ++a) {
        double x = pos[a];
        int64_t n = p->n[a];
        if (!(x >= 0.0) || !(x <= (double)(n - 1))) return -1;
        int64_t i = (int64_t)floor(x);
        if (i > n - 2) i = n - 2; /* the last node: the cell below, fraction 1 */
        if (i < 0) i = 0;         /* an axis of one node: fraction 0 */
        base[a + g->first] = i;
        f[a + g->first] = x - (double)i;
    }
    out->n = 0;
    for (int c = 0; c < 8; ++c) {
        double w = 1.0;
        int64_t ii[3];
        for (int a = 0; a < 3; ++a) {
            int bit = (c >> (2 - a)) & 1;
            if (a < g->first && bit) { w = 0.0; break; }
            ii[a] = base[a] + bit;
            w *= bit ? f[a] : 1.0 - f[a];
        }
        if (w == 0.0) continue;
        out->idx[out->n] = (ii[0] * g->n[1] + ii[1]) * g->n[2] + ii[2];
        out->w[out->n] = w;
        out->n++;
    }
    return 0;
}

/* Modified Bessel function of the first kind, order 0: its power series
 * sum_j ((x/2)^j / j!)^2, summed until the terms stop mattering. */
static double bessel_i0(double x)
{
    double term = 1.0, sum = 1.0, q = 0.25 * x * x;
    for (int j = 1; j < 200; ++j) {
        term *= q / ((double)j * (double)j);
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return sum;
}

/* Window shape b per half-width r = 1..8 (minimax criterion in the header). */
static const double kaiser_b[9] = {0.0, 1.3, 2.9, 4.5, 6.3, 7.9, 9.4, 10.9, 12.6};

/* Weight of a node at signed distance d (grid units) for half-width r. */
static double ksinc(double d, int r)
{
    double sinc;
    if (d == 0.0) sinc = 1.0;
    else if (d == floor(d)) sinc = 0.0;
    else sinc = sin(OR_PI * d) / (OR_PI * d);
    double t = d / (double)r;
    if (t * t >= 1.0) return 0.0;
    return sinc * bessel_i0(kaiser_b[r] * sqrt(1.0 - t * t)) / bessel_i0(kaiser_b[r]);
}

/* Kaiser-windowed sinc interpolation of a position: the product over the axes
 * of the 1-D weights of the 2r nodes around it, nodes inside the grid and of
 * nonzero weight only.  -1 if a coordinate is not finite or outside [0, n_a - 1]. */
static int sinc_stencil(const or_problem *p, const geom *g, const double *pos, int r,
                        stencil_pt *out)
{
    int64_t lo[3] = {0, 0, 0}, cnt[3] = {1, 1, 1};
    double w1[3][16];
    w1[0][0] = w1[1][0] = w1[2][0] = 1.0;
    for (int a = 0; a < p->ndim; ++a) {
        double x = pos[a];
        int64_t n = p->n[a];
        if (!(x >= 0.0) || !(x <= (double)(n - 1))) return -1;
        int64_t i0 = (int64_t)floor(x);
        int ax = a + g->first;
        lo[ax] = i0 - r + 1;
        cnt[ax] = 2 * r;
        for (int k = 0; k < 2 * r; ++k) {
            int64_t node = lo[ax] + k;
            w1[ax][k] = (node < 0 || node >= n) ? 0.0 : ksinc((double)node - x, r);
        }
    }
    out->n = 0;
    for (int k0 = 0; k0 < cnt[0]; ++k0)
        for (int k1 = 0; k1 < cnt[1]; ++k1)
            for (int k2 = 0; k2 < cnt[2]; ++k2) {
                double w = w1[0][k0] * w1[1][k1] * w1[2][k2];
                if (w == 0.0) continue;
                out->idx[out->n] = ((lo[0] + k0) * g->n[1] + (lo[1] + k1)) * g->n[2] + (lo[2] + k2);
                out->w[out->n] = w;
                out->n++;
            }
    return 0;
}

/* The stencil of point k of a set: one node of weight 1 for grid indices. */
static int set_stencil(const or_problem *p, const geom *g, const int32_t *idx, const double *pos,
                       int r, int k, stencil_pt *out)
{
    if (r < 0 || r > 8 || (r > 0 && !pos)) return -1;
    if (pos && r > 0) return sinc_stencil(p, g, pos + (int64_t)k * p->ndim, r, out);
    if (pos) return point_stencil(p, g, pos + (int64_t)k * p->ndim, out);
    int64_t i = point_index(p, g, idx + (int64_t)k * p->ndim);
    if (i < 0) return -1;
    out->n = 1;
    out->idx[0] = i;
    out->w[0] = 1.0;
    return 0;
}

/* The nodes (flat indices) and weights one point acts on, for the tests:
 * r = 0 multilinear, 1..8 windowed sinc.  Returns the node count, -1 on a bad
 * position or r, -2 if cap is too small. */
int or_point_weights(const or_problem *p, const double *pos, int r, int64_t *idx, double *w, int cap)
{
    geom g;
    if (make_geom(p, &g) || !pos || r < 0 || r > 8) return -1;
    stencil_pt *s = (stencil_pt *)malloc(sizeof(stencil_pt));
    if (!s) return -2;
    int rc = r > 0 ? sinc_stencil(p, &g, pos, r, s) : point_stencil(p, &g, pos, s);
    if (rc == 0 && s->n > cap) rc = -2;
    if (rc == 0) {
        for (int j = 0; j < s->n; ++j) {
            idx[j] = s->idx[j];
            w[j] = s->w[j];
        }
        rc = s->n;
    }
    free(s);
    return rc;
}

/* P u: the value a receiver (or an adjoint source sample) reads. */
static double sample(const stencil_pt *s, const double *u)
{
    double acc = 0.0;
    for (int j = 0; j < s->n; ++j) acc += s->w[j] * u[s->idx[j]];
    return acc;
}

/* u += A^{-1} P^T a: an amplitude a (already multiplied by its time factor)
 * spread over the point's nodes, each divided by its own 2m + dt damp. */
static void spread(const stencil_pt *s, double a, double dt, const double *m, const double *damp,
                   double *u)
{
    for (int j = 0; j < s->n; ++j) {
        int64_t i = s->idx[j];
        u[i] += s->w[j] * a / (dt * damp[i] + 2.0 * m[i]);
    }
}

typedef struct work {
    geom g;
    double c[OR_MAXM + 1];
    int M;
    double *m, *damp;
    stencil_pt *sp, *rp;
} work;

static int work_init(const or_problem *p, work *w)
{
    memset(w, 0, sizeof *w);
    if (make_geom(p, &w->g)) return -1;
    if (or_weights(p->so, w->c)) return -1;
    w->M = p->so / 2;
    if (p->nt < 0 || !(p->dt > 0) || !p->v) return -1;
    int64_t N = w->g.npts;
    w->m = (double *)malloc(sizeof(double) * N);
    w->damp = (double *)malloc(sizeof(double) * N);
    w->sp = (stencil_pt *)malloc(sizeof(stencil_pt) * (p->ns > 0 ? p->ns : 1));
    w->rp = (stencil_pt *)malloc(sizeof(stencil_pt) * (p->nr > 0 ? p->nr : 1));
    if (!w->m || !w->damp || !w->sp || !w->rp) return -2;
    for (int64_t i = 0; i < N; ++i) {
        if (!(p->v[i] > 0)) return -1;
        w->m[i] = 1.0 / (p->v[i] * p->v[i]);
    }
    damp_g(p, &w->g, w->damp);
    for (int s = 0; s < p->ns; ++s)
        if (set_stencil(p, &w->g, p->src, p->spos, p->ssinc, s, &w->sp[s])) return -3;
    for (int r = 0; r < p->nr; ++r)
        if (set_stencil(p, &w->g, p->rec, p->rpos, p->rsinc, r, &w->rp[r])) return -3;
    return 0;
}

static void work_free(work *w)
{
    free(w->m);
    free(w->damp);
    free(w->sp);
    free(w->rp);
}

/*
 * Forward sweep.  u_cur/u_prev hold (u^0, u^{-1}) on entry and (u^nt, u^{nt-1})
 * on return.  amp: [nt][ns] source samples w (may be NULL: no source).
 * rec_out: [nt][nr] (may be NULL).  hist: optional [(nt+2)][N] copy of
 * u^{-1}, u^0, u^1, ..., u^nt.
 */
int or_forward(const or_problem *p, const double *amp, double *rec_out,
               double *u_cur, double *u_prev, double *hist)
{
    work w;
    int rc = work_init(p, &w);
    if (rc) { work_free(&w); return rc; }
    int64_t N = w.g.npts;
    double *u_new = (double *)malloc(sizeof(double) * N);
    if (!u_new) { work_free(&w); return -2; }
    double dt2 = p->dt * p->dt;
    if (hist) {
        memcpy(hist, u_prev, sizeof(double) * N);
        memcpy(hist + N, u_cur, sizeof(double) * N);
    }
    for (int64_t n = 0; n < p->nt; ++n) {
        leapfrog_step(&w.g, w.c, w.M, p->dt, w.m, w.damp, u_cur, u_prev, u_new);
        if (amp)
            for (int s = 0; s < p->ns; ++s)
                spread(&w.sp[s], 2.0 * dt2 * amp[n * p->ns + s], p->dt, w.m, w.damp, u_new);
        if (rec_out)
            for (int r = 0; r < p->nr; ++r) rec_out[n * p->nr + r] = sample(&w.rp[r], u_new);
        /* rotate: prev <- cur, cur <- new */
        memcpy(u_prev, u_cur, sizeof(double) * N);
        memcpy(u_cur, u_new, sizeof(double) * N);
        if (hist) memcpy(hist + (n + 2) * N, u_cur, sizeof(double) * N);
    }
    free(u_new);
    work_free(&w);
    return 0;
}

/*
 * Adjoint sweep: y [nt][nr] is injected at the receivers, the result is read
 * at the sources: src_out[k-1][s] = 2 dt^2 lambda^k(s).  lam_hist (optional):
 * [(nt+2)][N] holding lambda^{nt+2}, lambda^{nt+1}, lambda^{nt}, ..., lambda^1
 * in that order (entry j = lambda^{nt+2-j}).
 */
static int adjoint_w(const or_problem *p, work *w, const double *y, double *src_out,
                     double *lam_hist, const double *uhist, double *gm)
{
    int64_t N = w->g.npts;
    double *l1 = (double *)calloc(N, sizeof(double)); /* lambda^{k+1} */
    double *l2 = (double *)calloc(N, sizeof(double)); /* lambda^{k+2} */
    double *l0 = (double *)malloc(sizeof(double) * N);
    if (!l1 || !l2 || !l0) { free(l1); free(l2); free(l0); return -2; }
    double dt2 = p->dt * p->dt;
    if (lam_hist) {
        memset(lam_hist, 0, sizeof(double) * 2 * N);
    }
    if (gm) memset(gm, 0, sizeof(double) * N);
    for (int64_t k = p->nt; k >= 1; --k) {
        leapfrog_step(&w->g, w->c, w->M, p->dt, w->m, w->damp, l1, l2, l0);
        for (int r = 0; r < p->nr; ++r) spread(&w->rp[r], y[(k - 1) * p->nr + r], p->dt, w->m, w->damp, l0);
        if (src_out)
            for (int s = 0; s < p->ns; ++s) src_out[(k - 1) * p->ns + s] = 2.0 * dt2 * sample(&w->sp[s], l0);
        if (lam_hist) memcpy(lam_hist + (p->nt + 2 - k) * N, l0, sizeof(double) * N);
        if (gm && uhist) {
            /* uhist entry j holds u^{j-1}: u^k at j = k+1 */
            const double *uk = uhist + (k + 1) * N, *uk1 = uhist + k * N, *uk2 = uhist + (k - 1) * N;
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < N; ++i)
                gm[i] += -2.0 * l0[i] * (uk[i] - 2.0 * uk1[i] + uk2[i]);
        }
        double *t = l2;
        l2 = l1;
        l1 = l0;
        l0 = t;
    }
    free(l0);
    free(l1);
    free(l2);
    return 0;
}

int or_adjoint(const or_problem *p, const double *y, double *src_out, double *lam_hist)
{
    work w;
    int rc = work_init(p, &w);
    if (!rc) rc = adjoint_w(p, &w, y, src_out, lam_hist, NULL, NULL);
    work_free(&w);
    return rc;
}

/*
 * Vector-Jacobian product of the map v -> d (receiver traces) for a given
 * trace cotangent y [nt][nr], zero initial state and source samples amp:
 * grad_m = -2 sum_k lambda^k (u^k - 2u^{k-1} + u^{k-2}), grad_v = grad_m * (-2/v^3).
 * Either output may be NULL.  Full time history is kept (no checkpointing).
 */
int or_vjp(const or_problem *p, const double *amp, const double *y, double *grad_v, double *grad_m)
{
    geom g;
    if (make_geom(p, &g)) return -1;
    int64_t N = g.npts;
    double *hist = (double *)malloc(sizeof(double) * N * (p->nt + 2));
    double *uc = (double *)calloc(N, sizeof(double));
    double *up = (double *)calloc(N, sizeof(double));
    double *gm = (double *)malloc(sizeof(double) * N);
    int rc = -2;
    if (hist && uc && up && gm) {
        rc = or_forward(p, amp, NULL, uc, up, hist);
        if (!rc) {
            work w;
            rc = work_init(p, &w);
            if (!rc) rc = adjoint_w(p, &w, y, NULL, NULL, hist, gm);
            work_free(&w);
        }
        if (!rc)
            for (int64_t i = 0; i < N; ++i) {
                if (grad_m) grad_m[i] = gm[i];
                if (grad_v) grad_v[i] = gm[i] * (-2.0 / (p->v[i] * p->v[i] * p->v[i]));
            }
    }
    free(hist);
    free(uc);
    free(up);
    free(gm);
    return rc;
}

/*
 * Born modelling: traces dd [nt][nr] of the perturbation wavefield for a
 * velocity perturbation dv (N^d), zero initial state, source samples amp.
 * The background and the perturbation advance together, step by step.
 */
int or_born(const or_problem *p, const double *amp, const double *dv, double *dd)
{
    work w;
    int rc = work_init(p, &w);
    if (rc) { work_free(&w); return rc; }
    int64_t N = w.g.npts;
    double *u[3], *du[3];
    for (int i = 0; i < 3; ++i) {
        u[i] = (double *)calloc(N, sizeof(double));
        du[i] = (double *)calloc(N, sizeof(double));
    }
    double *dm = (double *)malloc(sizeof(double) * N);
    if (!u[0] || !u[1] || !u[2] || !du[0] || !du[1] || !du[2] || !dm) rc = -2;
    if (!rc) {
        for (int64_t i = 0; i < N; ++i) dm[i] = -2.0 * dv[i] / (p->v[i] * p->v[i] * p->v[i]);
        double dt2 = p->dt * p->dt;
        /* u[0] = u^{k-2}, u[1] = u^{k-1}, u[2] <- u^k; du alike */
        for (int64_t n = 0; n < p->nt; ++n) {
            leapfrog_step(&w.g, w.c, w.M, p->dt, w.m, w.damp, u[1], u[0], u[2]);
            if (amp)
                for (int s = 0; s < p->ns; ++s) {
                    double a = 2.0 * dt2 * amp[n * p->ns + s];
                    spread(&w.sp[s], a, p->dt, w.m, w.damp, u[2]);
                }
            leapfrog_step(&w.g, w.c, w.M, p->dt, w.m, w.damp, du[1], du[0], du[2]);
            for (int64_t i = 0; i < N; ++i)
                du[2][i] += -2.0 * dm[i] * (u[2][i] - 2.0 * u[1][i] + u[0][i])
                            / (p->dt * w.damp[i] + 2.0 * w.m[i]);
            if (dd)
                for (int r = 0; r < p->nr; ++r) dd[n * p->nr + r] = sample(&w.rp[r], du[2]);
            double *t = u[0]; u[0] = u[1]; u[1] = u[2]; u[2] = t;
            t = du[0]; du[0] = du[1]; du[1] = du[2]; du[2] = t;
        }
    }
    for (int i = 0; i < 3; ++i) { free(u[i]); free(du[i]); }
    free(dm);
    work_free(&w);
    return rc;
}

/* Least-squares misfit J = 1/2 sum (d - d_obs)^2 and its gradient w.r.t. v. */
int or_gradient(const or_problem *p, const double *amp, const double *d_obs,
                double *grad_v, double *grad_m, double *misfit)
{
    int64_t N = 1;
    for (int a = 0; a < p->ndim; ++a) N *= p->n[a];
    double *uc = (double *)calloc(N, sizeof(double));
    double *up = (double *)calloc(N, sizeof(double));
    int64_t nd = p->nt * (int64_t)p->nr;
    double *d = (double *)malloc(sizeof(double) * (nd > 0 ? nd : 1));
    int rc = -2;
    if (!uc || !up || !d) goto done;
    rc = or_forward(p, amp, d, uc, up, NULL);
    if (rc) goto done;
    double J = 0.0;
    for (int64_t i = 0; i < nd; ++i) {
        d[i] -= d_obs[i];
        J += 0.5 * d[i] * d[i];
    }
    if (misfit) *misfit = J;
    rc = or_vjp(p, amp, d, grad_v, grad_m);
done:
    free(uc);
    free(up);
    free(d);
    return rc;
}
