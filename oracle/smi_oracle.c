/*
 * smi_oracle.c -- plain FP64 CPU reference of the SMIwiz modelling / imaging path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load this library.  It shares no code, header, table or
 * generator with the HIP path; it is written to be read against the paper:
 *
 *   Sec. 2.1, eq. (1)      first-order acoustic system, kappa = rho * Vp^2
 *   Sec. 2.1, eq. (2)-(3)  staggered leap-frog (p at integer, v at half points/steps)
 *   Sec. 2.1, eq. (4)      2N-order staggered first derivatives
 *   Sec. 2.1, eq. (5)      CFL condition (checked by the Python wrapper)
 *   Sec. 2.1 (last para.)  convolutional PML (Komatitsch & Martin 2007)
 *   Sec. 2.2, eq. (6)-(8)  L2 misfit, kappa gradient, adjoint system run by the same solver
 *   Sec. 2.3, eq. (10)     zero-lag cross-correlation image
 *   Alg. 2                 order of forward loop, adjoint source, reverse loop
 *   Sec. 4.1               evolving computing box
 *   Sec. 4.2               source-field reconstruction from saved boundaries
 *
 * Every array is double.  The padded grid is M[a] = n[a] + 2 nb along each active
 * axis; index (i1, i2, i3) -> i1 + M1*(i2 + M2*i3), i1 = z fastest.  v_a[i] sits half a
 * cell after node i along axis a.  A read outside the padded grid returns 0.
 * Loops are plain, unfused and unblocked; OpenMP only splits the outer loops.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OG_MAXN 8

typedef struct {
    int ndim;            /* 2 or 3 */
    int n1, n2, n3;      /* interior cells along z, x, y (n3 = 1 in 2D) */
    double d1, d2, d3;   /* spacing [m] */
    int nb;              /* absorbing layers per side */
    int order;           /* 2N: 2, 4, ..., 16 */
    int nt;              /* time steps */
    double dt;           /* step [s] */
    double fm;           /* centre frequency [Hz] (CPML alpha) */
    double vmax;         /* speed used by the CPML damping and the computing box */
    int pml;             /* 1: CPML, 0: no absorption (Dirichlet outside the padded grid) */
    int box;             /* 1: evolving computing box */
    int margin;          /* box margin in cells */
    int dr;              /* boundary decimation ratio */
    int band_p, band_v;  /* saved planes per face for p and the face-normal v (0: N) */
    int freesurf;        /* 1: free surface on the first interior row (no absorbing layer above) */
} og_grid;

typedef struct {
    og_grid g;
    int N;               /* half order */
    int nd;              /* active axes */
    int n[3], M[3];
    double d[3];
    size_t P;            /* padded cells */
    double c[3][OG_MAXN];/* a_l / d_a */
    double dV;
    double *kap, *bet[3];
    double *cpa_i[3], *cpb_i[3], *cpa_h[3], *cpb_h[3];
    int bp, bv;
} og_model;

typedef struct {
    double *p, *v[3], *psp[3], *psv[3];
} og_field;

/* Point operators of sources and receivers at positions off the grid (Sec. 2.1, Kaiser-
 * windowed sinc of Hicks): point i acts on the padded nodes idx[3t..3t+2] with weights w[t],
 * t in off[i] .. off[i+1].  A NULL operator means "the node given with the point".          */
typedef struct {
    int n;
    const int *off;
    const int *idx;
    const double *w;
} og_taps;

/* ------------------------------------------------------------------ coefficients */

/* Staggered first-derivative weights of order 2N (eq. 4): the unique a_l that make
 * sum_l a_l (f(+(2l-1)/2) - f(-(2l-1)/2)) exact for every polynomial of degree <= 2N-1.
 * Closed form of the Vandermonde solution:
 *   a_l = (-1)^(l+1)/(2l-1) * prod_{m!=l} (2m-1)^2 / |(2m-1)^2 - (2l-1)^2|            */
int og_fd_coef(int order, double *a)
{
    if (order < 2 || order > 2 * OG_MAXN || order % 2) return -1;
    int N = order / 2;
    for (int l = 1; l <= N; l++) {
        double prod = 1.0;
        double kl = (2.0 * l - 1.0) * (2.0 * l - 1.0);
        for (int m = 1; m <= N; m++) {
            if (m == l) continue;
            double km = (2.0 * m - 1.0) * (2.0 * m - 1.0);
            prod *= km / fabs(km - kl);
        }
        a[l - 1] = ((l % 2) ? 1.0 : -1.0) / (2.0 * l - 1.0) * prod;
    }
    return 0;
}

/* ------------------------------------------------------------------ CPML profiles */

/* Convolutional PML of Komatitsch & Martin (2007) with kappa_pml = 1:
 *   psi <- b psi + a * (du/dx),   filtered derivative = du/dx + psi
 *   b = exp(-(d + alpha) dt),     a = d (b - 1) / (d + alpha)     (a = 0 where d = 0)
 * d = d0 l^2 with l the normalised depth into the layer at the node, d0 from the target
 * reflection R of Collino & Tsogka, alpha = pi fm (1 - l).                           */
int og_cpml_profile(const og_grid *g, int axis, int half, double *cpa, double *cpb)
{
    int n = axis == 0 ? g->n1 : axis == 1 ? g->n2 : g->n3;
    double d = axis == 0 ? g->d1 : axis == 1 ? g->d2 : g->d3;
    int nb = g->nb, M = n + 2 * nb;
    double R = pow(10.0, -((log10((double)nb) - 1.0) / log10(2.0) + 3.0));
    double d0 = -3.0 * g->vmax * log(R) / (2.0 * nb * d);
    for (int i = 0; i < M; i++) {
        double x = i + (half ? 0.5 : 0.0);
        double dist = 0.0;
        if (x < nb) dist = g->freesurf && axis == 0 ? 0.0 : nb - x;   /* no layer above a free surface */
        else if (x > nb + n - 1) dist = x - (nb + n - 1);
        double l = dist / nb;
        double damp = d0 * l * l;
        double alpha = M_PI * g->fm * (1.0 - l);
        if (!g->pml || dist <= 0.0) {
            cpa[i] = 0.0;
            cpb[i] = g->pml ? exp(-alpha * g->dt) : 1.0;
        } else {
            cpb[i] = exp(-(damp + alpha) * g->dt);
            cpa[i] = damp * (cpb[i] - 1.0) / (damp + alpha);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ model */

static inline size_t IDX(const og_model *m, int i1, int i2, int i3)
{
    return (size_t)i1 + (size_t)m->M[0] * ((size_t)i2 + (size_t)m->M[1] * (size_t)i3);
}

static void og_free_model(og_model *m)
{
    free(m->kap);
    for (int a = 0; a < 3; a++) {
        free(m->bet[a]); free(m->cpa_i[a]); free(m->cpb_i[a]); free(m->cpa_h[a]); free(m->cpb_h[a]);
    }
    memset(m, 0, sizeof(*m));
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Pad vp and rho into the absorbing layers by edge replication, then
 * kappa = rho vp^2 (eq. 1) and the staggered buoyancy beta_a(i+1/2) = 2/(rho_i+rho_{i+1})
 * (arithmetic mean of rho; rho beyond the last node repeats the last node).           */
static int og_setup(og_model *m, const og_grid *g, const double *vp, const double *rho)
{
    memset(m, 0, sizeof(*m));
    if (g->ndim != 2 && g->ndim != 3) return -1;
    if (g->order < 2 || g->order > 2 * OG_MAXN || g->order % 2) return -1;
    m->g = *g;
    m->N = g->order / 2;
    m->nd = g->ndim;
    m->n[0] = g->n1; m->n[1] = g->n2; m->n[2] = g->ndim == 3 ? g->n3 : 1;
    m->d[0] = g->d1; m->d[1] = g->d2; m->d[2] = g->ndim == 3 ? g->d3 : 1.0;
    for (int a = 0; a < 3; a++) m->M[a] = a < m->nd ? m->n[a] + 2 * g->nb : 1;
    m->P = (size_t)m->M[0] * m->M[1] * m->M[2];
    m->dV = m->d[0] * m->d[1] * (m->nd == 3 ? m->d[2] : 1.0);
    m->bp = g->band_p > 0 ? g->band_p : m->N;
    m->bv = g->band_v > 0 ? g->band_v : m->N;
    double al[OG_MAXN];
    og_fd_coef(g->order, al);
    for (int a = 0; a < 3; a++)
        for (int l = 0; l < m->N; l++) m->c[a][l] = al[l] / m->d[a];

    double *rp = malloc(m->P * sizeof(double));
    m->kap = malloc(m->P * sizeof(double));
    for (int a = 0; a < 3; a++) m->bet[a] = malloc(m->P * sizeof(double));
    int nb = g->nb;
    for (int i3 = 0; i3 < m->M[2]; i3++)
        for (int i2 = 0; i2 < m->M[1]; i2++)
            for (int i1 = 0; i1 < m->M[0]; i1++) {
                int j1 = clampi(i1 - nb, 0, m->n[0] - 1);
                int j2 = clampi(i2 - nb, 0, m->n[1] - 1);
                int j3 = m->nd == 3 ? clampi(i3 - nb, 0, m->n[2] - 1) : 0;
                size_t s = (size_t)j1 + (size_t)m->n[0] * ((size_t)j2 + (size_t)m->n[1] * j3);
                size_t k = IDX(m, i1, i2, i3);
                rp[k] = rho[s];
                m->kap[k] = rho[s] * vp[s] * vp[s];
            }
    for (int a = 0; a < 3; a++)
        for (int i3 = 0; i3 < m->M[2]; i3++)
            for (int i2 = 0; i2 < m->M[1]; i2++)
                for (int i1 = 0; i1 < m->M[0]; i1++) {
                    int i[3] = {i1, i2, i3};
                    int j[3] = {i1, i2, i3};
                    if (a < m->nd) j[a] = clampi(i[a] + 1, 0, m->M[a] - 1);
                    size_t k = IDX(m, i1, i2, i3);
                    m->bet[a][k] = 2.0 / (rp[k] + rp[IDX(m, j[0], j[1], j[2])]);
                }
    free(rp);
    for (int a = 0; a < 3; a++) {
        int Ma = m->M[a];
        m->cpa_i[a] = calloc(Ma, sizeof(double)); m->cpb_i[a] = calloc(Ma, sizeof(double));
        m->cpa_h[a] = calloc(Ma, sizeof(double)); m->cpb_h[a] = calloc(Ma, sizeof(double));
        if (a < m->nd) {
            og_cpml_profile(g, a, 0, m->cpa_i[a], m->cpb_i[a]);
            og_cpml_profile(g, a, 1, m->cpa_h[a], m->cpb_h[a]);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ fields */

static void og_field_alloc(og_field *f, size_t P)
{
    f->p = calloc(P, sizeof(double));
    for (int a = 0; a < 3; a++) {
        f->v[a] = calloc(P, sizeof(double));
        f->psp[a] = calloc(P, sizeof(double));
        f->psv[a] = calloc(P, sizeof(double));
    }
}

static void og_field_free(og_field *f)
{
    free(f->p);
    for (int a = 0; a < 3; a++) { free(f->v[a]); free(f->psp[a]); free(f->psv[a]); }
}

/* f at point i of operator t (or at `node` when t is NULL) */
static double og_sample(const og_model *m, const double *f, const og_taps *t, int i, const int *node)
{
    if (!t) return f[IDX(m, node[0], node[1], node[2])];
    double s = 0.0;
    for (int q = t->off[i]; q < t->off[i + 1]; q++)
        s += t->w[q] * f[IDX(m, t->idx[3 * q], t->idx[3 * q + 1], t->idx[3 * q + 2])];
    return s;
}

/* f += amp * (operator weights of point i), scaled node-wise by `scale` when not NULL (the
 * transpose of og_sample, times the scale) */
static void og_spread(const og_model *m, double *f, const og_taps *t, int i, const int *node,
                      double amp, const double *scale)
{
    if (!t) {
        size_t k = IDX(m, node[0], node[1], node[2]);
        f[k] += amp * (scale ? scale[k] : 1.0);
        return;
    }
    for (int q = t->off[i]; q < t->off[i + 1]; q++) {
        size_t k = IDX(m, t->idx[3 * q], t->idx[3 * q + 1], t->idx[3 * q + 2]);
        f[k] += amp * t->w[q] * (scale ? scale[k] : 1.0);
    }
}

/* value of f at node i shifted by `off` along axis a; 0 outside the padded grid */
static inline double at(const og_model *m, const double *f, int i1, int i2, int i3, int a, int off)
{
    int j[3] = {i1, i2, i3};
    j[a] += off;
    if (j[a] < 0 || j[a] >= m->M[a]) return 0.0;
    return f[IDX(m, j[0], j[1], j[2])];
}

/* eq. (4), second row: d_a p at the v_a point i+1/2: sum_l a_l (p[i+l] - p[i-l+1]) / d_a */
static inline double dplus(const og_model *m, const double *p, int i1, int i2, int i3, int a)
{
    double s = 0.0;
    for (int l = 1; l <= m->N; l++)
        s += m->c[a][l - 1] * (at(m, p, i1, i2, i3, a, l) - at(m, p, i1, i2, i3, a, -(l - 1)));
    return s;
}

/* eq. (4), first row: d_a v_a at the p point i: sum_l a_l (v[i+l-1] - v[i-l]) / d_a
 * (v[j] stores v at j+1/2, so i+(2l-1)/2 -> j = i+l-1 and i-(2l-1)/2 -> j = i-l)      */
static inline double dminus(const og_model *m, const double *v, int i1, int i2, int i3, int a)
{
    double s = 0.0;
    for (int l = 1; l <= m->N; l++)
        s += m->c[a][l - 1] * (at(m, v, i1, i2, i3, a, l - 1) - at(m, v, i1, i2, i3, a, -l));
    return s;
}

static double divv(const og_model *m, const og_field *f, int i1, int i2, int i3)
{
    double s = 0.0;
    for (int a = 0; a < m->nd; a++) s += dminus(m, f->v[a], i1, i2, i3, a);
    return s;
}

/* One leap-frog step of eq. (3) with CPML on the region lo..hi (inclusive):
 * all v_a first (from p^n), then p (from v^{n+1/2}).                                 */
/* Free surface by the image method (Sec. 2.1, after Levander): the surface is the first
 * interior row z = nb; p is odd about it (zero on it), v_z (at half rows) even.  The rows
 * above the surface hold the mirror images, over the columns of [lo, hi].                */
static void og_fs_v(const og_model *m, og_field *f, const int *lo, const int *hi)
{
    int nb = m->g.nb;
    for (int i3 = lo[2]; i3 <= hi[2]; i3++)
        for (int i2 = lo[1]; i2 <= hi[1]; i2++)
            for (int k = 0; k < m->N; k++)
                f->v[0][IDX(m, nb - 1 - k, i2, i3)] = f->v[0][IDX(m, nb + k, i2, i3)];
}

static void og_fs_p(const og_model *m, double *p, const int *lo, const int *hi)
{
    int nb = m->g.nb;
    for (int i3 = lo[2]; i3 <= hi[2]; i3++)
        for (int i2 = lo[1]; i2 <= hi[1]; i2++) {
            p[IDX(m, nb, i2, i3)] = 0.0;
            for (int k = 1; k <= m->N; k++)
                p[IDX(m, nb - k, i2, i3)] = -p[IDX(m, nb + k, i2, i3)];
        }
}

static void og_step(const og_model *m, og_field *f, const int *lo, const int *hi)
{
    const double dt = m->g.dt;
    for (int a = 0; a < m->nd; a++) {
#pragma omp parallel for collapse(2) schedule(static)
        for (int i3 = lo[2]; i3 <= hi[2]; i3++)
            for (int i2 = lo[1]; i2 <= hi[1]; i2++)
                for (int i1 = lo[0]; i1 <= hi[0]; i1++) {
                    int ia = a == 0 ? i1 : a == 1 ? i2 : i3;
                    size_t k = IDX(m, i1, i2, i3);
                    double e = dplus(m, f->p, i1, i2, i3, a);
                    f->psp[a][k] = m->cpb_h[a][ia] * f->psp[a][k] + m->cpa_h[a][ia] * e;
                    f->v[a][k] -= dt * m->bet[a][k] * (e + f->psp[a][k]);
                }
    }
    if (m->g.freesurf) og_fs_v(m, f, lo, hi);
#pragma omp parallel for collapse(2) schedule(static)
    for (int i3 = lo[2]; i3 <= hi[2]; i3++)
        for (int i2 = lo[1]; i2 <= hi[1]; i2++)
            for (int i1 = lo[0]; i1 <= hi[0]; i1++) {
                size_t k = IDX(m, i1, i2, i3);
                double s = 0.0;
                for (int a = 0; a < m->nd; a++) {
                    int ia = a == 0 ? i1 : a == 1 ? i2 : i3;
                    double e = dminus(m, f->v[a], i1, i2, i3, a);
                    f->psv[a][k] = m->cpb_i[a][ia] * f->psv[a][k] + m->cpa_i[a][ia] * e;
                    s += e + f->psv[a][k];
                }
                f->p[k] -= dt * m->kap[k] * s;
            }
    if (m->g.freesurf) og_fs_p(m, f->p, lo, hi);
}

/* ------------------------------------------------------------------ computing box (Sec. 4.1) */

/* Forward box used by forward step `it` (which produces v^{it+1/2}, p^{it+1}): the
 * outermost wavefront after it+1 steps at the maximum speed, plus a margin, around the
 * source; clipped to the padded grid.                                                 */
static void og_fwd_box_m(const og_model *m, const int *src, int it, int *lo, int *hi)
{
    for (int a = 0; a < 3; a++) {
        if (a >= m->nd || !m->g.box) { lo[a] = 0; hi[a] = m->M[a] - 1; continue; }
        int r = (int)ceil(m->g.vmax * (it + 1) * m->g.dt / m->d[a]) + m->g.margin;
        lo[a] = src[a] - r < 0 ? 0 : src[a] - r;
        hi[a] = src[a] + r > m->M[a] - 1 ? m->M[a] - 1 : src[a] + r;
    }
}

/* Adjoint box used by reverse iteration `it`: the receivers' bounding box grown by the
 * distance travelled at the maximum speed since the end of the record, plus a margin. */
static void og_adj_box_m(const og_model *m, int nrec, const int *rec, int it, int *lo, int *hi)
{
    for (int a = 0; a < 3; a++) {
        if (a >= m->nd || !m->g.box || nrec == 0) { lo[a] = 0; hi[a] = m->M[a] - 1; continue; }
        int rmin = rec[a], rmax = rec[a];
        for (int r = 1; r < nrec; r++) {
            if (rec[3 * r + a] < rmin) rmin = rec[3 * r + a];
            if (rec[3 * r + a] > rmax) rmax = rec[3 * r + a];
        }
        int w = (int)ceil(m->g.vmax * (m->g.nt - it) * m->g.dt / m->d[a]) + m->g.margin;
        lo[a] = rmin - w < 0 ? 0 : rmin - w;
        hi[a] = rmax + w > m->M[a] - 1 ? m->M[a] - 1 : rmax + w;
    }
}

int og_fwd_box(const og_grid *g, const int *src, int it, int *lo, int *hi)
{
    og_model m;
    memset(&m, 0, sizeof(m));
    m.g = *g; m.nd = g->ndim;
    m.n[0] = g->n1; m.n[1] = g->n2; m.n[2] = g->ndim == 3 ? g->n3 : 1;
    m.d[0] = g->d1; m.d[1] = g->d2; m.d[2] = g->d3;
    for (int a = 0; a < 3; a++) m.M[a] = a < m.nd ? m.n[a] + 2 * g->nb : 1;
    og_fwd_box_m(&m, src, it, lo, hi);
    return 0;
}

/* ------------------------------------------------------------------ saved boundaries (Sec. 4.2) */

/* Bands saved per face of axis a: band_p planes of p and band_v planes of the face-normal
 * v_a just outside the interior, over the interior extent of the other axes:
 *   p   : [nb-bp, nb)  and [nb+n_a, nb+n_a+bp)
 *   v_a : [nb-bv, nb)  and [nb+n_a-1, nb+n_a-1+bv)
 * Layout of one saved level: for a = 0..nd-1: p left, p right, v_a left, v_a right.   */
static size_t og_plane(const og_model *m, int a)
{
    size_t s = 1;
    for (int b = 0; b < m->nd; b++) if (b != a) s *= (size_t)m->n[b];
    return s;
}

size_t og_band_size(const og_grid *g)
{
    og_model m;
    memset(&m, 0, sizeof(m));
    m.nd = g->ndim;
    m.n[0] = g->n1; m.n[1] = g->n2; m.n[2] = g->ndim == 3 ? g->n3 : 1;
    int N = g->order / 2;
    int bp = g->band_p > 0 ? g->band_p : N, bv = g->band_v > 0 ? g->band_v : N;
    size_t s = 0;
    for (int a = 0; a < m.nd; a++) s += 2 * (size_t)(bp + bv) * og_plane(&m, a);
    return s;
}

/* Saved band levels.  dr = 1: every level 0..nt-1.  dr > 1: the levels k dr for
 * k = 0 .. (nt-1)/dr + OG_TAPS, so that the time interpolator below finds all of its taps for
 * every level 0..nt-1 (the forward pass continues past nt, source off, to save the last
 * ones).                                                                               */
#define OG_TAPS 4          /* half-width, in saved levels, of the band interpolator */
#define OG_KAISER_BETA 6.31

size_t og_band_levels(const og_grid *g)
{
    return g->dr == 1 ? (size_t)g->nt : (size_t)((g->nt - 1) / g->dr + OG_TAPS + 1);
}

static double og_bessel_i0(double x)
{
    double s = 1.0, t = 1.0;
    for (int k = 1; k < 60; k++) {
        t *= (x / (2.0 * k)) * (x / (2.0 * k));
        s += t;
        if (t < 1e-17 * s) break;
    }
    return s;
}

/* Kaiser-windowed sinc weight of a sample at distance u (in saved levels), half-width R */
static double og_ksinc(double u)
{
    if (fabs(u) >= OG_TAPS) return 0.0;
    double x = u / OG_TAPS;
    double win = og_bessel_i0(OG_KAISER_BETA * sqrt(1.0 - x * x)) / og_bessel_i0(OG_KAISER_BETA);
    double sc = u == 0.0 ? 1.0 : sin(M_PI * u) / (M_PI * u);
    return sc * win;
}

/* copy planes [start, start+w) along axis a (interior extent elsewhere) between the field
 * and buf; dir = 0: field -> buf, 1: buf -> field, 2: field <- (1-wt)*buf + wt*buf2   */
static size_t og_block(const og_model *m, double *fld, int a, int start, int w, double *buf,
                       const double *buf2, double wt, int dir)
{
    int lo[3], hi[3];
    int nb = m->g.nb;
    for (int b = 0; b < 3; b++) {
        if (b >= m->nd) { lo[b] = 0; hi[b] = 0; }
        else if (b == a) { lo[b] = start; hi[b] = start + w - 1; }
        else { lo[b] = nb; hi[b] = nb + m->n[b] - 1; }
    }
    size_t q = 0;
    for (int i3 = lo[2]; i3 <= hi[2]; i3++)
        for (int i2 = lo[1]; i2 <= hi[1]; i2++)
            for (int i1 = lo[0]; i1 <= hi[0]; i1++, q++) {
                size_t k = IDX(m, i1, i2, i3);
                if (dir == 0) buf[q] = fld[k];
                else if (dir == 1) fld[k] = buf[q];
                else fld[k] = (1.0 - wt) * buf[q] + wt * buf2[q];
            }
    return q;
}

/* which = 0: p bands, 1: v bands, 2: both */
static void og_bands(const og_model *m, og_field *f, double *buf, const double *buf2, double wt,
                     int dir, int which)
{
    int nb = m->g.nb, bp = m->bp, bv = m->bv;
    size_t q = 0;
    for (int a = 0; a < m->nd; a++) {
        size_t pl = og_plane(m, a);
        int n = m->n[a];
        if (which != 1) {
            og_block(m, f->p, a, nb - bp, bp, buf + q, buf2 ? buf2 + q : NULL, wt, dir);
            og_block(m, f->p, a, nb + n, bp, buf + q + bp * pl, buf2 ? buf2 + q + bp * pl : NULL, wt, dir);
        }
        q += 2 * bp * pl;
        if (which != 0) {
            og_block(m, f->v[a], a, nb - bv, bv, buf + q, buf2 ? buf2 + q : NULL, wt, dir);
            og_block(m, f->v[a], a, nb + n - 1, bv, buf + q + bv * pl, buf2 ? buf2 + q + bv * pl : NULL, wt, dir);
        }
        q += 2 * bv * pl;
    }
}

/* ------------------------------------------------------------------ state copies */

static void og_state_get(const og_model *m, const og_field *f, double *dst)
{
    memcpy(dst, f->p, m->P * sizeof(double));
    for (int a = 0; a < 3; a++) memcpy(dst + (a + 1) * m->P, f->v[a], m->P * sizeof(double));
}

static void og_state_set(const og_model *m, og_field *f, const double *src)
{
    memcpy(f->p, src, m->P * sizeof(double));
    for (int a = 0; a < 3; a++) memcpy(f->v[a], src + (a + 1) * m->P, m->P * sizeof(double));
}

static void og_snap(const og_model *m, const double *p, double *dst)
{
    int nb = m->g.nb;
    size_t q = 0;
    for (int i3 = 0; i3 < m->n[2]; i3++)
        for (int i2 = 0; i2 < m->n[1]; i2++)
            for (int i1 = 0; i1 < m->n[0]; i1++)
                dst[q++] = p[IDX(m, i1 + nb, i2 + nb, m->nd == 3 ? i3 + nb : 0)];
}

static void og_take_snaps(const og_model *m, const double *p, int level, int nsnap,
                          const int *snap_it, double *snaps)
{
    size_t I = (size_t)m->n[0] * m->n[1] * m->n[2];
    for (int k = 0; k < nsnap; k++)
        if (snap_it[k] == level) og_snap(m, p, snaps + (size_t)k * I);
}

/* ------------------------------------------------------------------ forward (Alg. 2, forward loop) */

/* One shot.  src: padded node (i1,i2,i3); rec: nrec padded nodes; stf[nt].
 * Per step it: [save bands of (p^it, v^{it-1/2}) if it % dr == 0], v then p update (eq. 3)
 * with CPML, p[src] += dt stf[it] / dV (the explosive source f_p of eq. 1 as a cell
 * average), dcal[it][r] = p^{it+1}[rec_r].
 * Optional: init (4P: p, v1, v2, v3 at level 0), hist ((nt+1) x 4P: every (p^n, v^{n-1/2})),
 * bands (og_band_levels x og_band_size), final (4P at level nt), snaps of interior p. */
int og_forward(const og_grid *g, const double *vp, const double *rho, const int *src,
               const double *stf, int nrec, const int *rec, double *dcal, const double *init,
               double *hist, double *bands, double *final_state, int nsnap, const int *snap_it,
               double *snaps, const og_taps *st, const og_taps *rt)
{
    og_model m;
    if (og_setup(&m, g, vp, rho)) return -1;
    og_field f;
    og_field_alloc(&f, m.P);
    if (init) og_state_set(&m, &f, init);
    size_t B = og_band_size(g);
    /* with decimated bands the loop continues (source off, nothing recorded) until the last
     * saved level the interpolator needs */
    int last = g->nt;
    if (bands && g->dr > 1) last = (int)(og_band_levels(g) - 1) * g->dr;
    og_take_snaps(&m, f.p, 0, nsnap, snap_it, snaps);
    for (int it = 0; it <= last; it++) {
        if (hist && it <= g->nt) og_state_get(&m, &f, hist + (size_t)it * 4 * m.P);
        if (it == g->nt && final_state) og_state_get(&m, &f, final_state);
        if (bands && it % g->dr == 0 && (size_t)(it / g->dr) < og_band_levels(g))
            og_bands(&m, &f, bands + (size_t)(it / g->dr) * B, NULL, 0.0, 0, 2);
        if (it == last) break;
        int lo[3], hi[3];
        og_fwd_box_m(&m, src, it, lo, hi);
        og_step(&m, &f, lo, hi);
        if (it < g->nt) {
            og_spread(&m, f.p, st, 0, src, g->dt * stf[it] / m.dV, NULL);
            if (g->freesurf) og_fs_p(&m, f.p, lo, hi);
            for (int r = 0; r < nrec; r++)
                dcal[(size_t)it * nrec + r] = og_sample(&m, f.p, rt, r, rec + 3 * r);
            og_take_snaps(&m, f.p, it + 1, nsnap, snap_it, snaps);
        }
    }
    og_field_free(&f);
    og_free_model(&m);
    return 0;
}

/* ------------------------------------------------------------------ reconstruction (Sec. 4.2) */

/* Restore bands at level `it` (p^it and v^{it-1/2}).  dr = 1: a copy of the saved level.
 * dr > 1 (Sec. 4.2 interpolates decimated boundaries without naming the kernel): a
 * Kaiser-windowed sinc in time over the 2 OG_TAPS saved levels around `it`, weights
 * normalised to sum 1; levels before 0 are exactly zero (the field starts at rest).      */
static void og_restore(const og_model *m, og_field *f, const double *bands, int it, int which)
{
    size_t B = og_band_size(&m->g);
    int dr = m->g.dr;
    int k0 = it / dr;
    if (it % dr == 0) { og_bands(m, f, (double *)(bands + (size_t)k0 * B), NULL, 0.0, 1, which); return; }
    double u = (double)it / dr, wsum = 0.0;
    double *tmp = calloc(B, sizeof(double));
    for (int k = k0 - OG_TAPS + 1; k <= k0 + OG_TAPS; k++) {
        double w = og_ksinc(u - k);
        wsum += w;
        if (k < 0) continue;
        const double *b = bands + (size_t)k * B;
        for (size_t q = 0; q < B; q++) tmp[q] += w * b[q];
    }
    for (size_t q = 0; q < B; q++) tmp[q] /= wsum;
    og_bands(m, f, tmp, NULL, 0.0, 1, which);
    free(tmp);
}

/* One reverse iteration (Alg. 2 reverse loop, source-field part), from (p^{it+1}, v^{it+1/2})
 * to (p^it, v^{it-1/2}) on the interior, the inverse of one forward step there:
 *   p[src] -= dt stf[it]/dV;  p^it = p^{it+1} + dt kappa div v^{it+1/2};  restore p band;
 *   v_a^{it-1/2} = v_a^{it+1/2} + dt beta_a d_a p^it;                      restore v bands. */
static void og_recon_iter(const og_model *m, og_field *f, const int *src, const double *stf,
                          const double *bands, int it, const og_taps *st)
{
    const double dt = m->g.dt;
    int nb = m->g.nb;
    og_spread(m, f->p, st, 0, src, -dt * stf[it] / m->dV, NULL);
    int blo[3], bhi[3];
    og_fwd_box_m(m, src, it, blo, bhi);
    int lo[3], hi[3];
    for (int a = 0; a < 3; a++) {
        if (a >= m->nd) { lo[a] = hi[a] = 0; continue; }
        lo[a] = blo[a] > nb ? blo[a] : nb;
        hi[a] = bhi[a] < nb + m->n[a] - 1 ? bhi[a] : nb + m->n[a] - 1;
    }
#pragma omp parallel for collapse(2) schedule(static)
    for (int i3 = lo[2]; i3 <= hi[2]; i3++)
        for (int i2 = lo[1]; i2 <= hi[1]; i2++)
            for (int i1 = lo[0]; i1 <= hi[0]; i1++) {
                size_t k = IDX(m, i1, i2, i3);
                f->p[k] += dt * m->kap[k] * divv(m, f, i1, i2, i3);
            }
    if (m->g.freesurf && lo[0] == nb)   /* p^it vanishes on the surface */
        for (int i3 = lo[2]; i3 <= hi[2]; i3++)
            for (int i2 = lo[1]; i2 <= hi[1]; i2++) f->p[IDX(m, nb, i2, i3)] = 0.0;
    og_restore(m, f, bands, it, 0);
    for (int a = 0; a < m->nd; a++) {
        int vhi[3] = {hi[0], hi[1], hi[2]};
        if (vhi[a] > nb + m->n[a] - 2) vhi[a] = nb + m->n[a] - 2;
#pragma omp parallel for collapse(2) schedule(static)
        for (int i3 = lo[2]; i3 <= vhi[2]; i3++)
            for (int i2 = lo[1]; i2 <= vhi[1]; i2++)
                for (int i1 = lo[0]; i1 <= vhi[0]; i1++) {
                    size_t k = IDX(m, i1, i2, i3);
                    f->v[a][k] += dt * m->bet[a][k] * dplus(m, f->p, i1, i2, i3, a);
                }
    }
    og_restore(m, f, bands, it, 1);
}

/* Rebuild the source field backwards in time from the final state and the saved bands;
 * snaps receive interior p at the requested levels 0..nt.                            */
int og_reconstruct(const og_grid *g, const double *vp, const double *rho, const int *src,
                   const double *stf, const double *bands, const double *final_state, int nsnap,
                   const int *snap_it, double *snaps, const og_taps *st)
{
    og_model m;
    if (og_setup(&m, g, vp, rho)) return -1;
    og_field f;
    og_field_alloc(&f, m.P);
    og_state_set(&m, &f, final_state);
    og_take_snaps(&m, f.p, g->nt, nsnap, snap_it, snaps);
    for (int it = g->nt - 1; it >= 0; it--) {
        og_recon_iter(&m, &f, src, stf, bands, it, st);
        og_take_snaps(&m, f.p, it, nsnap, snap_it, snaps);
    }
    og_field_free(&f);
    og_free_model(&m);
    return 0;
}

/* ------------------------------------------------------------------ adjoint, gradient, image */

/* Reverse loop of Alg. 2 for one shot.  The adjoint of eq. (8) is run by the same solver
 * (eq. 3 + CPML) in the scaled variables p~ = kappa pbar, v~ = -beta vbar, for which the
 * transpose of the interior leap-frog recursion is the recursion itself run backwards in
 * time.  Per reverse iteration it = nt-1..0:
 *   p~[rec_r] += kappa(rec_r) G[it][r]                     (adjoint source, eq. 8 "-kappa dd")
 *   gk += dt (p~/kappa) (-div v^{it+1/2})                  (eq. 7, kappa gradient)
 *   adjoint step (v~ then p~, CPML)  -> level it
 *   source field -> (p^it, v^{it-1/2})                     (stored history or Sec. 4.2)
 *   image += dt p~^it p^it,  illum += dt (p^it)^2          (eq. 10, source illumination)
 * G = dt (dcal - dobs) gives dJ/dkappa of eq. (6); G = dt dobs gives the RTM image.
 * hist != NULL: the plain definition (full forward history (nt+1) x 4P).
 * hist == NULL: reconstruction from bands + final_state.
 * gk, image, illum: interior arrays (accumulated into; any may be NULL).             */
/* The density part of eq. (7) in the discrete scheme: J depends on rho through kappa and
 * through the staggered buoyancy beta_a = 2/(rho_i + rho_{i+1}) of every v update.  With the
 * same-solver adjoint velocity v~ (v~ = -beta vbar), dJ/dbeta_f = (dt/beta_f) sum_it
 * v~^{it+1/2}_f (D+_a p^it)_f, and dbeta_f/drho = -beta_f^2/2 for either node of the face, so
 * a face adds -(dt/2) beta_f v~ D+p to each interior node it touches (kappa held fixed).  The
 * faces of an axis run from the one below the first interior node to the one above the last;
 * the source field there comes from the restored bands.                                     */
static void og_rho_faces(const og_model *m, const og_field *q, const og_field *f, double *grk)
{
    int nb = m->g.nb;
    double dt = m->g.dt;
    for (int a = 0; a < m->nd; a++) {
        int lo[3], hi[3];
        for (int b = 0; b < 3; b++) {
            if (b >= m->nd) { lo[b] = 0; hi[b] = 0; }
            else if (b == a) { lo[b] = nb - 1; hi[b] = nb + m->n[b] - 1; }
            else { lo[b] = nb; hi[b] = nb + m->n[b] - 1; }
        }
        for (int i3 = lo[2]; i3 <= hi[2]; i3++)
            for (int i2 = lo[1]; i2 <= hi[1]; i2++)
                for (int i1 = lo[0]; i1 <= hi[0]; i1++) {
                    size_t k = IDX(m, i1, i2, i3);
                    double c = -0.5 * dt * m->bet[a][k] * q->v[a][k] * dplus(m, f->p, i1, i2, i3, a);
                    int j[3] = {i1 - nb, i2 - nb, m->nd == 3 ? i3 - nb : 0};
                    for (int side = 0; side < 2; side++) {     /* left node, right node */
                        int jj[3] = {j[0], j[1], j[2]};
                        jj[a] += side;
                        if (jj[a] < 0 || jj[a] >= m->n[a]) continue;
                        grk[(size_t)jj[0] + (size_t)m->n[0] * ((size_t)jj[1] + (size_t)m->n[1] * jj[2])] += c;
                    }
                }
    }
}

/* g_kappa += dt (p~ / kappa) (-div v) over the interior (eq. 7, kappa part) */
static void og_grad_kappa(const og_model *m, const og_field *q, const og_field *f, double *gk)
{
    int nb = m->g.nb;
#pragma omp parallel for collapse(2) schedule(static)
    for (int i3 = 0; i3 < m->n[2]; i3++)
        for (int i2 = 0; i2 < m->n[1]; i2++)
            for (int i1 = 0; i1 < m->n[0]; i1++) {
                int j3 = m->nd == 3 ? i3 + nb : 0;
                size_t k = IDX(m, i1 + nb, i2 + nb, j3);
                size_t s = (size_t)i1 + (size_t)m->n[0] * ((size_t)i2 + (size_t)m->n[1] * i3);
                gk[s] += m->g.dt * (q->p[k] / m->kap[k]) * (-divv(m, f, i1 + nb, i2 + nb, j3));
            }
}

/* literal, bit 0: the kappa gradient is taken where Alg. 2 writes it, after both updates of
 * the iteration (p~ at level it before the next injection, with v^{it-1/2}) -- a variant kept
 * only to show that it differs from the exact pairing at receiver cells alone.
 * Bits 1 and 2 plant mistakes in the image, kept only so that a test can show the image pin
 * catches them: bit 1 pairs p^it with the adjoint field before its step (one level early),
 * bit 2 drops the factor dt. */
/* nsnap, snap_it, snaps (optional): the source-field p of the interior at the listed levels
 * as the reverse loop holds it (from the stored history, or rebuilt from the bands). */
int og_adjoint(const og_grid *g, const double *vp, const double *rho, const int *src,
               const double *stf, int nrec, const int *rec, const double *G, const double *hist,
               const double *bands, const double *final_state, double *gk, double *image,
               double *illum, double *grk, const og_taps *st, const og_taps *rt, int literal,
               int nsnap, const int *snap_it, double *snaps)
{
    og_model m;
    if (og_setup(&m, g, vp, rho)) return -1;
    og_field f, q;
    og_field_alloc(&f, m.P);
    og_field_alloc(&q, m.P);
    if (!hist) {
        if (!bands || !final_state) { og_field_free(&f); og_field_free(&q); og_free_model(&m); return -2; }
        og_state_set(&m, &f, final_state);
    }
    int nb = m.g.nb;
    if (!hist) og_take_snaps(&m, f.p, g->nt, nsnap, snap_it, snaps);
    double *qearly = (literal & 2) ? calloc(m.P, sizeof(double)) : NULL;
    const double wdt = (literal & 4) ? 1.0 : g->dt;
    for (int it = g->nt - 1; it >= 0; it--) {
        for (int r = 0; r < nrec; r++)
            og_spread(&m, q.p, rt, r, rec + 3 * r, G[(size_t)it * nrec + r], m.kap);
        if (g->freesurf) {          /* the injected values get their images too */
            int flo[3] = {0, 0, 0}, fhi[3] = {m.M[0] - 1, m.M[1] - 1, m.M[2] - 1};
            og_fs_p(&m, q.p, flo, fhi);
        }
        if (hist) og_state_set(&m, &f, hist + (size_t)(it + 1) * 4 * m.P); /* v^{it+1/2} */
        if (gk && !(literal & 1)) og_grad_kappa(&m, &q, &f, gk);
        if (qearly) memcpy(qearly, q.p, m.P * sizeof(double));
        int lo[3], hi[3];
        og_adj_box_m(&m, nrec, rec, it, lo, hi);
        og_step(&m, &q, lo, hi);
        if (hist) og_state_set(&m, &f, hist + (size_t)it * 4 * m.P);
        else og_recon_iter(&m, &f, src, stf, bands, it, st);
        if (gk && (literal & 1)) og_grad_kappa(&m, &q, &f, gk);
        og_take_snaps(&m, f.p, it, nsnap, snap_it, snaps);
        const double *qi = qearly ? qearly : q.p;
        if (image || illum) {
#pragma omp parallel for collapse(2) schedule(static)
            for (int i3 = 0; i3 < m.n[2]; i3++)
                for (int i2 = 0; i2 < m.n[1]; i2++)
                    for (int i1 = 0; i1 < m.n[0]; i1++) {
                        size_t k = IDX(&m, i1 + nb, i2 + nb, m.nd == 3 ? i3 + nb : 0);
                        size_t s = (size_t)i1 + (size_t)m.n[0] * ((size_t)i2 + (size_t)m.n[1] * i3);
                        if (image) image[s] += wdt * qi[k] * f.p[k];
                        if (illum) illum[s] += g->dt * f.p[k] * f.p[k];
                    }
        }
        /* q.v holds v~^{it+1/2} (the p update of og_step leaves it), f.p holds p^it */
        if (grk) og_rho_faces(&m, &q, &f, grk);
    }
    free(qearly);
    og_field_free(&f);
    og_field_free(&q);
    og_free_model(&m);
    return 0;
}

/* ------------------------------------------------------------------ tangent-linear (Born) */

/* Linearisation of the forward map with respect to kappa (interior dkappa, zero in the
 * absorbing layers): the perturbation field obeys the same step, plus the secondary
 * source -dt dkappa div v^{n+1/2} in its p update; ddata[it][r] = dp^{it+1}[rec_r].    */
int og_born(const og_grid *g, const double *vp, const double *rho, const int *src,
            const double *stf, int nrec, const int *rec, const double *dkap, double *ddata,
            const og_taps *st, const og_taps *rt)
{
    og_model m;
    if (og_setup(&m, g, vp, rho)) return -1;
    og_field f, df;
    og_field_alloc(&f, m.P);
    og_field_alloc(&df, m.P);
    int nb = m.g.nb;
    int lo[3] = {0, 0, 0}, hi[3] = {m.M[0] - 1, m.M[1] - 1, m.M[2] - 1};
    for (int it = 0; it < g->nt; it++) {
        og_step(&m, &f, lo, hi);
        og_step(&m, &df, lo, hi);
#pragma omp parallel for collapse(2) schedule(static)
        for (int i3 = 0; i3 < m.n[2]; i3++)
            for (int i2 = 0; i2 < m.n[1]; i2++)
                for (int i1 = 0; i1 < m.n[0]; i1++) {
                    int j3 = m.nd == 3 ? i3 + nb : 0;
                    size_t k = IDX(&m, i1 + nb, i2 + nb, j3);
                    size_t s = (size_t)i1 + (size_t)m.n[0] * ((size_t)i2 + (size_t)m.n[1] * i3);
                    df.p[k] -= g->dt * dkap[s] * divv(&m, &f, i1 + nb, i2 + nb, j3);
                }
        og_spread(&m, f.p, st, 0, src, g->dt * stf[it] / m.dV, NULL);
        if (g->freesurf) {
            og_fs_p(&m, f.p, lo, hi);
            og_fs_p(&m, df.p, lo, hi);
        }
        for (int r = 0; r < nrec; r++)
            ddata[(size_t)it * nrec + r] = og_sample(&m, df.p, rt, r, rec + 3 * r);
    }
    og_field_free(&f);
    og_field_free(&df);
    og_free_model(&m);
    return 0;
}

/* ------------------------------------------------------------------ the image as a transpose (eq. 10) */

/* The zero-lag cross-correlation image of eq. (10), paired as og_adjoint pairs it (the adjoint
 * pressure after its step of reverse iteration it, times the source pressure p^it), is the
 * exact transpose of a linear map from an interior model perturbation m to data.  That map is
 * the derivative, at eps = 0, of a forward run in which every step starts by scaling p on the
 * interior by (1 + eps dt kappa m): a reaction term kappa eps m p added to the right-hand side
 * of the pressure equation of eq. (1), taken explicitly at level n.
 *   lin = 0: that perturbed forward run, data[it][r] = p^{it+1} sampled at receiver r;
 *   lin = 1: its tangent: a second field u obeys the same step and, before each step,
 *            u.p += dt kappa m p^it (p^it the unperturbed source field); data = u.p^{it+1}.
 * Both run on the whole padded grid (no computing box).  With the absorbing layers off, the
 * same-solver adjoint step is the exact transpose of the forward step in the scaled adjoint
 * variables, so <lin(m), G> = <m, image(G)> to rounding: a one-level slip in the pairing, a
 * lost dt or a lost kappa in the image breaks the identity.                                    */
static void og_scale_interior(const og_model *m, double *p, const double *dm, double c,
                              const double *by)
{
    int nb = m->g.nb;
#pragma omp parallel for collapse(2) schedule(static)
    for (int i3 = 0; i3 < m->n[2]; i3++)
        for (int i2 = 0; i2 < m->n[1]; i2++)
            for (int i1 = 0; i1 < m->n[0]; i1++) {
                size_t k = IDX(m, i1 + nb, i2 + nb, m->nd == 3 ? i3 + nb : 0);
                size_t s = (size_t)i1 + (size_t)m->n[0] * ((size_t)i2 + (size_t)m->n[1] * i3);
                p[k] += c * m->g.dt * m->kap[k] * dm[s] * by[k];
            }
}

int og_react(const og_grid *g, const double *vp, const double *rho, const int *src,
             const double *stf, int nrec, const int *rec, const double *dm, double eps, int lin,
             double *data, const og_taps *st, const og_taps *rt)
{
    og_model m;
    if (og_setup(&m, g, vp, rho)) return -1;
    og_field f, u;
    og_field_alloc(&f, m.P);
    og_field_alloc(&u, m.P);
    int lo[3] = {0, 0, 0}, hi[3] = {m.M[0] - 1, m.M[1] - 1, m.M[2] - 1};
    for (int it = 0; it < g->nt; it++) {
        if (lin) og_scale_interior(&m, u.p, dm, 1.0, f.p);     /* u.p += dt kappa m p^it */
        else og_scale_interior(&m, f.p, dm, eps, f.p);         /* p *= 1 + eps dt kappa m */
        og_step(&m, &f, lo, hi);
        if (lin) og_step(&m, &u, lo, hi);
        og_spread(&m, f.p, st, 0, src, g->dt * stf[it] / m.dV, NULL);
        if (g->freesurf) {
            og_fs_p(&m, f.p, lo, hi);
            if (lin) og_fs_p(&m, u.p, lo, hi);
        }
        const double *rp = lin ? u.p : f.p;
        for (int r = 0; r < nrec; r++)
            data[(size_t)it * nrec + r] = og_sample(&m, rp, rt, r, rec + 3 * r);
    }
    og_field_free(&f);
    og_field_free(&u);
    og_free_model(&m);
    return 0;
}
