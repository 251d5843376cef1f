/*
 * stride_oracle.c -- plain FP64 CPU oracle for the acoustic FWI hot path.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product path.  It shares no
 * source with the HIP library.  Every loop below is the textbook form of the
 * scheme: no tiling, no fusion beyond what the update formula states.
 *
 * Scheme (paper Sec. 2.4, acoustic equation with constant density and no
 * attenuation; Sec. 2.2 adjoint-state gradient):
 *   u^{n+1} = a (2 u^n + k (L u^n + S^n)) - b u^{n-1},   n = 0 .. nt-2,
 *   u^0 = u^{-1} = 0,  k = dt^2 vp^2,  a = 1/(1 + eta dt/2),  b = (1 - eta dt/2) a,
 *   L u = sum_axes (c0 u + sum_j cj (u_{+j} + u_{-j})) / dx_axis^2,
 *   S^n = sum_s W_s^T s_s^n / (cell volume),   traces[r][n] = W_r u^n.
 * Adjoint (exact transpose of the above, with w = a k lambda):
 *   w^m = a (2 w^{m+1} + k L w^{m+1}) - b w^{m+2} + a k R^T g^m,  w^{nt} = w^{nt+1} = 0,
 *   dJ/dk  = sum_{n=0}^{nt-2} (w^{n+1}/k) (L u^n + S^n),
 *   dJ/dvp = P^T [ (2/vp) sum_n w^{n+1} (L u^n + S^n) ],  P = edge-replicating pad,
 *   dJ/ds_s^n = W_s w^{n+1} / (cell volume).
 */
#include "stride_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define R0_SPONGE 1e-3

typedef struct {
    int nd;
    long n[3];      /* physical */
    long np[3];     /* padded (axis 2 = 1 in 2D) */
    long st[3];     /* strides of the padded array */
    long N;         /* padded points */
    int r;          /* stencil radius */
    double c[6];
    double inv_dx2[3];
    double cellvol;
} geo_t;

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Central second-derivative weights: the unique weights of the (2r+1)-point
 * symmetric stencil exact on polynomials of degree <= 2r+1 (Taylor moment
 * conditions); written as the exact rationals. */
int oracle_fd_weights(int space_order, double *c)
{
    switch (space_order) {
    case 2:  c[0] = -2.0;             c[1] = 1.0; break;
    case 4:  c[0] = -5.0 / 2.0;       c[1] = 4.0 / 3.0; c[2] = -1.0 / 12.0; break;
    case 6:  c[0] = -49.0 / 18.0;     c[1] = 3.0 / 2.0; c[2] = -3.0 / 20.0; c[3] = 1.0 / 90.0; break;
    case 8:  c[0] = -205.0 / 72.0;    c[1] = 8.0 / 5.0; c[2] = -1.0 / 5.0; c[3] = 8.0 / 315.0;
             c[4] = -1.0 / 560.0; break;
    case 10: c[0] = -5269.0 / 1800.0; c[1] = 5.0 / 3.0; c[2] = -5.0 / 21.0; c[3] = 5.0 / 126.0;
             c[4] = -5.0 / 1008.0; c[5] = 1.0 / 3150.0; break;
    default: return -1;
    }
    return 0;
}

/* Centred first-derivative weights: the unique antisymmetric (2r+1)-point
 * stencil exact on polynomials of degree <= 2r; exact rationals. */
int oracle_fd1_weights(int space_order, double *d)
{
    switch (space_order) {
    case 2:  d[1] = 1.0 / 2.0; break;
    case 4:  d[1] = 2.0 / 3.0; d[2] = -1.0 / 12.0; break;
    case 6:  d[1] = 3.0 / 4.0; d[2] = -3.0 / 20.0; d[3] = 1.0 / 60.0; break;
    case 8:  d[1] = 4.0 / 5.0; d[2] = -1.0 / 5.0; d[3] = 4.0 / 105.0; d[4] = -1.0 / 280.0; break;
    case 10: d[1] = 5.0 / 6.0; d[2] = -5.0 / 21.0; d[3] = 5.0 / 84.0; d[4] = -5.0 / 504.0;
             d[5] = 1.0 / 1260.0; break;
    default: return -1;
    }
    d[0] = 0.0;
    return 0;
}

static int make_geo(const oracle_grid_t *g, geo_t *G)
{
    if (!g || (g->ndim != 2 && g->ndim != 3) || g->nb < 0 || g->nt < 1 || !(g->dt > 0))
        return -1;
    memset(G, 0, sizeof(*G));
    G->nd = g->ndim;
    if (oracle_fd_weights(g->space_order, G->c) != 0)
        return -1;
    G->r = g->space_order / 2;
    G->cellvol = 1.0;
    for (int a = 0; a < 3; a++) {
        if (a < g->ndim) {
            if (g->shape[a] < 2 || !(g->spacing[a] > 0))
                return -1;
            G->n[a] = g->shape[a];
            G->np[a] = g->shape[a] + 2L * g->nb;
            G->inv_dx2[a] = 1.0 / (g->spacing[a] * g->spacing[a]);
            G->cellvol *= g->spacing[a];
        } else {
            G->n[a] = 1;
            G->np[a] = 1;
        }
    }
    G->st[2] = 1;
    G->st[1] = G->np[2];
    G->st[0] = G->np[1] * G->np[2];
    if (g->ndim == 2) {
        G->st[1] = 1;
        G->st[0] = G->np[1];
    }
    G->N = G->np[0] * G->np[1] * G->np[2];
    return 0;
}

long oracle_padded_points(const oracle_grid_t *g, long *npad3)
{
    geo_t G;
    if (make_geo(g, &G) != 0)
        return -1;
    if (npad3)
        for (int a = 0; a < 3; a++)
            npad3[a] = G.np[a];
    return G.N;
}

static long pidx(const geo_t *G, long i0, long i1, long i2)
{
    return i0 * G->st[0] + i1 * G->st[1] + (G->nd == 3 ? i2 : 0);
}

static long clampl(long v, long lo, long hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

int oracle_pad(const oracle_grid_t *g, const double *phys, double *pad)
{
    geo_t G;
    if (make_geo(g, &G) != 0)
        return -1;
    long nb = g->nb;
#pragma omp parallel for
    for (long i0 = 0; i0 < G.np[0]; i0++)
        for (long i1 = 0; i1 < G.np[1]; i1++)
            for (long i2 = 0; i2 < G.np[2]; i2++) {
                long j0 = clampl(i0 - nb, 0, G.n[0] - 1);
                long j1 = clampl(i1 - nb, 0, G.n[1] - 1);
                long j2 = G.nd == 3 ? clampl(i2 - nb, 0, G.n[2] - 1) : 0;
                long src = G.nd == 3 ? (j0 * G.n[1] + j1) * G.n[2] + j2 : j0 * G.n[1] + j1;
                pad[pidx(&G, i0, i1, i2)] = phys[src];
            }
    return 0;
}

int oracle_pad_transpose(const oracle_grid_t *g, const double *pad, double *phys)
{
    geo_t G;
    if (make_geo(g, &G) != 0)
        return -1;
    long nb = g->nb;
    long nphys = G.n[0] * G.n[1] * G.n[2];
    memset(phys, 0, sizeof(double) * nphys);
    /* serial: several padded cells add into one edge cell */
    for (long i0 = 0; i0 < G.np[0]; i0++)
        for (long i1 = 0; i1 < G.np[1]; i1++)
            for (long i2 = 0; i2 < G.np[2]; i2++) {
                long j0 = clampl(i0 - nb, 0, G.n[0] - 1);
                long j1 = clampl(i1 - nb, 0, G.n[1] - 1);
                long j2 = G.nd == 3 ? clampl(i2 - nb, 0, G.n[2] - 1) : 0;
                long dst = G.nd == 3 ? (j0 * G.n[1] + j1) * G.n[2] + j2 : j0 * G.n[1] + j1;
                phys[dst] += pad[pidx(&G, i0, i1, i2)];
            }
    return 0;
}

/* Cells into the layer along one axis: nb - i before the physical grid,
 * i - (nb + n - 1) after it, 0 inside. */
static long layer_depth(long i, long n, long nb)
{
    if (i < nb)
        return nb - i;
    if (i > nb + n - 1)
        return i - (nb + n - 1);
    return 0;
}

int oracle_eta(const oracle_grid_t *g, double *eta)
{
    geo_t G;
    if (make_geo(g, &G) != 0)
        return -1;
    double emax[3] = {0, 0, 0};
    if (g->nb > 0 && g->vref > 0)
        for (int a = 0; a < G.nd; a++)
            emax[a] = 3.0 * g->vref * log(1.0 / R0_SPONGE) / ((double)g->nb * g->spacing[a]);
#pragma omp parallel for
    for (long i0 = 0; i0 < G.np[0]; i0++)
        for (long i1 = 0; i1 < G.np[1]; i1++)
            for (long i2 = 0; i2 < G.np[2]; i2++) {
                long ii[3] = {i0, i1, i2};
                double e = 0.0;
                for (int a = 0; a < G.nd; a++) {
                    double d = (double)layer_depth(ii[a], G.n[a], g->nb) / (double)(g->nb > 0 ? g->nb : 1);
                    e += emax[a] * d * d;
                }
                eta[pidx(&G, i0, i1, i2)] = e;
            }
    return 0;
}

/* ---------------------------------------------------------------- off-grid points
 * Sec. 2.4: sources and receivers off the grid are spread over / sampled from
 * nearby nodes, by linear interpolation or by Hicks' Kaiser-windowed sinc.
 * The weights below are evaluated from their definitions, node by node:
 *   linear: hat(x) = max(0, 1 - |x|) per axis, x the node's offset from the
 *           point in cells (so a point on a node gives that node weight 1);
 *   sinc:   sinc(x) * I0(b sqrt(1 - (x/r)^2)) / I0(b) for |x| < r, else 0,
 *           with sinc exactly 0 at nonzero integers;
 * and a tap's weight is the product of its per-axis weights. */

static const double ORACLE_PI = 3.14159265358979323846;

/* I0(z) = (1/2pi) * integral over one period of exp(z cos t) dt.  The integrand
 * is smooth and periodic, so the equally spaced rule over the whole period is
 * exact up to aliasing terms 2 I_{kM}(z), k >= 1; with M = 64 nodes and the
 * arguments used here (|z| < 7) these are below 1e-40 of the result. */
static double i0_integral(double z)
{
    const int M = 64;
    double acc = 0.0;
    for (int m = 0; m < M; m++)
        acc += exp(z * cos(2.0 * ORACLE_PI * (double)m / (double)M));
    return acc / (double)M;
}

static double hat_weight(double x)
{
    double d = fabs(x);
    return d < 1.0 ? 1.0 - d : 0.0;
}

static double kaiser_sinc_weight(double x)
{
    const double r = ORACLE_SINC_HALF_WIDTH, b = ORACLE_SINC_KAISER_B;
    if (!(fabs(x) < r))
        return 0.0;
    double s;
    if (x == floor(x))                 /* integer offset: sinc is 1 at 0, 0 elsewhere */
        s = x == 0.0 ? 1.0 : 0.0;
    else
        s = sin(ORACLE_PI * x) / (ORACLE_PI * x);
    double q = x / r;
    return s * i0_integral(b * sqrt(1.0 - q * q)) / i0_integral(b);
}

int oracle_taps_per_point(const oracle_grid_t *g)
{
    if (!g || (g->ndim != 2 && g->ndim != 3) || (g->interp != 0 && g->interp != 1))
        return -1;
    int per_axis = g->interp == 1 ? 2 * ORACLE_SINC_HALF_WIDTH : 2;
    return g->ndim == 3 ? per_axis * per_axis * per_axis : per_axis * per_axis;
}

/* Per-axis node list of one point: every padded node closer than the reach
 * (1 cell linear, r cells sinc) with its weight; the list is then filled up to
 * `slots` entries with weight-0 copies of its first node. */
static int axis_nodes(const geo_t *G, const oracle_grid_t *g, int a, double x, int slots,
                      long *node, double *wt)
{
    double dx = g->spacing[a];
    double span = (double)(G->n[a] - 1) * dx;
    if (x < -1e-9 * dx || x > span + 1e-9 * dx || x != x)
        return -3;                               /* outside the physical grid */
    double pos = x / dx + (double)g->nb;        /* in padded node units */
    double near = floor(pos + 0.5);
    if (fabs(pos - near) < 1e-9)                 /* on a node, up to rounding */
        pos = near;
    int sinc = g->interp == 1;
    double reach = sinc ? (double)ORACLE_SINC_HALF_WIDTH : 1.0;
    if (sinc) {
        /* the point's window of 2r nodes must lie in the padded array */
        double lo = floor(pos) - (ORACLE_SINC_HALF_WIDTH - 1);
        double hi = floor(pos) + ORACLE_SINC_HALF_WIDTH;
        if (lo < 0.0 || hi > (double)(G->np[a] - 1))
            return -3;
    }
    int count = 0;
    for (long j = 0; j < G->np[a]; j++) {
        double off = (double)j - pos;
        if (!(fabs(off) < reach))
            continue;
        if (count == slots)
            return -1;                           /* cannot happen for these reaches */
        node[count] = j;
        wt[count] = sinc ? kaiser_sinc_weight(off) : hat_weight(off);
        count++;
    }
    if (count == 0)
        return -1;
    for (int s = count; s < slots; s++) {
        node[s] = node[0];
        wt[s] = 0.0;
    }
    return 0;
}

int oracle_taps(const oracle_grid_t *g, int npts, const double *xyz, long *idx, double *w)
{
    geo_t G;
    if (make_geo(g, &G) != 0 || npts < 0)
        return -1;
    const int T = oracle_taps_per_point(g);
    if (T < 0)
        return -1;
    const int slots = g->interp == 1 ? 2 * ORACLE_SINC_HALF_WIDTH : 2;
    long node[3][2 * ORACLE_SINC_HALF_WIDTH];
    double wt[3][2 * ORACLE_SINC_HALF_WIDTH];
    for (int p = 0; p < npts; p++) {
        for (int a = 0; a < G.nd; a++) {
            int rc = axis_nodes(&G, g, a, xyz[(long)p * G.nd + a], slots, node[a], wt[a]);
            if (rc != 0)
                return rc;
        }
        /* taps in C order over the per-axis lists (last axis fastest) */
        long *pi = idx + (long)p * T;
        double *pw = w + (long)p * T;
        int t = 0;
        if (G.nd == 2) {
            for (int j0 = 0; j0 < slots; j0++)
                for (int j1 = 0; j1 < slots; j1++, t++) {
                    pi[t] = pidx(&G, node[0][j0], node[1][j1], 0);
                    pw[t] = wt[0][j0] * wt[1][j1];
                }
        } else {
            for (int j0 = 0; j0 < slots; j0++)
                for (int j1 = 0; j1 < slots; j1++)
                    for (int j2 = 0; j2 < slots; j2++, t++) {
                        pi[t] = pidx(&G, node[0][j0], node[1][j1], node[2][j2]);
                        pw[t] = wt[0][j0] * wt[1][j1] * wt[2][j2];
                    }
        }
    }
    return 0;
}

static double lap_at(const geo_t *G, const double *u, long i0, long i1, long i2)
{
    long ii[3] = {i0, i1, i2};
    long p = pidx(G, i0, i1, i2);
    double total = 0.0;
    for (int a = 0; a < G->nd; a++) {
        double s = G->c[0] * u[p];
        for (int j = 1; j <= G->r; j++) {
            double up = (ii[a] + j < G->np[a]) ? u[p + j * G->st[a]] : 0.0;
            double um = (ii[a] - j >= 0) ? u[p - j * G->st[a]] : 0.0;
            s += G->c[j] * (up + um);
        }
        total += s * G->inv_dx2[a];
    }
    return total;
}

int oracle_laplacian(const oracle_grid_t *g, const double *u, double *lu)
{
    geo_t G;
    if (make_geo(g, &G) != 0)
        return -1;
#pragma omp parallel for
    for (long i0 = 0; i0 < G.np[0]; i0++)
        for (long i1 = 0; i1 < G.np[1]; i1++)
            for (long i2 = 0; i2 < G.np[2]; i2++)
                lu[pidx(&G, i0, i1, i2)] = lap_at(&G, u, i0, i1, i2);
    return 0;
}

/* Per-solve coefficient fields on the padded grid. */
typedef struct {
    geo_t G;
    double *k, *a, *b, *vpp;
    long *sidx, *ridx;
    double *sw, *rw;
    int nsrc, nrec, ntap;
} solve_t;

static void solve_free(solve_t *S)
{
    free(S->k);
    free(S->a);
    free(S->b);
    free(S->vpp);
    free(S->sidx);
    free(S->ridx);
    free(S->sw);
    free(S->rw);
}

static int solve_init(solve_t *S, const oracle_grid_t *g, const double *vp,
                      int nsrc, const double *src_xyz, int nrec, const double *rec_xyz)
{
    memset(S, 0, sizeof(*S));
    int rc = make_geo(g, &S->G);
    if (rc != 0)
        return rc;
    if (nsrc < 0 || nrec < 0)
        return -1;
    long N = S->G.N;
    S->nsrc = nsrc;
    S->nrec = nrec;
    S->ntap = oracle_taps_per_point(g);
    if (S->ntap < 0)
        return -1;
    S->k = malloc(sizeof(double) * N);
    S->a = malloc(sizeof(double) * N);
    S->b = malloc(sizeof(double) * N);
    S->vpp = malloc(sizeof(double) * N);
    S->sidx = malloc(sizeof(long) * S->ntap * (nsrc + 1));
    S->ridx = malloc(sizeof(long) * S->ntap * (nrec + 1));
    S->sw = malloc(sizeof(double) * S->ntap * (nsrc + 1));
    S->rw = malloc(sizeof(double) * S->ntap * (nrec + 1));
    if (!S->k || !S->a || !S->b || !S->vpp || !S->sidx || !S->ridx || !S->sw || !S->rw) {
        solve_free(S);
        return -7;
    }
    if ((rc = oracle_taps(g, nsrc, src_xyz, S->sidx, S->sw)) != 0 ||
        (rc = oracle_taps(g, nrec, rec_xyz, S->ridx, S->rw)) != 0) {
        solve_free(S);
        return rc;
    }
    oracle_pad(g, vp, S->vpp);
    oracle_eta(g, S->a); /* eta into a, then converted */
    double dt = g->dt;
    for (long p = 0; p < N; p++) {
        double eta = S->a[p];
        S->k[p] = dt * dt * S->vpp[p] * S->vpp[p];
        S->a[p] = 1.0 / (1.0 + eta * dt / 2.0);
        S->b[p] = (1.0 - eta * dt / 2.0) * S->a[p];
    }
    return 0;
}

/* Dense source term S^n = sum_s W_s^T wavelet[s][n] / cell volume. */
static void source_term(const solve_t *S, const double *wavelet, int nt, int n, double *dense)
{
    memset(dense, 0, sizeof(double) * S->G.N);
    for (int s = 0; s < S->nsrc; s++)
        for (int t = 0; t < S->ntap; t++)
            dense[S->sidx[(long)s * S->ntap + t]] +=
                S->sw[(long)s * S->ntap + t] * wavelet[(long)s * nt + n] / S->G.cellvol;
}

/* Dense adjoint source R^T g^m (no volume factor: sampling has none). */
static void receiver_transpose(const solve_t *S, const double *gtr, int nt, int m, double *dense)
{
    memset(dense, 0, sizeof(double) * S->G.N);
    for (int r = 0; r < S->nrec; r++)
        for (int t = 0; t < S->ntap; t++)
            dense[S->ridx[(long)r * S->ntap + t]] += S->rw[(long)r * S->ntap + t] * gtr[(long)r * nt + m];
}

static double sample(const solve_t *S, const long *idx, const double *w, int p, const double *u)
{
    double acc = 0.0;
    for (int t = 0; t < S->ntap; t++)
        acc += w[(long)p * S->ntap + t] * u[idx[(long)p * S->ntap + t]];
    return acc;
}

/* One forward leapfrog step: unext = a (2 ucur + k (L ucur + src)) - b uprev. */
static void forward_step(const solve_t *S, const double *ucur, const double *uprev,
                         const double *src, double *unext)
{
    const geo_t *G = &S->G;
#pragma omp parallel for
    for (long i0 = 0; i0 < G->np[0]; i0++)
        for (long i1 = 0; i1 < G->np[1]; i1++)
            for (long i2 = 0; i2 < G->np[2]; i2++) {
                long p = pidx(G, i0, i1, i2);
                double lap = lap_at(G, ucur, i0, i1, i2);
                unext[p] = S->a[p] * (2.0 * ucur[p] + S->k[p] * (lap + src[p])) - S->b[p] * uprev[p];
            }
}

/* Time-filtered source of the fourth-order scheme: (S^{n-1} + 10 S^n + S^{n+1}) / 12. */
static void source_term4(const solve_t *S, const double *wavelet, int nt, int n, double *dense)
{
    memset(dense, 0, sizeof(double) * S->G.N);
    for (int s = 0; s < S->nsrc; s++) {
        const double *w = wavelet + (long)s * nt;
        double wm = n >= 1 ? w[n - 1] : 0.0, wp = n + 1 < nt ? w[n + 1] : 0.0;
        double ws = (wm + 10.0 * w[n] + wp) / 12.0;
        for (int t = 0; t < S->ntap; t++)
            dense[S->sidx[(long)s * S->ntap + t]] += S->sw[(long)s * S->ntap + t] * ws / S->G.cellvol;
    }
}

/* One fourth-order step: p = k (L ucur + src); unext = a (2 ucur + p + (k/12) L p) - b uprev. */
static void forward_step4(const solve_t *S, const double *ucur, const double *uprev,
                          const double *src, double *p, double *unext)
{
    const geo_t *G = &S->G;
#pragma omp parallel for
    for (long i0 = 0; i0 < G->np[0]; i0++)
        for (long i1 = 0; i1 < G->np[1]; i1++)
            for (long i2 = 0; i2 < G->np[2]; i2++) {
                long q = pidx(G, i0, i1, i2);
                p[q] = S->k[q] * (lap_at(G, ucur, i0, i1, i2) + src[q]);
            }
#pragma omp parallel for
    for (long i0 = 0; i0 < G->np[0]; i0++)
        for (long i1 = 0; i1 < G->np[1]; i1++)
            for (long i2 = 0; i2 < G->np[2]; i2++) {
                long q = pidx(G, i0, i1, i2);
                double lp = lap_at(G, p, i0, i1, i2);
                unext[q] = S->a[q] * (2.0 * ucur[q] + p[q] + S->k[q] / 12.0 * lp) - S->b[q] * uprev[q];
            }
}

static int time_order_of(const oracle_grid_t *g)
{
    return g->time_order == 0 ? 2 : g->time_order;
}

int oracle_forward(const oracle_grid_t *g, const double *vp,
                   int nsrc, const double *src_xyz, const double *wavelet,
                   int nrec, const double *rec_xyz, double *traces,
                   int nsnap, const int *snap_steps, double *snaps)
{
    const int order = time_order_of(g);
    if (order != 2 && order != 4)
        return -1;
    solve_t S;
    int rc = solve_init(&S, g, vp, nsrc, src_xyz, nrec, rec_xyz);
    if (rc != 0)
        return rc;
    long N = S.G.N;
    int nt = g->nt;
    double *up = calloc(N, sizeof(double));
    double *uc = calloc(N, sizeof(double));
    double *un = calloc(N, sizeof(double));
    double *src = calloc(N, sizeof(double));
    double *pf = order == 4 ? calloc(N, sizeof(double)) : NULL;
    if (!up || !uc || !un || !src || (order == 4 && !pf)) {
        free(up); free(uc); free(un); free(src); free(pf);
        solve_free(&S);
        return -7;
    }
    for (int n = 0; n < nt; n++) {
        for (int r = 0; r < nrec; r++)
            traces[(long)r * nt + n] = sample(&S, S.ridx, S.rw, r, uc);
        for (int q = 0; q < nsnap; q++)
            if (snap_steps[q] == n)
                memcpy(snaps + (long)q * N, uc, sizeof(double) * N);
        if (n == nt - 1)
            break;
        if (order == 4) {
            source_term4(&S, wavelet, nt, n, src);
            forward_step4(&S, uc, up, src, pf, un);
        } else {
            source_term(&S, wavelet, nt, n, src);
            forward_step(&S, uc, up, src, un);
        }
        double *tmp = up;
        up = uc;
        uc = un;
        un = tmp;
    }
    free(up); free(uc); free(un); free(src); free(pf);
    solve_free(&S);
    return 0;
}

int oracle_adjoint(const oracle_grid_t *g, const double *vp,
                   int nsrc, const double *src_xyz, const double *wavelet,
                   int nrec, const double *rec_xyz, const double *grad_traces,
                   double *dvp, double *dwavelet, int seg)
{
    const int order = time_order_of(g);
    if (order != 2 && order != 4)
        return -1;
    solve_t S;
    int rc = solve_init(&S, g, vp, nsrc, src_xyz, nrec, rec_xyz);
    if (rc != 0)
        return rc;
    const geo_t *G = &S.G;
    long N = G->N;
    int nt = g->nt;
    if (seg <= 0)
        seg = (int)ceil(sqrt((double)nt));
    if (seg > nt)
        seg = nt;
    int nseg = (nt + seg - 1) / seg;

    /* checkpoints: state (u^i, u^{i-1}) at i = j*seg */
    double *ck = malloc(sizeof(double) * 2 * N * (size_t)nseg);
    double *useg = malloc(sizeof(double) * N * (size_t)seg);
    double *up = calloc(N, sizeof(double)), *uc = calloc(N, sizeof(double)), *un = calloc(N, sizeof(double));
    double *src = calloc(N, sizeof(double)), *q = calloc(N, sizeof(double));
    double *w1 = calloc(N, sizeof(double)), *w2 = calloc(N, sizeof(double)), *w0 = calloc(N, sizeof(double));
    double *G_acc = calloc(N, sizeof(double)), *lu = calloc(N, sizeof(double));
    double *pf = calloc(N, sizeof(double)), *lp = calloc(N, sizeof(double));
    double *qf = calloc(N, sizeof(double)), *lq = calloc(N, sizeof(double));
    if (!ck || !useg || !up || !uc || !un || !src || !q || !w1 || !w2 || !w0 || !G_acc || !lu ||
        !pf || !lp || !qf || !lq) {
        free(ck); free(useg); free(up); free(uc); free(un); free(src); free(q);
        free(w1); free(w2); free(w0); free(G_acc); free(lu);
        free(pf); free(lp); free(qf); free(lq);
        solve_free(&S);
        return -7;
    }

    /* forward sweep, keeping the segment-start states */
    for (int n = 0; n < nt; n++) {
        if (n % seg == 0) {
            memcpy(ck + (size_t)(n / seg) * 2 * N, uc, sizeof(double) * N);
            memcpy(ck + (size_t)(n / seg) * 2 * N + N, up, sizeof(double) * N);
        }
        if (n == nt - 1)
            break;
        if (order == 4) {
            source_term4(&S, wavelet, nt, n, src);
            forward_step4(&S, uc, up, src, pf, un);
        } else {
            source_term(&S, wavelet, nt, n, src);
            forward_step(&S, uc, up, src, un);
        }
        double *tmp = up;
        up = uc;
        uc = un;
        un = tmp;
    }

    if (dwavelet)
        memset(dwavelet, 0, sizeof(double) * (size_t)nsrc * nt);

    /* reverse sweep: w1 = w^{m+1}, w2 = w^{m+2} */
    for (int j = nseg - 1; j >= 0; j--) {
        int start = j * seg;
        int end = start + seg < nt ? start + seg : nt;
        memcpy(uc, ck + (size_t)j * 2 * N, sizeof(double) * N);
        memcpy(up, ck + (size_t)j * 2 * N + N, sizeof(double) * N);
        for (int n = start; n < end; n++) {
            memcpy(useg + (size_t)(n - start) * N, uc, sizeof(double) * N);
            if (n == end - 1)
                break;
            if (order == 4) {
                source_term4(&S, wavelet, nt, n, src);
                forward_step4(&S, uc, up, src, pf, un);
            } else {
                source_term(&S, wavelet, nt, n, src);
                forward_step(&S, uc, up, src, un);
            }
            double *tmp = up;
            up = uc;
            uc = un;
            un = tmp;
        }
        for (int m = end - 1; m >= start && order == 4; m--) {
            /* fourth order, with T = K + (1/12) K L K and w = K A lambda:
             *   v = L u^m + St^m, p = k v, q = k L w^{m+1}
             *   G += w^{m+1} (v + (1/12) L p) + (1/12) q v
             *   w^m = a (2 w^{m+1} + q + (k/12) L q + k R^T g^m) - b w^{m+2} */
            const double *um = useg + (size_t)(m - start) * N;
            oracle_laplacian(g, um, lu);
            source_term4(&S, wavelet, nt, m, src);
            for (long p = 0; p < N; p++)
                pf[p] = S.k[p] * (lu[p] + src[p]);
            oracle_laplacian(g, pf, lp);
            oracle_laplacian(g, w1, lq);
            for (long p = 0; p < N; p++)
                qf[p] = S.k[p] * lq[p];
#pragma omp parallel for
            for (long p = 0; p < N; p++) {
                double v = lu[p] + src[p];
                G_acc[p] += w1[p] * (v + lp[p] / 12.0) + qf[p] * v / 12.0;
            }
            /* source cotangent before the time filter: dJ/dSt^m = w^{m+1} + q/12,
             * sampled with the source taps / cell volume */
            if (dwavelet)
                for (int s = 0; s < nsrc; s++) {
                    double acc = 0.0;
                    for (int t = 0; t < S.ntap; t++) {
                        long i = S.sidx[(long)s * S.ntap + t];
                        acc += S.sw[(long)s * S.ntap + t] * (w1[i] + qf[i] / 12.0);
                    }
                    dwavelet[(long)s * nt + m] = acc / G->cellvol;
                }
            if (m == 0)
                break;
            oracle_laplacian(g, qf, lq);
            receiver_transpose(&S, grad_traces, nt, m, q);
#pragma omp parallel for
            for (long p = 0; p < N; p++)
                w0[p] = S.a[p] * (2.0 * w1[p] + qf[p] + S.k[p] / 12.0 * lq[p] + S.k[p] * q[p]) -
                        S.b[p] * w2[p];
            double *tmp = w2;
            w2 = w1;
            w1 = w0;
            w0 = tmp;
        }
        for (int m = end - 1; m >= start && order == 2; m--) {
            const double *um = useg + (size_t)(m - start) * N;
            /* imaging: G += w^{m+1} (L u^m + S^m) */
            oracle_laplacian(g, um, lu);
            source_term(&S, wavelet, nt, m, src);
#pragma omp parallel for
            for (long p = 0; p < N; p++)
                G_acc[p] += w1[p] * (lu[p] + src[p]);
            /* source cotangent: W_s w^{m+1} / cell volume */
            if (dwavelet)
                for (int s = 0; s < nsrc; s++)
                    dwavelet[(long)s * nt + m] = sample(&S, S.sidx, S.sw, s, w1) / G->cellvol;
            if (m == 0)
                break;
            /* adjoint step: w^m = a (2 w^{m+1} + k L w^{m+1}) - b w^{m+2} + a k R^T g^m */
            oracle_laplacian(g, w1, lu);
            receiver_transpose(&S, grad_traces, nt, m, q);
#pragma omp parallel for
            for (long p = 0; p < N; p++)
                w0[p] = S.a[p] * (2.0 * w1[p] + S.k[p] * lu[p]) - S.b[p] * w2[p] + S.a[p] * S.k[p] * q[p];
            double *tmp = w2;
            w2 = w1;
            w1 = w0;
            w0 = tmp;
        }
    }

    if (dwavelet && order == 4) {
        /* transpose of St^n = (S^{n-1} + 10 S^n + S^{n+1}) / 12 (zero outside 0..nt-1) */
        double *h = malloc(sizeof(double) * (size_t)nt);
        if (!h)
            rc = -7;
        for (int s = 0; s < nsrc && h; s++) {
            double *row = dwavelet + (long)s * nt;
            memcpy(h, row, sizeof(double) * (size_t)nt);
            for (int j = 0; j < nt; j++)
                row[j] = ((j >= 1 ? h[j - 1] : 0.0) + 10.0 * h[j] + (j + 1 < nt ? h[j + 1] : 0.0)) / 12.0;
        }
        free(h);
    }
    if (dvp) {
        /* dJ/dvp_pad = 2 G / vp_pad, then the transpose of the padding */
        for (long p = 0; p < N; p++)
            lu[p] = 2.0 * G_acc[p] / S.vpp[p];
        oracle_pad_transpose(g, lu, dvp);
    }
    free(ck); free(useg); free(up); free(uc); free(un); free(src); free(q);
    free(w1); free(w2); free(w0); free(G_acc); free(lu);
    free(pf); free(lp); free(qf); free(lq);
    solve_free(&S);
    return rc;
}

int oracle_gradient(const oracle_grid_t *g, const double *vp,
                    int nsrc, const double *src_xyz, const double *wavelet,
                    int nrec, const double *rec_xyz, const double *observed,
                    double *traces_out, double *misfit, double *dvp, int seg)
{
    if (!g || g->nt < 1 || nrec < 0 || (time_order_of(g) != 2 && time_order_of(g) != 4))
        return -1;
    size_t ntr = (size_t)nrec * g->nt;
    double *tr = malloc(sizeof(double) * (ntr + 1));
    double *res = malloc(sizeof(double) * (ntr + 1));
    if (!tr || !res) {
        free(tr); free(res);
        return -7;
    }
    int rc = oracle_forward(g, vp, nsrc, src_xyz, wavelet, nrec, rec_xyz, tr, 0, NULL, NULL);
    if (rc == 0) {
        double J = 0.0;
        for (size_t i = 0; i < ntr; i++) {
            res[i] = tr[i] - observed[i];
            J += 0.5 * res[i] * res[i];
        }
        if (misfit)
            *misfit = J;
        if (traces_out)
            memcpy(traces_out, tr, sizeof(double) * ntr);
        rc = oracle_adjoint(g, vp, nsrc, src_xyz, wavelet, nrec, rec_xyz, res, dvp, NULL, seg);
    }
    free(tr);
    free(res);
    return rc;
}

/* ------------------------------------------------------------------------
 * Heterogeneous medium: variable density and power-law attenuation (y = 0, 2).
 * See the header for the equation and the readings. */

typedef struct {
    double *gam[3];   /* gamma_a = -D_a ln(rho_pad) */
    double d[6];      /* first-derivative weights */
    double inv_dx[3];
} medium_t;

static void medium_free(medium_t *M)
{
    for (int a = 0; a < 3; a++)
        free(M->gam[a]);
}

/* gamma_a on the padded grid; ln rho repeats its edge value beyond the array. */
static int medium_init(medium_t *M, const oracle_grid_t *g, const geo_t *G, const double *rho)
{
    memset(M, 0, sizeof(*M));
    if (oracle_fd1_weights(g->space_order, M->d) != 0)
        return -1;
    long N = G->N;
    double *lr = malloc(sizeof(double) * N);
    if (!lr)
        return -7;
    for (int a = 0; a < G->nd; a++) {
        M->inv_dx[a] = 1.0 / g->spacing[a];
        M->gam[a] = calloc(N, sizeof(double));
        if (!M->gam[a]) {
            free(lr);
            medium_free(M);
            return -7;
        }
    }
    if (rho) {
        long nphys = G->n[0] * G->n[1] * G->n[2];
        for (long i = 0; i < nphys; i++)
            if (!(rho[i] > 0.0) || !isfinite(rho[i])) {
                free(lr);
                medium_free(M);
                return -1;
            }
        oracle_pad(g, rho, lr);
        for (long p = 0; p < N; p++)
            lr[p] = log(lr[p]);
        for (int a = 0; a < G->nd; a++) {
#pragma omp parallel for
            for (long i0 = 0; i0 < G->np[0]; i0++)
                for (long i1 = 0; i1 < G->np[1]; i1++)
                    for (long i2 = 0; i2 < G->np[2]; i2++) {
                        long ii[3] = {i0, i1, i2};
                        long p = pidx(G, i0, i1, i2);
                        double s = 0.0;
                        for (int j = 1; j <= G->r; j++) {
                            long ip = clampl(ii[a] + j, 0, G->np[a] - 1) - ii[a];
                            long im = clampl(ii[a] - j, 0, G->np[a] - 1) - ii[a];
                            s += M->d[j] * (lr[p + ip * G->st[a]] - lr[p + im * G->st[a]]);
                        }
                        M->gam[a][p] = -s * M->inv_dx[a];
                    }
        }
    }
    free(lr);
    return 0;
}

/* sum_a gamma_a D_a u at one point (u is zero beyond the padded array). */
static double density_term_at(const geo_t *G, const medium_t *M, const double *u,
                              long i0, long i1, long i2)
{
    long ii[3] = {i0, i1, i2};
    long p = pidx(G, i0, i1, i2);
    double total = 0.0;
    for (int a = 0; a < G->nd; a++) {
        double s = 0.0;
        for (int j = 1; j <= G->r; j++) {
            double up = (ii[a] + j < G->np[a]) ? u[p + j * G->st[a]] : 0.0;
            double um = (ii[a] - j >= 0) ? u[p - j * G->st[a]] : 0.0;
            s += M->d[j] * (up - um);
        }
        total += M->gam[a][p] * s * M->inv_dx[a];
    }
    return total;
}

int oracle_medium_operator(const oracle_grid_t *g, const double *rho, const double *u,
                           double *out)
{
    geo_t G;
    if (make_geo(g, &G) != 0)
        return -1;
    medium_t M;
    int rc = medium_init(&M, g, &G, rho);
    if (rc != 0)
        return rc;
#pragma omp parallel for
    for (long i0 = 0; i0 < G.np[0]; i0++)
        for (long i1 = 0; i1 < G.np[1]; i1++)
            for (long i2 = 0; i2 < G.np[2]; i2++)
                out[pidx(&G, i0, i1, i2)] =
                    lap_at(&G, u, i0, i1, i2) + density_term_at(&G, &M, u, i0, i1, i2);
    medium_free(&M);
    return 0;
}

int oracle_forward_medium(const oracle_grid_t *g, const double *vp, const double *rho,
                          const double *alpha0, int att_power,
                          int nsrc, const double *src_xyz, const double *wavelet,
                          int nrec, const double *rec_xyz, double *traces)
{
    if (!g || time_order_of(g) != 2 || (att_power != 0 && att_power != 2))
        return -1;
    solve_t S;
    int rc = solve_init(&S, g, vp, nsrc, src_xyz, nrec, rec_xyz);
    if (rc != 0)
        return rc;
    const geo_t *G = &S.G;
    long N = G->N;
    int nt = g->nt;
    double dt = g->dt;
    medium_t M;
    if ((rc = medium_init(&M, g, G, rho)) != 0) {
        solve_free(&S);
        return rc;
    }
    double *beta = calloc(N, sizeof(double));
    double *up = calloc(N, sizeof(double)), *uc = calloc(N, sizeof(double));
    double *un = calloc(N, sizeof(double)), *src = calloc(N, sizeof(double));
    double *al = calloc(N, sizeof(double));
    if (!beta || !up || !uc || !un || !src || !al) {
        free(beta); free(up); free(uc); free(un); free(src); free(al);
        medium_free(&M);
        solve_free(&S);
        return -7;
    }
    if (alpha0) {
        long nphys = G->n[0] * G->n[1] * G->n[2];
        for (long i = 0; i < nphys; i++)
            if (!(alpha0[i] >= 0.0) || !isfinite(alpha0[i])) {
                rc = -1;
                break;
            }
        if (rc == 0) {
            oracle_pad(g, alpha0, al);
            /* y = 0: eta += 2 alpha0 vp (a and b rebuilt); y = 2: beta = 2 alpha0 vp / dt */
            double *eta = calloc(N, sizeof(double));
            if (!eta) {
                rc = -7;
            } else {
                oracle_eta(g, eta);
                for (long p = 0; p < N; p++) {
                    if (att_power == 0) {
                        double e = eta[p] + 2.0 * al[p] * S.vpp[p];
                        S.a[p] = 1.0 / (1.0 + e * dt / 2.0);
                        S.b[p] = (1.0 - e * dt / 2.0) * S.a[p];
                    } else {
                        beta[p] = 2.0 * al[p] * S.vpp[p] / dt;
                    }
                }
                free(eta);
            }
        }
    }
    for (int n = 0; n < nt && rc == 0; n++) {
        for (int r = 0; r < nrec; r++)
            traces[(long)r * nt + n] = sample(&S, S.ridx, S.rw, r, uc);
        if (n == nt - 1)
            break;
        source_term(&S, wavelet, nt, n, src);
#pragma omp parallel for
        for (long i0 = 0; i0 < G->np[0]; i0++)
            for (long i1 = 0; i1 < G->np[1]; i1++)
                for (long i2 = 0; i2 < G->np[2]; i2++) {
                    long p = pidx(G, i0, i1, i2);
                    double lap = lap_at(G, uc, i0, i1, i2);
                    double v = lap + density_term_at(G, &M, uc, i0, i1, i2) + src[p];
                    if (att_power == 2)
                        v += beta[p] * (lap - lap_at(G, up, i0, i1, i2));
                    un[p] = S.a[p] * (2.0 * uc[p] + S.k[p] * v) - S.b[p] * up[p];
                }
        double *tmp = up;
        up = uc;
        uc = un;
        un = tmp;
    }
    free(beta); free(up); free(uc); free(un); free(src); free(al);
    medium_free(&M);
    solve_free(&S);
    return rc;
}

/* Adjoint of the heterogeneous-medium forward (see the header).  State
 * recurrence u^{n+1} = a (2 u^n + k v^n) - b u^{n-1} with
 *   v^n = A u^n + S^n + beta (L u^n - L u^{n-1}),  A = L + sum_a gamma_a D_a;
 * stationarity of the Lagrangian and w = a k lambda give
 *   w^m = a (2 w^{m+1} + k (A^T w^{m+1} + L(beta (w^{m+1} - w^{m+2})) + R^T g^m)) - b w^{m+2},
 *   A^T w = L w - sum_a D_a (gamma_a w)    (D_a^T = -D_a with the zero extension),
 * and, differentiating F^n = a (2 u^n + k v^n) - b u^{n-1} in vp at each point
 * (k = dt^2 vp^2; y = 0: a, b through eta + 2 alpha0 vp; y = 2: beta = 2 alpha0 vp / dt),
 *   dJ/dvp_pad = sum_n w^{n+1} [ (2/vp) v^n
 *                               + (y = 2) (2 alpha0 / dt) (L u^n - L u^{n-1})
 *                               + (y = 0) (dt alpha0 a / k) (2 u^{n-1} - 2 u^n - k v^n) ],
 * then the padding transpose.  dJ/ds_s^n = W_s w^{n+1} / cell volume. */

/* v^n at every point from u^n, u^{n-1} and the dense source (lu: L u^n out). */
static void medium_rhs(const geo_t *G, const medium_t *M, const double *beta, const double *uc,
                       const double *up, const double *src, double *lu, double *v)
{
#pragma omp parallel for
    for (long i0 = 0; i0 < G->np[0]; i0++)
        for (long i1 = 0; i1 < G->np[1]; i1++)
            for (long i2 = 0; i2 < G->np[2]; i2++) {
                long p = pidx(G, i0, i1, i2);
                double l = lap_at(G, uc, i0, i1, i2);
                lu[p] = l;
                double x = l + density_term_at(G, M, uc, i0, i1, i2) + src[p];
                if (beta[p] != 0.0)
                    x += beta[p] * (l - lap_at(G, up, i0, i1, i2));
                v[p] = x;
            }
}

int oracle_adjoint_medium(const oracle_grid_t *g, const double *vp, const double *rho,
                          const double *alpha0, int att_power, int nsrc, const double *src_xyz,
                          const double *wavelet, int nrec, const double *rec_xyz,
                          const double *grad_traces, double *dvp, double *dwavelet, int seg)
{
    if (!g || time_order_of(g) != 2 || (att_power != 0 && att_power != 2))
        return -1;
    solve_t S;
    int rc = solve_init(&S, g, vp, nsrc, src_xyz, nrec, rec_xyz);
    if (rc != 0)
        return rc;
    const geo_t *G = &S.G;
    const long N = G->N;
    const int nt = g->nt, nd = G->nd;
    const double dt = g->dt;
    medium_t M;
    if ((rc = medium_init(&M, g, G, rho)) != 0) {
        solve_free(&S);
        return rc;
    }
    if (seg <= 0)
        seg = (int)ceil(sqrt((double)nt));
    if (seg > nt)
        seg = nt;
    const int nseg = (nt + seg - 1) / seg;
    double *al = calloc(N, sizeof(double)), *beta = calloc(N, sizeof(double));
    double *ck = malloc(sizeof(double) * 2 * N * (size_t)nseg);
    double *useg = malloc(sizeof(double) * N * (size_t)(seg + 1));
    double *up = calloc(N, sizeof(double)), *uc = calloc(N, sizeof(double)), *un = calloc(N, sizeof(double));
    double *src = calloc(N, sizeof(double)), *lu = calloc(N, sizeof(double)), *v = calloc(N, sizeof(double));
    double *w0 = calloc(N, sizeof(double)), *w1 = calloc(N, sizeof(double)), *w2 = calloc(N, sizeof(double));
    double *y = calloc(N, sizeof(double)), *q = calloc(N, sizeof(double)), *Gacc = calloc(N, sizeof(double));
    double *z[3] = {NULL, NULL, NULL};
    int ok = al && beta && ck && useg && up && uc && un && src && lu && v && w0 && w1 && w2 && y && q && Gacc;
    for (int a = 0; a < nd; a++)
        ok = ok && (z[a] = calloc(N, sizeof(double))) != NULL;
    if (!ok) {
        rc = -7;
        goto done;
    }
    if (alpha0) {
        long nphys = G->n[0] * G->n[1] * G->n[2];
        for (long i = 0; i < nphys; i++)
            if (!(alpha0[i] >= 0.0) || !isfinite(alpha0[i])) {
                rc = -1;
                goto done;
            }
        oracle_pad(g, alpha0, al);
        double *eta = v; /* scratch */
        oracle_eta(g, eta);
        for (long p = 0; p < N; p++) {
            if (att_power == 0) {
                double e = eta[p] + 2.0 * al[p] * S.vpp[p];
                S.a[p] = 1.0 / (1.0 + e * dt / 2.0);
                S.b[p] = (1.0 - e * dt / 2.0) * S.a[p];
            } else {
                beta[p] = 2.0 * al[p] * S.vpp[p] / dt;
            }
        }
    }
    /* forward sweep, keeping (u^n, u^{n-1}) at the segment starts */
    for (int n = 0; n < nt; n++) {
        if (n % seg == 0) {
            memcpy(ck + (size_t)(n / seg) * 2 * N, uc, sizeof(double) * N);
            memcpy(ck + (size_t)(n / seg) * 2 * N + N, up, sizeof(double) * N);
        }
        if (n == nt - 1)
            break;
        source_term(&S, wavelet, nt, n, src);
        medium_rhs(G, &M, beta, uc, up, src, lu, v);
        for (long p = 0; p < N; p++)
            un[p] = S.a[p] * (2.0 * uc[p] + S.k[p] * v[p]) - S.b[p] * up[p];
        double *tmp = up;
        up = uc;
        uc = un;
        un = tmp;
    }
    if (dwavelet)
        memset(dwavelet, 0, sizeof(double) * (size_t)nsrc * nt);
    /* reverse sweep: w1 = w^{m+1}, w2 = w^{m+2}; useg[0] = u^{start-1}, useg[1 + i] = u^{start+i} */
    for (int j = nseg - 1; j >= 0; j--) {
        int start = j * seg;
        int end = start + seg < nt ? start + seg : nt;
        memcpy(uc, ck + (size_t)j * 2 * N, sizeof(double) * N);
        memcpy(up, ck + (size_t)j * 2 * N + N, sizeof(double) * N);
        memcpy(useg, up, sizeof(double) * N);
        for (int n = start; n < end; n++) {
            memcpy(useg + (size_t)(n - start + 1) * N, uc, sizeof(double) * N);
            if (n == end - 1)
                break;
            source_term(&S, wavelet, nt, n, src);
            medium_rhs(G, &M, beta, uc, up, src, lu, v);
            for (long p = 0; p < N; p++)
                un[p] = S.a[p] * (2.0 * uc[p] + S.k[p] * v[p]) - S.b[p] * up[p];
            double *tmp = up;
            up = uc;
            uc = un;
            un = tmp;
        }
        for (int m = end - 1; m >= start; m--) {
            const double *um = useg + (size_t)(m - start + 1) * N;
            const double *umm = useg + (size_t)(m - start) * N;
            /* imaging of step m (u^m -> u^{m+1}) with lambda^{m+1} = w^{m+1} / (a k) */
            source_term(&S, wavelet, nt, m, src);
            medium_rhs(G, &M, beta, um, umm, src, lu, v);
            if (att_power == 2)
                oracle_laplacian(g, umm, q);   /* L u^{m-1} */
#pragma omp parallel for
            for (long p = 0; p < N; p++) {
                double d = 2.0 * v[p] / S.vpp[p];
                if (alpha0 && att_power == 2)
                    d += 2.0 * al[p] / dt * (lu[p] - q[p]);
                if (alpha0 && att_power == 0)
                    d += dt * al[p] * S.a[p] / S.k[p] * (2.0 * umm[p] - 2.0 * um[p] - S.k[p] * v[p]);
                Gacc[p] += w1[p] * d;
            }
            if (dwavelet)
                for (int s2 = 0; s2 < nsrc; s2++)
                    dwavelet[(long)s2 * nt + m] = sample(&S, S.sidx, S.sw, s2, w1) / G->cellvol;
            if (m == 0)
                break;
            /* adjoint step */
            for (long p = 0; p < N; p++)
                y[p] = (1.0 + beta[p]) * w1[p] - beta[p] * w2[p];
            for (int a = 0; a < nd; a++)
                for (long p = 0; p < N; p++)
                    z[a][p] = M.gam[a][p] * w1[p];
            receiver_transpose(&S, grad_traces, nt, m, q);
#pragma omp parallel for
            for (long i0 = 0; i0 < G->np[0]; i0++)
                for (long i1 = 0; i1 < G->np[1]; i1++)
                    for (long i2 = 0; i2 < G->np[2]; i2++) {
                        long ii[3] = {i0, i1, i2};
                        long p = pidx(G, i0, i1, i2);
                        double rhs = lap_at(G, y, i0, i1, i2) + q[p];
                        for (int a = 0; a < nd; a++) {
                            double sd = 0.0;
                            for (int jj = 1; jj <= G->r; jj++) {
                                double zp = (ii[a] + jj < G->np[a]) ? z[a][p + jj * G->st[a]] : 0.0;
                                double zm = (ii[a] - jj >= 0) ? z[a][p - jj * G->st[a]] : 0.0;
                                sd += M.d[jj] * (zp - zm);
                            }
                            rhs -= sd * M.inv_dx[a];
                        }
                        w0[p] = S.a[p] * (2.0 * w1[p] + S.k[p] * rhs) - S.b[p] * w2[p];
                    }
            double *tmp = w2;
            w2 = w1;
            w1 = w0;
            w0 = tmp;
        }
    }
    if (dvp)
        oracle_pad_transpose(g, Gacc, dvp);
done:
    free(al); free(beta); free(ck); free(useg); free(up); free(uc); free(un); free(src);
    free(lu); free(v); free(w0); free(w1); free(w2); free(y); free(q); free(Gacc);
    for (int a = 0; a < 3; a++)
        free(z[a]);
    medium_free(&M);
    solve_free(&S);
    return rc;
}

int oracle_gradient_medium(const oracle_grid_t *g, const double *vp, const double *rho,
                           const double *alpha0, int att_power, int nsrc, const double *src_xyz,
                           const double *wavelet, int nrec, const double *rec_xyz,
                           const double *observed, double *traces_out, double *misfit, double *dvp,
                           int seg)
{
    if (!g || g->nt < 1 || nrec < 0)
        return -1;
    size_t ntr = (size_t)nrec * g->nt;
    double *tr = malloc(sizeof(double) * (ntr + 1)), *res = malloc(sizeof(double) * (ntr + 1));
    if (!tr || !res) {
        free(tr); free(res);
        return -7;
    }
    int rc = oracle_forward_medium(g, vp, rho, alpha0, att_power, nsrc, src_xyz, wavelet, nrec,
                                   rec_xyz, tr);
    if (rc == 0) {
        double J = 0.0;
        for (size_t i = 0; i < ntr; i++) {
            res[i] = tr[i] - observed[i];
            J += 0.5 * res[i] * res[i];
        }
        if (misfit)
            *misfit = J;
        if (traces_out)
            memcpy(traces_out, tr, sizeof(double) * ntr);
        rc = oracle_adjoint_medium(g, vp, rho, alpha0, att_power, nsrc, src_xyz, wavelet, nrec,
                                   rec_xyz, res, dvp, NULL, seg);
    }
    free(tr);
    free(res);
    return rc;
}

/* ------------------------------------------------------------------------
 * Perfectly matched layer (see the header).  Per axis a, in the layer of that
 * axis, the stretched derivatives (1/s_a) d_a with s_a = 1 + zeta_a / (i w)
 * become d_a - (memory term): the first derivative loses psi_a and the second
 * chi_a, where psi_a and chi_a follow d_a u and d_a(d_a u - psi_a) through a
 * relaxation of rate zeta_a.  Outside every layer psi = chi = 0 and the step is
 * the plain leapfrog. */

/* Second derivative along axis a (one axis of the Laplacian) at point p. */
static double d2_axis(const geo_t *G, const double *u, const long *ii, long p, int a)
{
    double s = G->c[0] * u[p];
    for (int j = 1; j <= G->r; j++) {
        double up = (ii[a] + j < G->np[a]) ? u[p + j * G->st[a]] : 0.0;
        double um = (ii[a] - j >= 0) ? u[p - j * G->st[a]] : 0.0;
        s += G->c[j] * (up + um);
    }
    return s * G->inv_dx2[a];
}

/* Centred first derivative along axis a at point p (zero beyond the array). */
static double d1_axis(const geo_t *G, const double *d, double inv_dx, const double *u,
                      const long *ii, long p, int a)
{
    double s = 0.0;
    for (int j = 1; j <= G->r; j++) {
        double up = (ii[a] + j < G->np[a]) ? u[p + j * G->st[a]] : 0.0;
        double um = (ii[a] - j >= 0) ? u[p - j * G->st[a]] : 0.0;
        s += d[j] * (up - um);
    }
    return s * inv_dx;
}

int oracle_forward_pml(const oracle_grid_t *g, const double *vp, int nsrc, const double *src_xyz,
                       const double *wavelet, int nrec, const double *rec_xyz, double *traces)
{
    if (!g || time_order_of(g) != 2)
        return -1;
    solve_t S;
    int rc = solve_init(&S, g, vp, nsrc, src_xyz, nrec, rec_xyz);
    if (rc != 0)
        return rc;
    const geo_t *G = &S.G;
    const long N = G->N;
    const int nd = G->nd, nt = g->nt;
    const double dt = g->dt;
    double d[6];
    oracle_fd1_weights(g->space_order, d);
    double zmax[3] = {0, 0, 0}, inv_dx[3] = {0, 0, 0};
    for (int a = 0; a < nd; a++) {
        inv_dx[a] = 1.0 / g->spacing[a];
        if (g->nb > 0 && g->vref > 0)
            zmax[a] = 3.0 * g->vref * log(1.0 / ORACLE_PML_R0) / (2.0 * g->nb * g->spacing[a]);
    }
    double *up = calloc(N, sizeof(double)), *uc = calloc(N, sizeof(double));
    double *un = calloc(N, sizeof(double)), *src = calloc(N, sizeof(double));
    double *psi[3] = {NULL, NULL, NULL}, *psin[3] = {NULL, NULL, NULL}, *chi[3] = {NULL, NULL, NULL};
    int ok = up && uc && un && src;
    for (int a = 0; a < nd; a++) {
        psi[a] = calloc(N, sizeof(double));
        psin[a] = calloc(N, sizeof(double));
        chi[a] = calloc(N, sizeof(double));
        ok = ok && psi[a] && psin[a] && chi[a];
    }
    if (!ok) {
        rc = -7;
        goto done;
    }
    for (int n = 0; n < nt; n++) {
        for (int r = 0; r < nrec; r++)
            traces[(long)r * nt + n] = sample(&S, S.ridx, S.rw, r, uc);
        if (n == nt - 1)
            break;
        source_term(&S, wavelet, nt, n, src);
#pragma omp parallel for
        for (long i0 = 0; i0 < G->np[0]; i0++)
            for (long i1 = 0; i1 < G->np[1]; i1++)
                for (long i2 = 0; i2 < G->np[2]; i2++) {
                    long ii[3] = {i0, i1, i2};
                    long p = pidx(G, i0, i1, i2);
                    double rhs = src[p];
                    for (int a = 0; a < nd; a++) {
                        double lu = d2_axis(G, uc, ii, p, a);
                        double depth = (double)layer_depth(ii[a], G->n[a], g->nb) / (double)(g->nb > 0 ? g->nb : 1);
                        double zeta = zmax[a] * depth * depth;
                        if (zeta == 0.0) {
                            rhs += lu;
                            psin[a][p] = 0.0;
                            continue;
                        }
                        double E = exp(-zeta * dt);
                        double dpsi = d1_axis(G, d, inv_dx[a], psi[a], ii, p, a);
                        chi[a][p] = E * chi[a][p] + (1.0 - E) * (lu - dpsi);
                        psin[a][p] = E * psi[a][p] + (1.0 - E) * d1_axis(G, d, inv_dx[a], uc, ii, p, a);
                        rhs += lu - dpsi - chi[a][p];
                    }
                    un[p] = 2.0 * uc[p] - up[p] + S.k[p] * rhs;
                }
        double *tmp = up;
        up = uc;
        uc = un;
        un = tmp;
        for (int a = 0; a < nd; a++) {
            tmp = psi[a];
            psi[a] = psin[a];
            psin[a] = tmp;
        }
    }
done:
    free(up); free(uc); free(un); free(src);
    for (int a = 0; a < 3; a++) {
        free(psi[a]);
        free(psin[a]);
        free(chi[a]);
    }
    solve_free(&S);
    return rc;
}

/* ------------------------------------------------------------------------
 * Zero-phase FIR low-pass (see the header). */
int oracle_lowpass(const double *in, double *out, int count, int nt, double dt, double f_max)
{
    if (!in || !out || count < 0 || nt < 1 || !(dt > 0) || !(f_max > 0) || f_max * dt >= 0.5)
        return -1;
    const double pi = 3.14159265358979323846;
    int K = (int)ceil(2.0 / (f_max * dt));
    double *h = malloc(sizeof(double) * (2 * K + 1));
    if (!h)
        return -7;
    double sum = 0.0;
    for (int k = -K; k <= K; k++) {
        double x = 2.0 * f_max * dt * k;
        double sc = k == 0 ? 1.0 : sin(pi * x) / (pi * x);
        double win = 0.5 + 0.5 * cos(pi * k / (K + 1.0));
        h[k + K] = 2.0 * f_max * dt * sc * win;
        sum += h[k + K];
    }
    for (int k = 0; k <= 2 * K; k++)
        h[k] /= sum;
    for (int c = 0; c < count; c++)
        for (int n = 0; n < nt; n++) {
            double acc = 0.0;
            for (int k = -K; k <= K; k++) {
                int m = n - k;
                if (m >= 0 && m < nt)
                    acc += h[k + K] * in[(long)c * nt + m];
            }
            out[(long)c * nt + n] = acc;
        }
    free(h);
    return K;
}
