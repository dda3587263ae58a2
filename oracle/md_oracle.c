/*
 * FP64 CPU oracle for one short-range molecular-dynamics time step:
 * Embedded Atom Method (Cr-Cr) + Morse (Cr-C) forces and velocity-Verlet integration.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is linked by the test suite, by the package's
 * smoke check and by the benchmark's CPU-baseline leg.  The product path (the HIP
 * library) never links, loads or calls it, and it shares no code with that path.
 *
 * Every function is the plain definition of what it computes, written for a reader to
 * check against the paper by eye:
 *   - neighbour sets: brute force over all atom pairs (no cells, no blocking);
 *   - electron density and embedding derivative: Section 3.1, first pass;
 *   - force: Eq. (1) of Section 3.1 with V = the pair potential;
 *   - energy: Eq. (A1) without the M(P) term (the synthetic potential has none),
 *     plus the shifted Cr-C Morse pair energy (form of Eq. (A5));
 *   - integrator: Eqs. (A11)-(A13) for Task 3 and the final half kick of Task 5;
 *   - list maintenance: the outer list is rebuilt when any atom has moved more than
 *     half the skin since the last build (Section 2.6);
 *   - global sums: Neumaier compensated summation (the self-compensated summation of
 *     Section 2.3).
 * Loops over atoms are owner-computes (each iteration writes only its own atom, as in
 * Section 3.3.1) and are split over OpenMP threads.
 *
 * Two potentials.  The paper's own EAM form (Appendix, Eqs. A1-A4: logarithmic embedding
 * F(rho), the M(P) term with P_i = sum_j f^2(r_ij), power-law density f, Pasianot pair Phi),
 * evaluated with synthetic parameter values because the paper prints none, and:
 * Synthetic potential of the benchmark workloads (the paper does not print its parameters):
 *   phi(r) = (r-c)^2 (c0 + c1 r + c2 r^2) for r < c        pair potential
 *   f(r)   = (r-d)^2                      for r < d        density function
 *   F(rho) = -A sqrt(rho), F'(0) taken as 0               embedding function
 *   phiM(r) = D [exp(-2 alpha (r-r0)) - 2 exp(-alpha (r-r0))] for r < rc, energy shifted
 * Units: eV, Angstrom, fs, u.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double lo[3];
    double len[3];
    int32_t periodic[3];
    int32_t pad;
} orc_box;

typedef struct {
    double A, c, d, c0, c1, c2;
} orc_eam;

typedef struct {
    double D, alpha, r0, rc;
} orc_morse;

/* The paper's EAM form (Appendix):
 *   F(rho) = -Fo [1 - n ln(rho/rho_e)] (rho/rho_e)^n          (A3; ln of a power written out)
 *   M(P)   = alpha (P/P_e - 1)^2 exp(-(P/P_e - 1)^2)            (A3)
 *   f(r)   = fe (re/r)^beta for r < rc, else 0                   (A2; rc the cutoff r*)
 *   Phi(r) = (x-d)^2 (a3 x^3 + a2 x^2 + a1 x + a0), x = r/re < d  (A4)
 *   rho_i = sum_j f(r_ij), P_i = sum_j f(r_ij)^2                (A2) */
typedef struct {
    double Fo, n, rho_e, alpha, P_e, fe, re, beta, a0, a1, a2, a3, d, rc;
} orc_paper;

/* Conversion factors between eV, u, Angstrom and fs (CODATA 2018 values of e and u). */
static double orc_acc_factor(void)
{
    /* (eV / (Angstrom u)) -> Angstrom / fs^2 */
    return 1.602176634e-19 / 1.66053906660e-27 * 1e-10;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ---------------------------------------------------------------------------------- */
/* Geometry                                                                             */
/* ---------------------------------------------------------------------------------- */

/* Bring each periodic coordinate back into [lo, lo + len) by one shift of len. */
void orc_wrap(const orc_box *b, int64_t n, double *x)
{
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            if (!b->periodic[a]) continue;
            double hi = b->lo[a] + b->len[a];
            if (x[3 * i + a] >= hi)
                x[3 * i + a] -= b->len[a];
            else if (x[3 * i + a] < b->lo[a])
                x[3 * i + a] += b->len[a];
        }
}

/* Minimum-image component of a separation along one axis. */
static double min_image(const orc_box *b, int a, double d)
{
    if (b->periodic[a]) {
        double half = 0.5 * b->len[a];
        if (d > half)
            d -= b->len[a];
        else if (d < -half)
            d += b->len[a];
    }
    return d;
}

/* Separation s = xj - xi (minimum image) and its squared length (dx dx + dy dy) + dz dz. */
static double separation(const orc_box *b, const double *xi, const double *xj, double s[3])
{
    for (int a = 0; a < 3; ++a) s[a] = min_image(b, a, xj[a] - xi[a]);
    return (s[0] * s[0] + s[1] * s[1]) + s[2] * s[2];
}

/* Position of carbon atom k: its base position moved by the indenter displacement along z. */
static void carbon_position(const double *xc, int64_t k, double ind_z, double p[3])
{
    p[0] = xc[3 * k + 0];
    p[1] = xc[3 * k + 1];
    p[2] = xc[3 * k + 2] + ind_z;
}

/* ---------------------------------------------------------------------------------- */
/* Neighbour sets (brute force)                                                         */
/* ---------------------------------------------------------------------------------- */

/*
 * For each atom i in `rows` (all atoms when rows == NULL), the set
 * { j != i : |x_j - x_i|^2 < r^2 } in ascending j.  Row t of idx holds up to cap
 * entries; cnt[t] is the full set size (it may exceed cap).  Returns the largest count.
 */
int64_t orc_neighbors(const orc_box *b, double r, int64_t n, const double *x,
                      int64_t nrows, const int64_t *rows, int64_t cap, int32_t *cnt, int32_t *idx)
{
    const double r2 = r * r;
    int64_t m = rows ? nrows : n;
    int64_t maxc = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(max : maxc)
    for (int64_t t = 0; t < m; ++t) {
        int64_t i = rows ? rows[t] : t;
        int64_t c = 0;
        double s[3];
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            if (separation(b, x + 3 * i, x + 3 * j, s) < r2) {
                if (c < cap) idx[t * cap + c] = (int32_t)j;
                ++c;
            }
        }
        cnt[t] = (int32_t)c;
        if (c > maxc) maxc = c;
    }
    return maxc;
}

/* Carbon atoms within r of each Cr atom: same predicate against xc + (0,0,ind_z). */
int64_t orc_cross_neighbors(const orc_box *b, double r, int64_t n, const double *x,
                            int64_t nc, const double *xc, double ind_z,
                            int64_t nrows, const int64_t *rows, int64_t cap, int32_t *cnt,
                            int32_t *idx)
{
    const double r2 = r * r;
    int64_t m = rows ? nrows : n;
    int64_t maxc = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(max : maxc)
    for (int64_t t = 0; t < m; ++t) {
        int64_t i = rows ? rows[t] : t;
        int64_t c = 0;
        double s[3], p[3];
        for (int64_t k = 0; k < nc; ++k) {
            carbon_position(xc, k, ind_z, p);
            if (separation(b, x + 3 * i, p, s) < r2) {
                if (c < cap) idx[t * cap + c] = (int32_t)k;
                ++c;
            }
        }
        cnt[t] = (int32_t)c;
        if (c > maxc) maxc = c;
    }
    return maxc;
}

/* ---------------------------------------------------------------------------------- */
/* Neighbour sets from a cell grid (the cell-linked list of Section 2.6)                 */
/* ---------------------------------------------------------------------------------- */

/*
 * The same sets as orc_neighbors / orc_cross_neighbors (same predicate, ascending index),
 * found by binning the candidates into cells of edge >= r so that only the 27 cells around
 * an atom's own cell need testing: along each axis any pair closer than r lies in the same
 * or an adjacent cell (across the face on periodic axes).  A periodic axis with fewer than
 * three cells has every cell visited once.  For large systems only (the CPU baseline);
 * the parity tests use the brute-force sets.
 */
typedef struct {
    double lo[3], edge[3];
    int64_t nc[3];
    int64_t *start;    /* [ncell + 1] first entry of each cell in `item` */
    int64_t *item;     /* [m] point indices by cell, ascending within a cell */
} orc_grid;

/* Cell coordinate of position coordinate v along axis a (folded into the box on periodic
 * axes, clamped into the grid on open ones). */
static int64_t grid_coord(const orc_box *b, const orc_grid *g, int a, double v)
{
    if (b->periodic[a]) v = v - b->len[a] * floor((v - b->lo[a]) / b->len[a]);
    double t = floor((v - g->lo[a]) / g->edge[a]);
    if (!(t >= 0.0)) t = 0.0;
    if (t > (double)(g->nc[a] - 1)) t = (double)(g->nc[a] - 1);
    return (int64_t)t;
}

/* Grid of cells of edge >= r over the box (periodic axes) or the points' extent (open axes),
 * holding the m points p (stride 3, shifted by dz along z). */
static void grid_build(const orc_box *b, double r, int64_t m, const double *p, double dz, orc_grid *g)
{
    for (int a = 0; a < 3; ++a) {
        double lo, ext;
        if (b->periodic[a]) {
            lo = b->lo[a];
            ext = b->len[a];
        } else {
            double mn = INFINITY, mx = -INFINITY;
            for (int64_t i = 0; i < m; ++i) {
                double v = p[3 * i + a] + (a == 2 ? dz : 0.0);
                if (v < mn) mn = v;
                if (v > mx) mx = v;
            }
            if (!(mn <= mx)) { mn = 0.0; mx = 0.0; }
            lo = mn;
            ext = mx - mn;
        }
        int64_t n = (int64_t)floor(ext / r);
        if (n < 1) n = 1;
        g->lo[a] = lo;
        g->nc[a] = n;
        g->edge[a] = ext > 0.0 ? ext / (double)n : r;
        if (g->edge[a] < r) g->edge[a] = r;
    }
    int64_t ncell = g->nc[0] * g->nc[1] * g->nc[2];
    int64_t *cell = (int64_t *)malloc(sizeof(int64_t) * (m ? m : 1));
    g->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    g->item = (int64_t *)malloc(sizeof(int64_t) * (m ? m : 1));
    for (int64_t i = 0; i < m; ++i) {
        int64_t c[3];
        for (int a = 0; a < 3; ++a) c[a] = grid_coord(b, g, a, p[3 * i + a] + (a == 2 ? dz : 0.0));
        cell[i] = (c[2] * g->nc[1] + c[1]) * g->nc[0] + c[0];
        g->start[cell[i] + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) g->start[c + 1] += g->start[c];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncell ? ncell : 1));
    memcpy(fill, g->start, sizeof(int64_t) * (size_t)ncell);
    for (int64_t i = 0; i < m; ++i) g->item[fill[cell[i]]++] = i;   /* ascending i per cell */
    free(fill);
    free(cell);
}

static void grid_free(orc_grid *g)
{
    free(g->start);
    free(g->item);
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t u = *(const int32_t *)a, v = *(const int32_t *)b;
    return (u > v) - (u < v);
}

/* Cells to visit along one axis around cell c: c-1, c, c+1 (periodic wrap; outside an open
 * axis skipped), or every cell once on a periodic axis with fewer than three. */
static int stencil_axis(const orc_box *b, const orc_grid *g, int a, int64_t c, int64_t out[3])
{
    int k = 0;
    if (b->periodic[a] && g->nc[a] < 3) {
        for (int64_t t = 0; t < g->nc[a]; ++t) out[k++] = t;
        return k;
    }
    for (int64_t t = c - 1; t <= c + 1; ++t) {
        int64_t u = t;
        if (b->periodic[a]) u = (t + g->nc[a]) % g->nc[a];
        else if (t < 0 || t >= g->nc[a]) continue;
        out[k++] = u;
    }
    return k;
}

/* Row t of (cnt, idx): the points of grid g (positions p, shifted by dz along z) within r of
 * position xi, except `self`, ascending; returns the set size (entries beyond cap dropped). */
static int64_t grid_query(const orc_box *b, const orc_grid *g, const double *p, double dz, double r2,
                          const double *xi, int64_t self, int64_t cap, int32_t *row)
{
    int64_t cx[3], cy[3], cz[3], c = 0;
    int nx = stencil_axis(b, g, 0, grid_coord(b, g, 0, xi[0]), cx);
    int ny = stencil_axis(b, g, 1, grid_coord(b, g, 1, xi[1]), cy);
    int nz = stencil_axis(b, g, 2, grid_coord(b, g, 2, xi[2]), cz);
    double s[3], pj[3];
    for (int iz = 0; iz < nz; ++iz)
        for (int iy = 0; iy < ny; ++iy)
            for (int ix = 0; ix < nx; ++ix) {
                int64_t cell = (cz[iz] * g->nc[1] + cy[iy]) * g->nc[0] + cx[ix];
                for (int64_t e = g->start[cell]; e < g->start[cell + 1]; ++e) {
                    int64_t j = g->item[e];
                    if (j == self) continue;
                    pj[0] = p[3 * j + 0];
                    pj[1] = p[3 * j + 1];
                    pj[2] = p[3 * j + 2] + dz;
                    if (separation(b, xi, pj, s) < r2) {
                        if (c < cap) row[c] = (int32_t)j;
                        ++c;
                    }
                }
            }
    qsort(row, (size_t)(c < cap ? c : cap), sizeof(int32_t), cmp_i32);
    return c;
}

/* orc_neighbors' sets (all atoms), from a cell grid.  cnt[i] is the full set size; a set
 * larger than cap keeps cap of its entries, not necessarily the smallest (callers treat any
 * count above cap as an error, as with orc_neighbors). */
int64_t orc_neighbors_cells(const orc_box *b, double r, int64_t n, const double *x, int64_t cap,
                            int32_t *cnt, int32_t *idx)
{
    orc_grid g;
    grid_build(b, r, n, x, 0.0, &g);
    const double r2 = r * r;
    int64_t maxc = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(max : maxc)
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = grid_query(b, &g, x, 0.0, r2, x + 3 * i, i, cap, idx + i * cap);
        cnt[i] = (int32_t)c;
        if (c > maxc) maxc = c;
    }
    grid_free(&g);
    return maxc;
}

/* orc_cross_neighbors' sets (all atoms), from a cell grid over the carbons. */
int64_t orc_cross_neighbors_cells(const orc_box *b, double r, int64_t n, const double *x, int64_t nc,
                                  const double *xc, double ind_z, int64_t cap, int32_t *cnt, int32_t *idx)
{
    orc_grid g;
    grid_build(b, r, nc, xc, ind_z, &g);
    const double r2 = r * r;
    int64_t maxc = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(max : maxc)
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = nc ? grid_query(b, &g, xc, ind_z, r2, x + 3 * i, -1, cap, idx + i * cap) : 0;
        cnt[i] = (int32_t)c;
        if (c > maxc) maxc = c;
    }
    grid_free(&g);
    return maxc;
}

/* ---------------------------------------------------------------------------------- */
/* Potential functions                                                                  */
/* ---------------------------------------------------------------------------------- */

static double pair_phi(const orc_eam *p, double r)
{
    double u = r - p->c;
    return u * u * (p->c0 + p->c1 * r + p->c2 * r * r);
}

static double pair_dphi(const orc_eam *p, double r)
{
    double u = r - p->c;
    return 2.0 * u * (p->c0 + p->c1 * r + p->c2 * r * r) + u * u * (p->c1 + 2.0 * p->c2 * r);
}

static double dens_f(const orc_eam *p, double r)
{
    double u = r - p->d;
    return u * u;
}

static double dens_df(const orc_eam *p, double r)
{
    return 2.0 * (r - p->d);
}

static double embed_F(const orc_eam *p, double rho)
{
    return -p->A * sqrt(rho);
}

static double embed_dF(const orc_eam *p, double rho)
{
    return rho > 0.0 ? -p->A / (2.0 * sqrt(rho)) : 0.0;
}

static double morse_phi(const orc_morse *m, double r)
{
    double e = exp(-m->alpha * (r - m->r0));
    return m->D * (e * e - 2.0 * e);
}

static double morse_dphi(const orc_morse *m, double r)
{
    double e = exp(-m->alpha * (r - m->r0));
    return m->D * (-2.0 * m->alpha * e * e + 2.0 * m->alpha * e);
}

void orc_potential_values(const orc_eam *p, const orc_morse *m, double r, double out[8])
{
    out[0] = r < p->c ? pair_phi(p, r) : 0.0;
    out[1] = r < p->c ? pair_dphi(p, r) : 0.0;
    out[2] = r < p->d ? dens_f(p, r) : 0.0;
    out[3] = r < p->d ? dens_df(p, r) : 0.0;
    out[4] = embed_F(p, r);      /* r used as rho */
    out[5] = embed_dF(p, r);
    out[6] = r < m->rc ? morse_phi(m, r) : 0.0;
    out[7] = r < m->rc ? morse_dphi(m, r) : 0.0;
}

/* The paper's form, each function the plain definition (derivatives by the product rule,
 * not the paper's simplified A6-A8, which the tests use to check these). */
static double paper_f(const orc_paper *p, double r)
{
    return r < p->rc ? p->fe * pow(p->re / r, p->beta) : 0.0;
}

static double paper_df(const orc_paper *p, double r)
{
    /* d/dr fe (re/r)^beta = fe beta (re/r)^(beta-1) (-re/r^2) */
    return r < p->rc ? p->fe * p->beta * pow(p->re / r, p->beta - 1.0) * (-p->re / (r * r)) : 0.0;
}

static double paper_phi(const orc_paper *p, double r)
{
    double x = r / p->re;
    if (!(x < p->d)) return 0.0;
    double u = x - p->d;
    return u * u * (p->a3 * x * x * x + p->a2 * x * x + p->a1 * x + p->a0);
}

static double paper_dphi(const orc_paper *p, double r)
{
    double x = r / p->re;
    if (!(x < p->d)) return 0.0;
    double u = x - p->d;
    double poly = p->a3 * x * x * x + p->a2 * x * x + p->a1 * x + p->a0;
    double dpoly = 3.0 * p->a3 * x * x + 2.0 * p->a2 * x + p->a1;
    return (2.0 * u * poly + u * u * dpoly) / p->re;   /* dPhi/dx dx/dr */
}

static double paper_F(const orc_paper *p, double rho)
{
    if (!(rho > 0.0)) return 0.0;
    double t = rho / p->rho_e;
    return -p->Fo * (1.0 - p->n * log(t)) * pow(t, p->n);
}

static double paper_dF(const orc_paper *p, double rho)
{
    if (!(rho > 0.0)) return 0.0;   /* an atom without neighbours: taken as 0 */
    double t = rho / p->rho_e;
    /* product rule: d/drho of [1 - n ln t] is -n/rho; of t^n it is n t^n / rho */
    return -p->Fo * ((-p->n / rho) * pow(t, p->n) + (1.0 - p->n * log(t)) * p->n * pow(t, p->n) / rho);
}

static double paper_M(const orc_paper *p, double P)
{
    double u = P / p->P_e - 1.0;
    return p->alpha * u * u * exp(-u * u);
}

static double paper_dM(const orc_paper *p, double P)
{
    double u = P / p->P_e - 1.0;
    /* d/dP of u^2 exp(-u^2) = (2u exp(-u^2) + u^2 exp(-u^2) (-2u)) / P_e */
    return p->alpha * (2.0 * u * exp(-u * u) + u * u * exp(-u * u) * (-2.0 * u)) / p->P_e;
}

/* f, f', Phi, Phi', F, F', M, M' of the paper's form at one argument (r for the pair
 * functions, rho for F, P for M), for the tests. */
void orc_paper_values(const orc_paper *p, double r, double rho, double P, double out[8])
{
    out[0] = paper_f(p, r);
    out[1] = paper_df(p, r);
    out[2] = paper_phi(p, r);
    out[3] = paper_dphi(p, r);
    out[4] = paper_F(p, rho);
    out[5] = paper_dF(p, rho);
    out[6] = paper_M(p, P);
    out[7] = paper_dM(p, P);
}

/* ---------------------------------------------------------------------------------- */
/* Neumaier compensated sum                                                             */
/* ---------------------------------------------------------------------------------- */

typedef struct {
    double s, c;
} orc_sum;

static void sum_add(orc_sum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

static double sum_get(const orc_sum *a)
{
    return a->s + a->c;
}

/* ---------------------------------------------------------------------------------- */
/* Task 4: density, embedding derivative, forces, energies                              */
/* ---------------------------------------------------------------------------------- */

/*
 * Neighbour candidates of atom i: its list row when a list is given (row i of `nl`, cnt
 * entries), else every other atom.  The cutoff tests below make both give the same sums.
 */
#define FOR_CANDIDATES(i, jvar, ...)                                         \
    do {                                                                    \
        if (nl) {                                                           \
            for (int64_t t_ = 0; t_ < nlcnt[i]; ++t_) {                     \
                int64_t jvar = nl[(i)*nlcap + t_];                          \
                __VA_ARGS__                                                 \
            }                                                               \
        } else {                                                            \
            for (int64_t jvar = 0; jvar < n; ++jvar) {                      \
                if (jvar == (i)) continue;                                  \
                __VA_ARGS__                                                 \
            }                                                               \
        }                                                                   \
    } while (0)

/* First pass (Section 3.3.1.2): rho_i = sum_j f(r_ij) and F'(rho_i). */
void orc_density(const orc_box *b, const orc_eam *p, int64_t n, const double *x,
                 const int32_t *nlcnt, const int32_t *nl, int64_t nlcap,
                 double *rho, double *dF)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0, s[3];
        FOR_CANDIDATES(i, j, {
            double r = sqrt(separation(b, x + 3 * i, x + 3 * j, s));
            if (r < p->d) acc += dens_f(p, r);
        });
        rho[i] = acc;
        dF[i] = embed_dF(p, acc);
    }
}

/*
 * Second pass, Eq. (1):
 *   F_i = - sum_j [ (F'(rho_i) + F'(rho_j)) f'(r_ij) + phi'(r_ij) ] (q_i - q_j) / r_ij
 * with f' and phi' zero beyond their cutoffs.  Also returns, per atom, half the pair
 * energy sum_j phi(r_ij) / 2 and half the pair virial -1/2 sum_j (q_i-q_j)_a (F_ij)_b.
 */
void orc_eam_forces(const orc_box *b, const orc_eam *p, int64_t n, const double *x,
                    const int32_t *nlcnt, const int32_t *nl, int64_t nlcap,
                    const double *dF, double *f, double *epair, double *vir)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double fi[3] = {0.0, 0.0, 0.0}, e = 0.0, w[6] = {0, 0, 0, 0, 0, 0}, s[3];
        FOR_CANDIDATES(i, j, {
            double r = sqrt(separation(b, x + 3 * i, x + 3 * j, s));
            if (r < p->c) {
                double g = pair_dphi(p, r);
                if (r < p->d) g += (dF[i] + dF[j]) * dens_df(p, r);
                double qij[3] = {-s[0], -s[1], -s[2]};   /* q_i - q_j */
                double fij[3];
                for (int a = 0; a < 3; ++a) {
                    fij[a] = -g * qij[a] / r;
                    fi[a] += fij[a];
                }
                e += 0.5 * pair_phi(p, r);
                w[0] += 0.5 * qij[0] * fij[0];
                w[1] += 0.5 * qij[1] * fij[1];
                w[2] += 0.5 * qij[2] * fij[2];
                w[3] += 0.5 * qij[0] * fij[1];
                w[4] += 0.5 * qij[0] * fij[2];
                w[5] += 0.5 * qij[1] * fij[2];
            }
        });
        for (int a = 0; a < 3; ++a) f[3 * i + a] = fi[a];
        if (epair) epair[i] = e;
        if (vir)
            for (int a = 0; a < 6; ++a) vir[6 * i + a] = w[a];
    }
}

/* First pass with the paper's form: rho_i = sum_j f(r_ij), P_i = sum_j f(r_ij)^2 and the two
 * derivatives F'(rho_i), M'(P_i) (the paper's position + two-derivative array, Section 3.1). */
void orc_density_paper(const orc_box *b, const orc_paper *p, int64_t n, const double *x,
                       const int32_t *nlcnt, const int32_t *nl, int64_t nlcap,
                       double *rho, double *P, double *dF, double *dM)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0, accp = 0.0, s[3];
        FOR_CANDIDATES(i, j, {
            double r = sqrt(separation(b, x + 3 * i, x + 3 * j, s));
            if (r < p->rc) {
                double fr = paper_f(p, r);
                acc += fr;
                accp += fr * fr;
            }
        });
        rho[i] = acc;
        P[i] = accp;
        dF[i] = paper_dF(p, acc);
        dM[i] = paper_dM(p, accp);
    }
}

/*
 * Second pass with the paper's form: Eq. (1) with V = Phi and the M(P) term added the same
 * way (P_i and P_j both depend on r_ij through f^2):
 *   F_i = - sum_j [ (F'(rho_i) + F'(rho_j)) f'(r) + (M'(P_i) + M'(P_j)) 2 f(r) f'(r) + Phi'(r) ]
 *           (q_i - q_j) / r
 * Per-atom half pair energy and half virial as in orc_eam_forces.
 */
void orc_eam_forces_paper(const orc_box *b, const orc_paper *p, int64_t n, const double *x,
                          const int32_t *nlcnt, const int32_t *nl, int64_t nlcap,
                          const double *dF, const double *dM, double *f, double *epair, double *vir)
{
    const double rmax = p->rc > p->d * p->re ? p->rc : p->d * p->re;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double fi[3] = {0.0, 0.0, 0.0}, e = 0.0, w[6] = {0, 0, 0, 0, 0, 0}, s[3];
        FOR_CANDIDATES(i, j, {
            double r = sqrt(separation(b, x + 3 * i, x + 3 * j, s));
            if (r < rmax) {
                double fr = paper_f(p, r), dfr = paper_df(p, r);
                double g = paper_dphi(p, r) + (dF[i] + dF[j]) * dfr + (dM[i] + dM[j]) * 2.0 * fr * dfr;
                double qij[3] = {-s[0], -s[1], -s[2]};   /* q_i - q_j */
                double fij[3];
                for (int a = 0; a < 3; ++a) {
                    fij[a] = -g * qij[a] / r;
                    fi[a] += fij[a];
                }
                e += 0.5 * paper_phi(p, r);
                w[0] += 0.5 * qij[0] * fij[0];
                w[1] += 0.5 * qij[1] * fij[1];
                w[2] += 0.5 * qij[2] * fij[2];
                w[3] += 0.5 * qij[0] * fij[1];
                w[4] += 0.5 * qij[0] * fij[2];
                w[5] += 0.5 * qij[1] * fij[2];
            }
        });
        for (int a = 0; a < 3; ++a) f[3 * i + a] = fi[a];
        if (epair) epair[i] = e;
        if (vir)
            for (int a = 0; a < 6; ++a) vir[6 * i + a] = w[a];
    }
}

/*
 * Cr-C Morse: force on each Cr atom  F_i = - sum_k phiM'(r_ik) (q_i - q_k) / r_ik  for
 * r_ik < rc, written to fm; per-atom Morse energy sum_k [phiM(r_ik) - phiM(rc)].
 * Candidates: row i of the cross list when given, else every carbon atom.
 */
void orc_morse_forces(const orc_box *b, const orc_morse *m, int64_t n, const double *x,
                      int64_t nc, const double *xc, double ind_z,
                      const int32_t *xlcnt, const int32_t *xl, int64_t xlcap,
                      double *fm, double *em)
{
    const double shift = morse_phi(m, m->rc);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double fi[3] = {0.0, 0.0, 0.0}, e = 0.0, s[3], pk[3];
        int64_t ncand = xl ? xlcnt[i] : nc;
        for (int64_t t = 0; t < ncand; ++t) {
            int64_t k = xl ? xl[i * xlcap + t] : t;
            carbon_position(xc, k, ind_z, pk);
            double r = sqrt(separation(b, x + 3 * i, pk, s));
            if (r < m->rc) {
                double g = morse_dphi(m, r);
                for (int a = 0; a < 3; ++a) fi[a] += -g * (-s[a]) / r;
                e += morse_phi(m, r) - shift;
            }
        }
        for (int a = 0; a < 3; ++a) fm[3 * i + a] = fi[a];
        if (em) em[i] = e;
    }
}

/* ---------------------------------------------------------------------------------- */
/* Sampled evaluation for large systems: the full definition for chosen atoms only        */
/* ---------------------------------------------------------------------------------- */

static double density_at(const orc_box *b, const orc_eam *p, int64_t n, const double *x, int64_t i)
{
    double acc = 0.0, s[3];
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double r = sqrt(separation(b, x + 3 * i, x + 3 * j, s));
        if (r < p->d) acc += dens_f(p, r);
    }
    return acc;
}

/*
 * For each sampled atom i: rho_i, F'(rho_i) and the total force (Eq. (1) plus Morse),
 * each from all-atom loops.  rho_j of every neighbour j within d is recomputed from
 * scratch, so the result depends on nothing but the positions.
 */
void orc_sample_forces(const orc_box *b, const orc_eam *p, const orc_morse *m, int64_t n,
                       const double *x, int64_t nc, const double *xc, double ind_z,
                       int64_t ns, const int64_t *sample, double *f_out, double *rho_out,
                       double *dF_out, double *fm_out)
{
    const double shift = morse_phi(m, m->rc);
    (void)shift;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < ns; ++t) {
        int64_t i = sample[t];
        double rho_i = density_at(b, p, n, x, i);
        double dFi = embed_dF(p, rho_i);
        double fi[3] = {0.0, 0.0, 0.0}, s[3];
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double r = sqrt(separation(b, x + 3 * i, x + 3 * j, s));
            if (r < p->c) {
                double g = pair_dphi(p, r);
                if (r < p->d) g += (dFi + embed_dF(p, density_at(b, p, n, x, j))) * dens_df(p, r);
                for (int a = 0; a < 3; ++a) fi[a] += -g * (-s[a]) / r;
            }
        }
        double fmi[3] = {0.0, 0.0, 0.0}, pk[3];
        for (int64_t k = 0; k < nc; ++k) {
            carbon_position(xc, k, ind_z, pk);
            double r = sqrt(separation(b, x + 3 * i, pk, s));
            if (r < m->rc) {
                double g = morse_dphi(m, r);
                for (int a = 0; a < 3; ++a) fmi[a] += -g * (-s[a]) / r;
            }
        }
        for (int a = 0; a < 3; ++a) {
            f_out[3 * t + a] = fi[a] + fmi[a];
            if (fm_out) fm_out[3 * t + a] = fmi[a];
        }
        if (rho_out) rho_out[t] = rho_i;
        if (dF_out) dF_out[t] = dFi;
    }
}

/* rho_i and P_i of one atom with the paper's form, from all-atom loops. */
static void paper_density_at(const orc_box *b, const orc_paper *p, int64_t n, const double *x, int64_t i,
                             double *rho, double *P)
{
    double acc = 0.0, accp = 0.0, s[3];
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double r = sqrt(separation(b, x + 3 * i, x + 3 * j, s));
        if (r < p->rc) {
            double fr = paper_f(p, r);
            acc += fr;
            accp += fr * fr;
        }
    }
    *rho = acc;
    *P = accp;
}

/* orc_sample_forces with the paper's form: for each sampled atom, rho, F'(rho) and the total
 * force (the paper-form Eq. (1) plus Morse), each neighbour's rho and P recomputed from
 * scratch. */
void orc_sample_forces_paper(const orc_box *b, const orc_paper *p, const orc_morse *m, int64_t n,
                             const double *x, int64_t nc, const double *xc, double ind_z,
                             int64_t ns, const int64_t *sample, double *f_out, double *rho_out,
                             double *dF_out)
{
    const double rmax = p->rc > p->d * p->re ? p->rc : p->d * p->re;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < ns; ++t) {
        int64_t i = sample[t];
        double rho_i, P_i;
        paper_density_at(b, p, n, x, i, &rho_i, &P_i);
        double dFi = paper_dF(p, rho_i), dMi = paper_dM(p, P_i);
        double fi[3] = {0.0, 0.0, 0.0}, s[3];
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double r = sqrt(separation(b, x + 3 * i, x + 3 * j, s));
            if (r < rmax) {
                double rho_j = 0.0, P_j = 0.0;
                if (r < p->rc) paper_density_at(b, p, n, x, j, &rho_j, &P_j);
                double fr = paper_f(p, r), dfr = paper_df(p, r);
                double g = paper_dphi(p, r) + (dFi + paper_dF(p, rho_j)) * dfr +
                           (dMi + paper_dM(p, P_j)) * 2.0 * fr * dfr;
                for (int a = 0; a < 3; ++a) fi[a] += -g * (-s[a]) / r;
            }
        }
        double pk[3];
        for (int64_t k = 0; k < nc; ++k) {
            carbon_position(xc, k, ind_z, pk);
            double r = sqrt(separation(b, x + 3 * i, pk, s));
            if (r < m->rc) {
                double g = morse_dphi(m, r);
                for (int a = 0; a < 3; ++a) fi[a] += -g * (-s[a]) / r;
            }
        }
        for (int a = 0; a < 3; ++a) f_out[3 * t + a] = fi[a];
        if (rho_out) rho_out[t] = rho_i;
        if (dF_out) dF_out[t] = dFi;
    }
}

/* ---------------------------------------------------------------------------------- */
/* Whole-system evaluation and the time loop                                            */
/* ---------------------------------------------------------------------------------- */

typedef struct {
    orc_box box;
    orc_eam eam;
    orc_morse morse;
    double mass;     /* u */
    double dt;       /* fs */
    double v_ind;    /* indenter velocity along z, Angstrom/fs */
    double skin;     /* Angstrom */
    int32_t use_lists;   /* 0: all pairs; 1: forces over Verlet lists built by brute force;
                            2: the same lists built from a cell grid (large systems) */
    int32_t cap;         /* list capacity per atom when use_lists */
    int32_t potential;   /* 0: the synthetic potential `eam`; 1: the paper's form `paper` */
    int32_t pad;
    orc_paper paper;
} orc_params;

/* Largest cutoff of the Cr-Cr interaction (the Verlet list holds pairs within it + skin). */
static double cr_cutoff(const orc_params *P)
{
    if (P->potential == 1) return P->paper.rc > P->paper.d * P->paper.re ? P->paper.rc : P->paper.d * P->paper.re;
    return P->eam.c;
}

/* Energies and observables, in this order. */
enum {
    ORC_E_EMBED = 0, ORC_E_PAIR, ORC_E_MORSE, ORC_E_KIN,
    ORC_W_XX, ORC_W_YY, ORC_W_ZZ, ORC_W_XY, ORC_W_XZ, ORC_W_YZ,
    ORC_FIND_X, ORC_FIND_Y, ORC_FIND_Z, ORC_IND_Z, ORC_NBUILDS, ORC_NOBS = 16
};

typedef struct {
    int64_t n, nc;
    double *x, *v, *f;       /* [n][3] */
    const uint8_t *fixed;    /* [n] */
    const double *xc;        /* [nc][3] base carbon positions */
    double ind_z;            /* indenter displacement along z */
    /* list state */
    double *x_ref;           /* [n][3] positions at the last build */
    double ind_z_ref;
    int32_t *nlcnt, *nl;     /* [n], [n][cap] */
    int32_t *xlcnt, *xl;     /* [n], [n][cap] */
    int64_t nbuilds;
    int64_t overflow;        /* largest list count seen above cap (0 if none) */
    /* scratch */
    double *rho, *dF, *epair, *vir, *fm, *em;
    double *Pd, *dM;         /* P_i and M'(P_i) (paper's form) */
} orc_state;

/* Task 1: wrap periodic coordinates, record reference positions, rebuild the lists. */
static void build_lists(const orc_params *P, orc_state *S)
{
    orc_wrap(&P->box, S->n, S->x);
    memcpy(S->x_ref, S->x, (size_t)S->n * 3 * sizeof(double));
    S->ind_z_ref = S->ind_z;
    S->nbuilds++;
    if (P->use_lists == 2) {
        int64_t m1 = orc_neighbors_cells(&P->box, cr_cutoff(P) + P->skin, S->n, S->x, P->cap, S->nlcnt,
                                         S->nl);
        int64_t m2 = orc_cross_neighbors_cells(&P->box, P->morse.rc + P->skin, S->n, S->x, S->nc,
                                               S->xc, S->ind_z, P->cap, S->xlcnt, S->xl);
        int64_t mx = m1 > m2 ? m1 : m2;
        if (mx > P->cap && mx > S->overflow) S->overflow = mx;
    } else if (P->use_lists) {
        int64_t m1 = orc_neighbors(&P->box, cr_cutoff(P) + P->skin, S->n, S->x, 0, NULL, P->cap,
                                   S->nlcnt, S->nl);
        int64_t m2 = orc_cross_neighbors(&P->box, P->morse.rc + P->skin, S->n, S->x, S->nc,
                                         S->xc, S->ind_z, 0, NULL, P->cap, S->xlcnt, S->xl);
        int64_t mx = m1 > m2 ? m1 : m2;
        if (mx > P->cap && mx > S->overflow) S->overflow = mx;
    }
}

/* Section 2.6: the list is stale once any atom (or the indenter) moved more than skin/2. */
static int lists_stale(const orc_params *P, const orc_state *S)
{
    double lim = 0.5 * P->skin;
    if (fabs(S->ind_z - S->ind_z_ref) > lim) return 1;
    for (int64_t i = 0; i < S->n; ++i) {
        double d0 = S->x[3 * i] - S->x_ref[3 * i];
        double d1 = S->x[3 * i + 1] - S->x_ref[3 * i + 1];
        double d2 = S->x[3 * i + 2] - S->x_ref[3 * i + 2];
        if ((d0 * d0 + d1 * d1) + d2 * d2 > lim * lim) return 1;
    }
    return 0;
}

/* Task 4: density pass, then Eq. (1) forces and the Morse forces; observables in obs. */
static void compute_forces(const orc_params *P, orc_state *S, double *obs)
{
    const int32_t *nlc = P->use_lists ? S->nlcnt : NULL, *nl = P->use_lists ? S->nl : NULL;
    const int32_t *xlc = P->use_lists ? S->xlcnt : NULL, *xl = P->use_lists ? S->xl : NULL;
    if (P->potential == 1) {
        orc_density_paper(&P->box, &P->paper, S->n, S->x, nlc, nl, P->cap, S->rho, S->Pd, S->dF, S->dM);
        orc_eam_forces_paper(&P->box, &P->paper, S->n, S->x, nlc, nl, P->cap, S->dF, S->dM, S->f, S->epair,
                             S->vir);
    } else {
        orc_density(&P->box, &P->eam, S->n, S->x, nlc, nl, P->cap, S->rho, S->dF);
        orc_eam_forces(&P->box, &P->eam, S->n, S->x, nlc, nl, P->cap, S->dF, S->f, S->epair, S->vir);
    }
    orc_morse_forces(&P->box, &P->morse, S->n, S->x, S->nc, S->xc, S->ind_z, xlc, xl, P->cap,
                     S->fm, S->em);
    orc_sum e_emb = {0, 0}, e_pair = {0, 0}, e_m = {0, 0}, w[6], fi[3];
    memset(w, 0, sizeof w);
    memset(fi, 0, sizeof fi);
    for (int64_t i = 0; i < S->n; ++i) {
        for (int a = 0; a < 3; ++a) {
            S->f[3 * i + a] += S->fm[3 * i + a];
            sum_add(&fi[a], -S->fm[3 * i + a]);   /* load on the indenter */
        }
        if (P->potential == 1) {   /* the embedding and M(P) terms of Eq. (A1), per atom */
            sum_add(&e_emb, paper_F(&P->paper, S->rho[i]));
            sum_add(&e_emb, paper_M(&P->paper, S->Pd[i]));
        } else {
            sum_add(&e_emb, embed_F(&P->eam, S->rho[i]));
        }
        sum_add(&e_pair, S->epair[i]);
        sum_add(&e_m, S->em[i]);
        for (int a = 0; a < 6; ++a) sum_add(&w[a], S->vir[6 * i + a]);
    }
    if (obs) {
        obs[ORC_E_EMBED] = sum_get(&e_emb);
        obs[ORC_E_PAIR] = sum_get(&e_pair);
        obs[ORC_E_MORSE] = sum_get(&e_m);
        for (int a = 0; a < 6; ++a) obs[ORC_W_XX + a] = sum_get(&w[a]);
        for (int a = 0; a < 3; ++a) obs[ORC_FIND_X + a] = sum_get(&fi[a]);
    }
}

static double kinetic_energy(const orc_params *P, const orc_state *S)
{
    orc_sum k = {0, 0};
    for (int64_t i = 0; i < S->n; ++i) {
        if (S->fixed[i]) continue;
        double v2 = (S->v[3 * i] * S->v[3 * i] + S->v[3 * i + 1] * S->v[3 * i + 1]) +
                    S->v[3 * i + 2] * S->v[3 * i + 2];
        sum_add(&k, 0.5 * P->mass * v2);
    }
    return sum_get(&k) / orc_acc_factor();
}

static void alloc_state(orc_state *S, int64_t cap, int use_lists)
{
    int64_t n = S->n;
    S->x_ref = (double *)malloc(sizeof(double) * 3 * (n ? n : 1));
    S->rho = (double *)malloc(sizeof(double) * (n ? n : 1));
    S->dF = (double *)malloc(sizeof(double) * (n ? n : 1));
    S->epair = (double *)malloc(sizeof(double) * (n ? n : 1));
    S->vir = (double *)malloc(sizeof(double) * 6 * (n ? n : 1));
    S->fm = (double *)malloc(sizeof(double) * 3 * (n ? n : 1));
    S->em = (double *)malloc(sizeof(double) * (n ? n : 1));
    S->Pd = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
    S->dM = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
    if (use_lists) {
        S->nlcnt = (int32_t *)malloc(sizeof(int32_t) * (n ? n : 1));
        S->nl = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1) * cap);
        S->xlcnt = (int32_t *)malloc(sizeof(int32_t) * (n ? n : 1));
        S->xl = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1) * cap);
    }
}

static void free_state(orc_state *S)
{
    free(S->x_ref); free(S->rho); free(S->dF); free(S->epair); free(S->vir);
    free(S->fm); free(S->em); free(S->Pd); free(S->dM);
    free(S->nlcnt); free(S->nl); free(S->xlcnt); free(S->xl);
}

/*
 * Run `nsteps` velocity-Verlet steps in the order of Table 1, after an initial list
 * build and force evaluation at t = 0:
 *   Task 2  move the indenter by v_ind dt along z;
 *   Task 3  r(t+dt) = r + v dt + a dt^2 / 2  (A11),  v(t+dt/2) = v + a dt / 2  (A12);
 *   Task 1  rebuild the lists if stale (checked at the positions the forces are taken at);
 *   Task 4  forces and energies at t + dt  (A13: a = F / m);
 *   Task 5  v(t+dt) = v(t+dt/2) + a(t+dt) dt / 2.
 * Fixed atoms keep v = 0 and never move; their forces are still computed.
 * obs receives ORC_NOBS values for t = 0 and after every step ((nsteps+1) rows).
 * Positions are never wrapped except at list builds.  Returns 0, or the needed list
 * capacity if a list overflowed.
 */
int64_t orc_md_run(const orc_params *P, int64_t n, double *x, double *v, double *f,
                   const uint8_t *fixed, int64_t nc, const double *xc, double *ind_z,
                   int64_t nsteps, double *obs)
{
    orc_state S;
    memset(&S, 0, sizeof S);
    S.n = n; S.nc = nc; S.x = x; S.v = v; S.f = f; S.fixed = fixed; S.xc = xc;
    S.ind_z = *ind_z;
    alloc_state(&S, P->cap, P->use_lists);
    const double acc = orc_acc_factor() / P->mass;
    const double dt = P->dt;

    build_lists(P, &S);
    compute_forces(P, &S, obs);
    if (obs) {
        obs[ORC_E_KIN] = kinetic_energy(P, &S);
        obs[ORC_IND_Z] = S.ind_z;
        obs[ORC_NBUILDS] = (double)S.nbuilds;
    }
    for (int64_t step = 1; step <= nsteps; ++step) {
        S.ind_z += P->v_ind * dt;                                         /* Task 2 */
        for (int64_t i = 0; i < n; ++i) {                                 /* Task 3 */
            if (fixed[i]) continue;
            for (int a = 0; a < 3; ++a) {
                double ai = f[3 * i + a] * acc;
                x[3 * i + a] = x[3 * i + a] + v[3 * i + a] * dt + 0.5 * ai * dt * dt;
                v[3 * i + a] = v[3 * i + a] + 0.5 * ai * dt;
            }
        }
        if (lists_stale(P, &S)) build_lists(P, &S);                       /* Task 1 */
        double *o = obs ? obs + step * ORC_NOBS : NULL;
        compute_forces(P, &S, o);                                         /* Task 4 */
        for (int64_t i = 0; i < n; ++i) {                                 /* Task 5 */
            if (fixed[i]) continue;
            for (int a = 0; a < 3; ++a) v[3 * i + a] += 0.5 * f[3 * i + a] * acc * dt;
        }
        if (o) {
            o[ORC_E_KIN] = kinetic_energy(P, &S);
            o[ORC_IND_Z] = S.ind_z;
            o[ORC_NBUILDS] = (double)S.nbuilds;
        }
    }
    *ind_z = S.ind_z;
    int64_t ovf = S.overflow;
    free_state(&S);
    return ovf;
}

/* Forces, per-atom density and observables of one configuration (no time stepping). */
void orc_evaluate(const orc_params *P, int64_t n, const double *x, double *f, double *rho,
                  double *dF, int64_t nc, const double *xc, double ind_z, double *fm, double *obs,
                  double *Pout, double *dMout)
{
    orc_state S;
    memset(&S, 0, sizeof S);
    S.n = n; S.nc = nc; S.x = (double *)x; S.f = f; S.xc = xc; S.ind_z = ind_z;
    orc_params Q = *P;
    Q.use_lists = 0;
    alloc_state(&S, 1, 0);
    compute_forces(&Q, &S, obs);
    if (rho) memcpy(rho, S.rho, sizeof(double) * n);
    if (dF) memcpy(dF, S.dF, sizeof(double) * n);
    if (fm) memcpy(fm, S.fm, sizeof(double) * 3 * n);
    if (Pout) memcpy(Pout, S.Pd, sizeof(double) * n);
    if (dMout) memcpy(dMout, S.dM, sizeof(double) * n);
    free_state(&S);
}
