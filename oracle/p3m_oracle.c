/*
 * p3m_oracle.c -- plain, slow FP64 CPU oracle of the P3M force evaluation.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may call, link or
 * load this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it. It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * What it computes (Wyssling & Adelmann, "On Boundary Conditions in the
 * sub-mesh interaction of the P3M algorithm", arXiv 2103.02046):
 *
 *  - the Ewald split of the Coulomb kernel 1/r = erfc(a r)/r + erf(a r)/r
 *    (Sec. 2.2, eq. ewald_split); a is the split parameter;
 *  - the short-range (PP) force, summed directly over pairs closer than the
 *    cutoff r_c, with the particle itself omitted (Sec. 1, eq.
 *    summation_short; Sec. 2.2; Sec. 2.5, eq. eom_p3m_coord second term);
 *  - charge assignment to a vertex-centred mesh x_k = x0 + k h with cardinal
 *    B-splines (Sec. 2.4.2, eqs. grid_potential and
 *    interpolation_splines_b0: b1 = cloud-in-cell; b2 = triangular-shaped
 *    cloud, the next step of the same recursion);
 *  - the long-range potential as the aperiodic discrete convolution of the
 *    mesh charge with the erf(a r)/r kernel sampled on the mesh (Sec. 2.2,
 *    charge screening; Sec. 3, eq. phi_L with the free-space Green's
 *    function eq. free_gf);
 *  - the force on a particle as minus the gradient of its interpolation
 *    weights against the mesh potential (Sec. 2.5, eq. eom_p3m_coord first
 *    term and the finite-difference reading of dW/dxi that follows it).
 *
 * Units: SI. ke_q2 = k_e q^2 for the common macro-particle charge q; qw[i]
 * is an optional dimensionless per-particle charge weight (NULL = 1).
 * Mesh charge Q is in units of q; the mesh potential phi is in 1/m (the
 * physical potential is k_e q phi).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)
#define OR_EDOMAIN (-5)
#define OR_ENONFINITE (-6)

static const double OR_PI = 3.14159265358979323846;

static double qweight(const double *qw, int64_t i) { return qw ? qw[i] : 1.0; }

/* ------------------------------------------------------------------------
 * Placement of the mesh over the bunch.
 *
 * The paper puts the mesh on [0, L] with nodes x_k = k h (Sec. 2.4.2) and
 * says nothing about where the bunch sits or how the mesh follows it. The
 * reading used here: centre the mesh on the bounding box of the particles;
 * if the box is wider than the nodes an assignment stencil may touch
 * (N-1 nodes for CIC, N-2 for TSC), scale h, r_c by a common zoom s >= 1
 * and the split parameter by 1/s. Then every stencil lies on the mesh.
 *
 * out[0..2] = x0 (position of node 0), out[3] = s, out[4..6] = s*h.
 * ---------------------------------------------------------------------- */
int oracle_placement(int64_t n, const double *x, const int32_t *grid,
                     const double *h, int order, int zoom, int margin, double *out)
{
    if (n < 1 || (order != 1 && order != 2) || margin < 0) return OR_EINVAL;
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) { lo[d] = INFINITY; hi[d] = -INFINITY; }
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            double v = x[3 * i + d];
            if (!isfinite(v)) return OR_ENONFINITE;
            if (v < lo[d]) lo[d] = v;
            if (v > hi[d]) hi[d] = v;
        }
    double s = 1.0;
    for (int d = 0; d < 3; ++d) {
        double usable = (double)((order == 1 ? grid[d] - 1 : grid[d] - 2) - 2 * margin);
        if (usable <= 0) return OR_EINVAL;
        double need = (hi[d] - lo[d]) * (1.0 + 1e-6) / (usable * h[d]);
        if (need > s) s = need;
    }
    if (s > 1.0 && !zoom) return OR_EDOMAIN;
    for (int d = 0; d < 3; ++d) {
        double hp = s * h[d];
        double c = 0.5 * (lo[d] + hi[d]);
        out[d] = c - 0.5 * (double)(grid[d] - 1) * hp;
        out[4 + d] = hp;
    }
    out[3] = s;
    return OR_OK;
}

/* ------------------------------------------------------------------------
 * Short-range pair force (Sec. 2.2 eq. ewald_split, erfc part; Sec. 1 eq.
 * summation_short restricted to pairs with 0 < r < r_c).
 *   F_i += k_e q_i q_j [erfc(a r)/r + (2a/sqrt(pi)) exp(-a^2 r^2)] (x_i-x_j)/r^2
 * which is minus the gradient of k_e q_i q_j erfc(a r)/r.
 * ---------------------------------------------------------------------- */
static double pp_scalar(double r, double a)
{
    double ar = a * r;
    return (erfc(ar) / r + 2.0 * a / sqrt(OR_PI) * exp(-ar * ar)) / (r * r);
}

/* O(N^2): every ordered pair (i, j), j != i. */
void oracle_pp_brute(int64_t n, const double *x, const double *qw, double rc,
                     double a, double ke_q2, double *f)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double fx = 0, fy = 0, fz = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[3 * i] - x[3 * j];
            double dy = x[3 * i + 1] - x[3 * j + 1];
            double dz = x[3 * i + 2] - x[3 * j + 2];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (!(r2 > 0.0)) continue;           /* coincident particles */
            double r = sqrt(r2);
            if (!(r < rc)) continue;
            double g = ke_q2 * qweight(qw, i) * qweight(qw, j) * pp_scalar(r, a);
            fx += g * dx; fy += g * dy; fz += g * dz;
        }
        f[3 * i] = fx; f[3 * i + 1] = fy; f[3 * i + 2] = fz;
    }
}

/* Linked cells over the bounding box, cell edge >= rc. head[c] is the first
 * particle of cell c, next[i] the following one (-1 ends a list). */
typedef struct {
    double lo[3], cs[3];
    int64_t nc[3];
    int64_t *head, *next;
} cells_t;

static int cells_build(cells_t *c, int64_t n, const double *x, double rc)
{
    for (int d = 0; d < 3; ++d) { c->lo[d] = INFINITY; }
    double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            if (x[3 * i + d] < c->lo[d]) c->lo[d] = x[3 * i + d];
            if (x[3 * i + d] > hi[d]) hi[d] = x[3 * i + d];
        }
    int64_t total = 1;
    for (int d = 0; d < 3; ++d) {
        double w = hi[d] - c->lo[d];
        int64_t k = (int64_t)floor(w / rc);
        if (k < 1) k = 1;
        if (k > 1024) k = 1024;
        c->nc[d] = k;
        c->cs[d] = w > 0 ? w / (double)k : 1.0;
        total *= k;
    }
    c->head = (int64_t *)malloc(sizeof(int64_t) * total);
    c->next = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    if (!c->head || !c->next) { free(c->head); free(c->next); return OR_ENOMEM; }
    for (int64_t k = 0; k < total; ++k) c->head[k] = -1;
    /* insert in reverse so every list runs in increasing particle index */
    for (int64_t i = n - 1; i >= 0; --i) {
        int64_t id[3];
        for (int d = 0; d < 3; ++d) {
            int64_t k = (int64_t)floor((x[3 * i + d] - c->lo[d]) / c->cs[d]);
            if (k < 0) k = 0;
            if (k >= c->nc[d]) k = c->nc[d] - 1;
            id[d] = k;
        }
        int64_t cell = (id[2] * c->nc[1] + id[1]) * c->nc[0] + id[0];
        c->next[i] = c->head[cell];
        c->head[cell] = i;
    }
    return OR_OK;
}

static void cells_free(cells_t *c) { free(c->head); free(c->next); }

static int64_t cell_coord(const cells_t *c, const double *p, int d)
{
    int64_t k = (int64_t)floor((p[d] - c->lo[d]) / c->cs[d]);
    if (k < 0) k = 0;
    if (k >= c->nc[d]) k = c->nc[d] - 1;
    return k;
}

/* Force on particle i from every other particle within rc, via the cells. */
static void pp_one(const cells_t *c, const double *x, const double *qw,
                   int64_t i, double rc, double a, double ke_q2, double *out)
{
    double fx = 0, fy = 0, fz = 0;
    const double *pi = x + 3 * i;
    int64_t k0 = cell_coord(c, pi, 0), k1 = cell_coord(c, pi, 1), k2 = cell_coord(c, pi, 2);
    for (int64_t cz = (k2 > 0 ? k2 - 1 : 0); cz <= k2 + 1 && cz < c->nc[2]; ++cz)
        for (int64_t cy = (k1 > 0 ? k1 - 1 : 0); cy <= k1 + 1 && cy < c->nc[1]; ++cy)
            for (int64_t cx = (k0 > 0 ? k0 - 1 : 0); cx <= k0 + 1 && cx < c->nc[0]; ++cx) {
                int64_t cell = (cz * c->nc[1] + cy) * c->nc[0] + cx;
                for (int64_t j = c->head[cell]; j >= 0; j = c->next[j]) {
                    if (j == i) continue;
                    double dx = pi[0] - x[3 * j], dy = pi[1] - x[3 * j + 1], dz = pi[2] - x[3 * j + 2];
                    double r2 = dx * dx + dy * dy + dz * dz;
                    if (!(r2 > 0.0)) continue;
                    double r = sqrt(r2);
                    if (!(r < rc)) continue;
                    double g = ke_q2 * qweight(qw, i) * qweight(qw, j) * pp_scalar(r, a);
                    fx += g * dx; fy += g * dy; fz += g * dz;
                }
            }
    out[0] = fx; out[1] = fy; out[2] = fz;
}

/* Same pair set and force as oracle_pp_brute, found through linked cells. */
int oracle_pp_cells(int64_t n, const double *x, const double *qw, double rc,
                    double a, double ke_q2, double *f)
{
    if (n == 0) return OR_OK;
    cells_t c;
    int st = cells_build(&c, n, x, rc);
    if (st) return st;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) pp_one(&c, x, qw, i, rc, a, ke_q2, f + 3 * i);
    cells_free(&c);
    return OR_OK;
}

/* PP force on the particles listed in idx only (for sampled checks at full size). */
int oracle_pp_sample(int64_t n, const double *x, const double *qw, double rc,
                     double a, double ke_q2, int64_t m, const int64_t *idx, double *f)
{
    cells_t c;
    int st = cells_build(&c, n, x, rc);
    if (st) return st;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < m; ++k) pp_one(&c, x, qw, idx[k], rc, a, ke_q2, f + 3 * k);
    cells_free(&c);
    return OR_OK;
}

/* Short-range pair energy sum over unordered pairs of k_e q_i q_j erfc(a r)/r. */
double oracle_pp_energy(int64_t n, const double *x, const double *qw, double rc,
                        double a, double ke_q2)
{
    double e = 0.0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : e)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            double dx = x[3 * i] - x[3 * j], dy = x[3 * i + 1] - x[3 * j + 1],
                   dz = x[3 * i + 2] - x[3 * j + 2];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (!(r2 > 0.0)) continue;
            double r = sqrt(r2);
            if (!(r < rc)) continue;
            e += ke_q2 * qweight(qw, i) * qweight(qw, j) * erfc(a * r) / r;
        }
    return e;
}

/* ------------------------------------------------------------------------
 * Assignment weights (Sec. 2.4.2, eq. interpolation_splines_b0).
 * Particle at mesh coordinate u = (x - x0)/h'. The weight of node m is the
 * cardinal B-spline b_p(u - m): p = 1 (CIC) is the hat 1 - |t|, p = 2 (TSC)
 * is 3/4 - t^2 on |t| <= 1/2 and (3/2 - |t|)^2 / 2 on 1/2 <= |t| <= 3/2.
 * w[] gets the weights, dw[] their derivatives d b_p(u - m)/du, for the
 * stencil nodes base, base+1, ... (2 nodes CIC, 3 nodes TSC).
 * ---------------------------------------------------------------------- */
static int64_t stencil(int order, double u, int64_t nodes, double *w, double *dw)
{
    if (order == 1) {
        int64_t b = (int64_t)floor(u);
        if (b > nodes - 2) b = nodes - 2;      /* u == nodes-1 exactly */
        if (b < 0) b = 0;
        double t = u - (double)b;              /* distance to node b */
        w[0] = 1.0 - t;  dw[0] = -1.0;
        w[1] = t;        dw[1] = 1.0;
        return b;
    }
    int64_t c = (int64_t)floor(u + 0.5);       /* nearest node, ties up */
    double d = u - (double)c;                  /* in [-1/2, 1/2) */
    w[0] = 0.5 * (0.5 - d) * (0.5 - d);  dw[0] = -(0.5 - d);
    w[1] = 0.75 - d * d;                 dw[1] = -2.0 * d;
    w[2] = 0.5 * (0.5 + d) * (0.5 + d);  dw[2] = 0.5 + d;
    return c - 1;
}

/* Q_m = sum_i qw_i prod_d b_p(u_{i,d} - m_d) (Sec. 2.5, eq. eom_p3m_poiss_L
 * right-hand side; Sec. 3, eq. rho_L). Q is (grid[2], grid[1], grid[0])
 * row-major, x fastest, and is overwritten. */
int oracle_deposit(int64_t n, const double *x, const double *qw, const int32_t *grid,
                   const double *x0, const double *hp, int order, double *Q)
{
    int64_t nx = grid[0], ny = grid[1], nz = grid[2];
    memset(Q, 0, sizeof(double) * nx * ny * nz);
    int ns = order + 1;
    for (int64_t i = 0; i < n; ++i) {
        double w[3][3], dw[3][3];
        int64_t b[3];
        for (int d = 0; d < 3; ++d) {
            double u = (x[3 * i + d] - x0[d]) / hp[d];
            b[d] = stencil(order, u, grid[d], w[d], dw[d]);
            if (b[d] < 0 || b[d] + ns - 1 > grid[d] - 1) return OR_EDOMAIN;
        }
        double qi = qweight(qw, i);
        for (int c = 0; c < ns; ++c)
            for (int bb = 0; bb < ns; ++bb)
                for (int a = 0; a < ns; ++a)
                    Q[((b[2] + c) * ny + (b[1] + bb)) * nx + (b[0] + a)] +=
                        qi * w[0][a] * w[1][bb] * w[2][c];
    }
    return OR_OK;
}

/* Sampled long-range kernel between nodes offset by (i, j, k):
 * G = erf(a r)/r with r = |(i h'_x, j h'_y, k h'_z)|, and its limit 2a/sqrt(pi)
 * at r = 0 (Sec. 2.2: the erf part of the split; the screened charge rho (x)
 * gamma with the free-space Green's function). */
double oracle_green(int64_t i, int64_t j, int64_t k, const double *hp, double a)
{
    double rx = (double)i * hp[0], ry = (double)j * hp[1], rz = (double)k * hp[2];
    double r = sqrt(rx * rx + ry * ry + rz * rz);
    if (r == 0.0) return 2.0 * a / sqrt(OR_PI);
    return erf(a * r) / r;
}

/* phi_m = sum_m' G(m - m') Q_m', plain aperiodic O(M^2) sum over the mesh
 * (Sec. 3, eq. phi_L read as an aperiodic discrete convolution on the
 * mesh charge). */
void oracle_conv_direct(const int32_t *grid, const double *hp, double a,
                        const double *Q, double *phi)
{
    int64_t nx = grid[0], ny = grid[1], nz = grid[2];
    int64_t M = nx * ny * nz;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t m = 0; m < M; ++m) {
        int64_t mx = m % nx, my = (m / nx) % ny, mz = m / (nx * ny);
        double s = 0.0;
        for (int64_t k = 0; k < M; ++k) {
            if (Q[k] == 0.0) continue;
            int64_t kx = k % nx, ky = (k / nx) % ny, kz = k / (nx * ny);
            s += oracle_green(mx - kx, my - ky, mz - kz, hp, a) * Q[k];
        }
        phi[m] = s;
    }
}

/* The same sum, evaluated only at the listed node indices. */
void oracle_phi_at(const int32_t *grid, const double *hp, double a, const double *Q,
                   int64_t m, const int64_t *nodes, double *out)
{
    int64_t nx = grid[0], ny = grid[1], nz = grid[2];
    int64_t M = nx * ny * nz;
    for (int64_t t = 0; t < m; ++t) {
        int64_t node = nodes[t];
        int64_t mx = node % nx, my = (node / nx) % ny, mz = node / (nx * ny);
        double s = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : s)
        for (int64_t k = 0; k < M; ++k) {
            if (Q[k] == 0.0) continue;
            int64_t kx = k % nx, ky = (k / nx) % ny, kz = k / (nx * ny);
            s += oracle_green(mx - kx, my - ky, mz - kz, hp, a) * Q[k];
        }
        out[t] = s;
    }
}

/* Grounded plane z = zc (Sec. 3.1, eq. GreenFunc_planar_cathode with the
 * mirror map of eq. symmetry_planar_cathode): every node charge acts through
 * the screened kernel together with its mirror image of opposite sign.
 * Potential of the mesh charge at an arbitrary point y (mesh origin x0). */
static double green_r(double r, double a)
{
    if (r == 0.0) return 2.0 * a / sqrt(OR_PI);
    return erf(a * r) / r;
}

double oracle_phi_image_point(const int32_t *grid, const double *x0, const double *hp, double a,
                              double zc, const double *Q, const double *y)
{
    int64_t nx = grid[0], ny = grid[1], nz = grid[2];
    int64_t M = nx * ny * nz;
    double s = 0.0;
    for (int64_t k = 0; k < M; ++k) {
        if (Q[k] == 0.0) continue;
        int64_t kx = k % nx, ky = (k / nx) % ny, kz = k / (nx * ny);
        double px = x0[0] + kx * hp[0], py = x0[1] + ky * hp[1], pz = x0[2] + kz * hp[2];
        double mz = 2.0 * zc - pz;               /* S(p) */
        double dx = y[0] - px, dy = y[1] - py;
        double r1 = sqrt(dx * dx + dy * dy + (y[2] - pz) * (y[2] - pz));
        double r2 = sqrt(dx * dx + dy * dy + (y[2] - mz) * (y[2] - mz));
        s += Q[k] * (green_r(r1, a) - green_r(r2, a));
    }
    return s;
}

/* phi_m for every node by the plain O(M^2) sum with images. */
void oracle_conv_direct_image(const int32_t *grid, const double *x0, const double *hp, double a,
                              double zc, const double *Q, double *phi)
{
    int64_t nx = grid[0], ny = grid[1], nz = grid[2];
    int64_t M = nx * ny * nz;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t m = 0; m < M; ++m) {
        int64_t mx = m % nx, my = (m / nx) % ny, mz = m / (nx * ny);
        double y[3] = {x0[0] + mx * hp[0], x0[1] + my * hp[1], x0[2] + mz * hp[2]};
        phi[m] = oracle_phi_image_point(grid, x0, hp, a, zc, Q, y);
    }
}

/* Mesh nodes touched by particle i's stencil (for sampled checks). Returns
 * the count ((order+1)^3) and writes the linear node indices. */
int oracle_stencil_nodes(const double *xi, const int32_t *grid, const double *x0,
                         const double *hp, int order, int64_t *nodes)
{
    double w[3][3], dw[3][3];
    int64_t b[3];
    int ns = order + 1;
    for (int d = 0; d < 3; ++d) b[d] = stencil(order, (xi[d] - x0[d]) / hp[d], grid[d], w[d], dw[d]);
    int t = 0;
    for (int c = 0; c < ns; ++c)
        for (int bb = 0; bb < ns; ++bb)
            for (int a = 0; a < ns; ++a)
                nodes[t++] = ((b[2] + c) * (int64_t)grid[1] + (b[1] + bb)) * grid[0] + (b[0] + a);
    return t;
}

/* F_{i,d} = -k_e q^2 qw_i (1/h'_d) sum_m phi_m b_p'(u_d - m_d) prod_{e!=d} b_p(u_e - m_e)
 * (Sec. 2.5, eq. eom_p3m_coord first term: the gradient of the assignment
 * weight of each node against the mesh potential). Overwrites f. */
int oracle_gather(int64_t n, const double *x, const double *qw, const int32_t *grid,
                  const double *x0, const double *hp, int order, const double *phi,
                  double ke_q2, double *f)
{
    int64_t nx = grid[0], ny = grid[1];
    int ns = order + 1;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < n; ++i) {
        double w[3][3], dw[3][3];
        int64_t b[3];
        for (int d = 0; d < 3; ++d) {
            double u = (x[3 * i + d] - x0[d]) / hp[d];
            b[d] = stencil(order, u, grid[d], w[d], dw[d]);
            if (b[d] < 0 || b[d] + ns - 1 > grid[d] - 1) bad = 1;
        }
        if (bad) continue;
        double gx = 0, gy = 0, gz = 0;
        for (int c = 0; c < ns; ++c)
            for (int bb = 0; bb < ns; ++bb)
                for (int a = 0; a < ns; ++a) {
                    double ph = phi[((b[2] + c) * ny + (b[1] + bb)) * nx + (b[0] + a)];
                    gx += ph * dw[0][a] * w[1][bb] * w[2][c];
                    gy += ph * w[0][a] * dw[1][bb] * w[2][c];
                    gz += ph * w[0][a] * w[1][bb] * dw[2][c];
                }
        double s = -ke_q2 * qweight(qw, i);
        f[3 * i] = s * gx / hp[0];
        f[3 * i + 1] = s * gy / hp[1];
        f[3 * i + 2] = s * gz / hp[2];
    }
    return bad ? OR_EDOMAIN : OR_OK;
}

/* Momentum-conserving alternative to the variational force (the reading of
 * the remark after Sec. 2.5, eq. eom_p3m_coord that differences the mesh
 * potential first): the mesh field by central differences,
 *   E_{m,d} = -(phi_{m+e_d} - phi_{m-e_d}) / (2 h'_d),
 * interpolated with the assignment weights,
 *   F_{i,d} = k_e q^2 qw_i sum_m b_p(u_i - m) E_{m,d}.
 * Needs the stencil one node inside the mesh (placement margin 1); a
 * stencil touching the outer nodes is EDOMAIN. Overwrites f. */
int oracle_gather_momentum(int64_t n, const double *x, const double *qw, const int32_t *grid,
                           const double *x0, const double *hp, int order, const double *phi,
                           double ke_q2, double *f)
{
    int64_t nx = grid[0], ny = grid[1];
    int ns = order + 1;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < n; ++i) {
        double w[3][3], dw[3][3];
        int64_t b[3];
        for (int d = 0; d < 3; ++d) {
            double u = (x[3 * i + d] - x0[d]) / hp[d];
            b[d] = stencil(order, u, grid[d], w[d], dw[d]);
            if (b[d] < 1 || b[d] + ns - 1 > grid[d] - 2) bad = 1;
        }
        if (bad) continue;
        const int64_t step[3] = {1, nx, nx * ny};
        double e[3] = {0, 0, 0};
        for (int c = 0; c < ns; ++c)
            for (int bb = 0; bb < ns; ++bb)
                for (int a = 0; a < ns; ++a) {
                    int64_t m = ((b[2] + c) * ny + (b[1] + bb)) * nx + (b[0] + a);
                    double wm = w[0][a] * w[1][bb] * w[2][c];
                    for (int d = 0; d < 3; ++d)
                        e[d] += wm * -(phi[m + step[d]] - phi[m - step[d]]) / (2.0 * hp[d]);
                }
        double s = ke_q2 * qweight(qw, i);
        for (int d = 0; d < 3; ++d) f[3 * i + d] = s * e[d];
    }
    return bad ? OR_EDOMAIN : OR_OK;
}

/* ------------------------------------------------------------------------
 * Pieces of the adjoint (Hessian-vector products of the P3M potential).
 * The force is F = -dU/dx with U = U_PP + U_PM, so the Jacobian H = dF/dx is
 * symmetric and one product routine serves both the JVP and the VJP.
 * ---------------------------------------------------------------------- */

/* (H_PP v)_i = sum_j K_ij (v_i - v_j) with F_ij = k_e q_i q_j f(r) d, d = x_i-x_j,
 * K_ij = dF_ij/dx_i = f(r) I + (f'(r)/r) d d^T. f' is by differentiation of
 * f(r) = [erfc(a r)/r + (2a/sqrt(pi)) e^{-a^2 r^2}] / r^2. Brute force O(N^2). */
void oracle_pp_hvp(int64_t n, const double *x, const double *qw, double rc, double a,
                   double ke_q2, const double *v, double *out)
{
    const double c2 = 2.0 / sqrt(OR_PI);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double o[3] = {0, 0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3] = {x[3 * i] - x[3 * j], x[3 * i + 1] - x[3 * j + 1], x[3 * i + 2] - x[3 * j + 2]};
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (!(r2 > 0.0)) continue;
            double r = sqrt(r2);
            if (!(r < rc)) continue;
            double ar = a * r, e = exp(-ar * ar), ec = erfc(ar);
            /* g(r) = erfc(ar)/r + c2 a e ; f = g / r^2 */
            double g = ec / r + c2 * a * e;
            /* g'(r) = -erfc/r^2 - c2 a e / r - 2 c2 a^3 r e */
            double gp = -ec / r2 - c2 * a * e / r - 2.0 * c2 * a * a * a * r * e;
            double f = g / r2;
            double fp = gp / r2 - 2.0 * g / (r2 * r);
            double k = ke_q2 * qweight(qw, i) * qweight(qw, j);
            double dv[3] = {v[3 * i] - v[3 * j], v[3 * i + 1] - v[3 * j + 1], v[3 * i + 2] - v[3 * j + 2]};
            double dd = d[0] * dv[0] + d[1] * dv[1] + d[2] * dv[2];
            for (int c = 0; c < 3; ++c) o[c] += k * (f * dv[c] + fp / r * d[c] * dd);
        }
        out[3 * i] = o[0]; out[3 * i + 1] = o[1]; out[3 * i + 2] = o[2];
    }
}

/* R_m = sum_j qw_j grad W_m(x_j) . v_j : the mesh charge change under a
 * displacement v (derivative of the deposit). Overwrites R. */
int oracle_deposit_grad(int64_t n, const double *x, const double *qw, const int32_t *grid,
                        const double *x0, const double *hp, int order, const double *v,
                        double *R)
{
    int64_t nx = grid[0], ny = grid[1], nz = grid[2];
    memset(R, 0, sizeof(double) * nx * ny * nz);
    int ns = order + 1;
    for (int64_t i = 0; i < n; ++i) {
        double w[3][3], dw[3][3];
        int64_t b[3];
        for (int d = 0; d < 3; ++d) {
            b[d] = stencil(order, (x[3 * i + d] - x0[d]) / hp[d], grid[d], w[d], dw[d]);
            if (b[d] < 0 || b[d] + ns - 1 > grid[d] - 1) return OR_EDOMAIN;
        }
        double qi = qweight(qw, i);
        double vx = v[3 * i] / hp[0], vy = v[3 * i + 1] / hp[1], vz = v[3 * i + 2] / hp[2];
        for (int c = 0; c < ns; ++c)
            for (int bb = 0; bb < ns; ++bb)
                for (int a = 0; a < ns; ++a)
                    R[((b[2] + c) * ny + (b[1] + bb)) * nx + (b[0] + a)] +=
                        qi * (dw[0][a] * w[1][bb] * w[2][c] * vx +
                              w[0][a] * dw[1][bb] * w[2][c] * vy +
                              w[0][a] * w[1][bb] * dw[2][c] * vz);
    }
    return OR_OK;
}

/* (H_PM v)_i = -k_e q^2 qw_i [ sum_m psi_m grad W_m(x_i)
 *                              + sum_m phi_m (grad grad W_m(x_i)) v_i ]
 * with psi = G (x) R (R from oracle_deposit_grad). The second derivative of
 * the B-spline: CIC has none away from nodes (0); TSC has b2'' = 1, -2, 1. */
int oracle_gather_hvp(int64_t n, const double *x, const double *qw, const int32_t *grid,
                      const double *x0, const double *hp, int order, const double *phi,
                      const double *psi, const double *v, double ke_q2, double *out)
{
    int64_t nx = grid[0], ny = grid[1];
    int ns = order + 1;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < n; ++i) {
        double w[3][3], dw[3][3], d2[3][3];
        int64_t b[3];
        for (int d = 0; d < 3; ++d) {
            b[d] = stencil(order, (x[3 * i + d] - x0[d]) / hp[d], grid[d], w[d], dw[d]);
            if (b[d] < 0 || b[d] + ns - 1 > grid[d] - 1) bad = 1;
            if (order == 1) { d2[d][0] = 0; d2[d][1] = 0; d2[d][2] = 0; }
            else { d2[d][0] = 1.0; d2[d][1] = -2.0; d2[d][2] = 1.0; }
        }
        if (bad) continue;
        double gpsi[3] = {0, 0, 0};
        double hess[3][3] = {{0}};
        for (int c = 0; c < ns; ++c)
            for (int bb = 0; bb < ns; ++bb)
                for (int a = 0; a < ns; ++a) {
                    int64_t node = ((b[2] + c) * ny + (b[1] + bb)) * nx + (b[0] + a);
                    double ps = psi[node], ph = phi[node];
                    double W[3] = {w[0][a], w[1][bb], w[2][c]};
                    double D[3] = {dw[0][a], dw[1][bb], dw[2][c]};
                    double S[3] = {d2[0][a], d2[1][bb], d2[2][c]};
                    gpsi[0] += ps * D[0] * W[1] * W[2];
                    gpsi[1] += ps * W[0] * D[1] * W[2];
                    gpsi[2] += ps * W[0] * W[1] * D[2];
                    for (int p = 0; p < 3; ++p)
                        for (int q = 0; q < 3; ++q) {
                            double prod = 1.0;
                            for (int e = 0; e < 3; ++e) {
                                if (p == q && e == p) prod *= S[e];
                                else if (e == p || e == q) prod *= D[e];
                                else prod *= W[e];
                            }
                            hess[p][q] += ph * prod;
                        }
                }
        double s = -ke_q2 * qweight(qw, i);
        for (int p = 0; p < 3; ++p) {
            double acc = gpsi[p] / hp[p];
            for (int q = 0; q < 3; ++q) acc += hess[p][q] * v[3 * i + q] / (hp[p] * hp[q]);
            out[3 * i + p] = s * acc;
        }
    }
    return bad ? OR_EDOMAIN : OR_OK;
}

/* Number of OpenMP threads the oracle's parallel loops use. */
#ifdef _OPENMP
#include <omp.h>
int oracle_threads(void) { return omp_get_max_threads(); }
#else
int oracle_threads(void) { return 1; }
#endif
