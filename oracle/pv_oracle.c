/*
 * FP64 reference for the SPH density loop of the pseudo-Verlet paper.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the tests, the smoke check and the bench's CPU-baseline
 * leg load it; the product path never does.  It shares no code, header, table
 * or constant with the GPU library.
 *
 * What it computes is the plain definition of the quantities the paper's
 * neighbour loop produces (the paper's Fig. 1 caption: a density found as a
 * kernel-weighted sum over all neighbours closer than the cut-off h_i; the
 * in-range test of Listings 1-2 is the strict r < h):
 *
 *   Delta_ij = x_j - x_i - L round((x_j - x_i) / L)        (minimum image)
 *   r_ij     = |Delta_ij|,   H_i = GAMMA h_i,   u = r_ij / H_i
 *   w(u)  = 1 - 6u^2 + 6u^3   (0 <= u < 1/2),   2 (1-u)^3   (1/2 <= u < 1),  0 else
 *   w'(u) = -12u + 18u^2      (0 <= u < 1/2),  -6 (1-u)^2   (1/2 <= u < 1),  0 else
 *   W(r, H) = 8 / (pi H^3) w(r/H)                           (M4 cubic spline)
 *
 *   rho_i     = sum_{j : r_ij < H_i} m_j W(r_ij, H_i)           (j = i included)
 *   wcount_i  = sum_{j : r_ij < H_i} W(r_ij, H_i)               (j = i included)
 *   drho_dh_i = -8 / (pi H_i^3 h_i) sum_{j : r_ij < H_i} m_j [3 w(u) + u w'(u)]
 *   ncount_i  = #{ j != i : r_ij < H_i }
 *
 * and, for an upstream gradient G_i = dL/drho_i, the adjoint
 *
 *   dL/dh_k = G_k drho_dh_k
 *   dL/dx_k = sum_{j != k} [ G_k m_j W_r(r_kj, H_k) + G_j m_k W_r(r_kj, H_j) ]
 *                          (x_k - x_j)_mi / r_kj,      W_r = 8 / (pi H^4) w'(u)
 *
 * (terms with r >= H vanish and an r = 0 term is zero).
 *
 * The neighbour search is the cell list of the paper's Section 2 in its plain
 * form (Listing 1): cells of edge >= max cut-off, each receiver tests every
 * particle of the 27 surrounding cells.  No sorting and no pruning happen here;
 * the cell list only restricts the j range to a superset of the neighbours.
 * Everything is fp64; fp32 inputs are promoted exactly by the caller.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_GAMMA 1.825742
#define OR_PI 3.14159265358979323846

typedef struct {
    int64_t n;
    const double *x;   /* n*3, caller-owned, kept by reference */
    const double *h;   /* n */
    const double *m;   /* n */
    double L[3];
    int g[3];
    int64_t ncell;
    int64_t *start;    /* ncell + 1 */
    int64_t *items;    /* particle indices grouped by cell */
    int *cell_of;      /* n */
} or_grid;

/* M4 cubic spline in the support-radius form above. */
void or_kernel(double u, double *w, double *dw)
{
    if (u < 0.5) {
        *w = 1.0 - 6.0 * u * u + 6.0 * u * u * u;
        *dw = -12.0 * u + 18.0 * u * u;
    } else if (u < 1.0) {
        double v = 1.0 - u;
        *w = 2.0 * v * v * v;
        *dw = -6.0 * v * v;
    } else {
        *w = 0.0;
        *dw = 0.0;
    }
}

double or_gamma(void) { return OR_GAMMA; }

static int cell_coord(double x, double L, int g)
{
    double y = x - L * floor(x / L);
    int c = (int)floor(y / L * g);
    if (c < 0) c = 0;
    if (c >= g) c = g - 1;
    return c;
}

static void min_image(const or_grid *G, int64_t i, int64_t j, double d[3])
{
    for (int a = 0; a < 3; ++a) {
        double t = G->x[3 * j + a] - G->x[3 * i + a];
        d[a] = t - G->L[a] * nearbyint(t / G->L[a]);
    }
}

/* Returns NULL if the grid is illegal (fewer than 3 cells on an axis, or a cell
 * edge below the largest cut-off). */
or_grid *or_grid_build(int64_t n, const double *x, const double *h, const double *m,
                       const double L[3], const int g[3])
{
    double Hmax = 0.0;
    for (int64_t i = 0; i < n; ++i)
        if (OR_GAMMA * h[i] > Hmax) Hmax = OR_GAMMA * h[i];
    for (int a = 0; a < 3; ++a) {
        if (g[a] < 3) return NULL;
        if (L[a] / g[a] < Hmax) return NULL;
    }
    or_grid *G = (or_grid *)calloc(1, sizeof(or_grid));
    G->n = n; G->x = x; G->h = h; G->m = m;
    for (int a = 0; a < 3; ++a) { G->L[a] = L[a]; G->g[a] = g[a]; }
    G->ncell = (int64_t)g[0] * g[1] * g[2];
    G->start = (int64_t *)calloc((size_t)G->ncell + 1, sizeof(int64_t));
    G->items = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    G->cell_of = (int *)malloc(sizeof(int) * (size_t)(n ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        int cx = cell_coord(x[3 * i + 0], L[0], g[0]);
        int cy = cell_coord(x[3 * i + 1], L[1], g[1]);
        int cz = cell_coord(x[3 * i + 2], L[2], g[2]);
        int c = (cx * g[1] + cy) * g[2] + cz;
        G->cell_of[i] = c;
        G->start[c + 1]++;
    }
    for (int64_t c = 0; c < G->ncell; ++c) G->start[c + 1] += G->start[c];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)G->ncell);
    memcpy(fill, G->start, sizeof(int64_t) * (size_t)G->ncell);
    for (int64_t i = 0; i < n; ++i) G->items[fill[G->cell_of[i]]++] = i;
    free(fill);
    return G;
}

void or_grid_free(or_grid *G)
{
    if (!G) return;
    free(G->start); free(G->items); free(G->cell_of); free(G);
}

/* The 27 distinct cells around cell c (the grid has >= 3 cells per axis). */
static void stencil(const or_grid *G, int c, int out[27])
{
    int cz = c % G->g[2], cy = (c / G->g[2]) % G->g[1], cx = c / (G->g[2] * G->g[1]);
    int k = 0;
    for (int ox = -1; ox <= 1; ++ox)
        for (int oy = -1; oy <= 1; ++oy)
            for (int oz = -1; oz <= 1; ++oz) {
                int bx = (cx + ox + G->g[0]) % G->g[0];
                int by = (cy + oy + G->g[1]) % G->g[1];
                int bz = (cz + oz + G->g[2]) % G->g[2];
                out[k++] = (bx * G->g[1] + by) * G->g[2] + bz;
            }
}

/* for every particle j of the 27 cells around particle i's cell */
#define FOR_STENCIL(G, i, ...)                                                    \
    do {                                                                          \
        int cells_[27];                                                           \
        stencil((G), (G)->cell_of[i], cells_);                                    \
        for (int s_ = 0; s_ < 27; ++s_)                                           \
            for (int64_t q_ = (G)->start[cells_[s_]];                             \
                 q_ < (G)->start[cells_[s_] + 1]; ++q_) {                         \
                int64_t j = (G)->items[q_];                                       \
                __VA_ARGS__                                                       \
            }                                                                     \
    } while (0)

/* Density of receiver i.  S_dh = sum of |m_j (3w + u w')| times the prefactor
 * magnitude: the scale against which the signed drho_dh is compared. */
static void density_one(const or_grid *G, int64_t i, double *rho, double *wc,
                        double *dh, int64_t *cnt, double *dh_abs)
{
    double H = OR_GAMMA * G->h[i];
    double s_rho = 0, s_wc = 0, s_dh = 0, s_abs = 0;
    int64_t c = 0;
    FOR_STENCIL(G, i, {
        double d[3];
        min_image(G, i, j, d);
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (r < H) {
            double u = r / H, w, dw;
            or_kernel(u, &w, &dw);
            s_rho += G->m[j] * w;
            s_wc += w;
            s_dh += G->m[j] * (3.0 * w + u * dw);
            s_abs += fabs(G->m[j] * (3.0 * w + u * dw));
            if (j != i) c++;
        }
    });
    double norm = 8.0 / (OR_PI * H * H * H);
    *rho = norm * s_rho;
    *wc = norm * s_wc;
    *dh = -norm / G->h[i] * s_dh;
    *dh_abs = norm / G->h[i] * s_abs;
    *cnt = c;
}

/* recv == NULL: every particle, outputs indexed by particle.  Otherwise outputs
 * are indexed by position in recv[]. Any output pointer may be NULL. */
void or_density(const or_grid *G, const int64_t *recv, int64_t nrecv, double *rho,
                double *wcount, double *drho_dh, int64_t *ncount, double *dh_abs)
{
    int64_t nr = recv ? nrecv : G->n;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t k = 0; k < nr; ++k) {
        int64_t i = recv ? recv[k] : k;
        double a, b, c, e;
        int64_t n;
        density_one(G, i, &a, &b, &c, &n, &e);
        if (rho) rho[k] = a;
        if (wcount) wcount[k] = b;
        if (drho_dh) drho_dh[k] = c;
        if (ncount) ncount[k] = n;
        if (dh_abs) dh_abs[k] = e;
    }
}

/* Adjoint of rho for upstream gradient Gr (length n, particle order).
 * gx: nrecv*3, gh: nrecv, gx_abs: nrecv*3 (sum of |terms| per component). */
void or_density_grad(const or_grid *G, const double *Gr, const int64_t *recv,
                     int64_t nrecv, double *gx, double *gh, double *gx_abs, double *gh_abs)
{
    int64_t nr = recv ? nrecv : G->n;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t q = 0; q < nr; ++q) {
        int64_t k = recv ? recv[q] : q;
        double Hk = OR_GAMMA * G->h[k];
        double acc[3] = {0, 0, 0}, aab[3] = {0, 0, 0};
        FOR_STENCIL(G, k, {
            if (j != k) {
                double d[3];
                min_image(G, k, j, d);             /* d = x_j - x_k */
                double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                double Hj = OR_GAMMA * G->h[j];
                if (r > 0.0 && (r < Hk || r < Hj)) {
                    double coef = 0.0, w, dw;
                    if (r < Hk) {
                        or_kernel(r / Hk, &w, &dw);
                        coef += Gr[k] * G->m[j] * 8.0 / (OR_PI * Hk * Hk * Hk * Hk) * dw;
                    }
                    if (r < Hj) {
                        or_kernel(r / Hj, &w, &dw);
                        coef += Gr[j] * G->m[k] * 8.0 / (OR_PI * Hj * Hj * Hj * Hj) * dw;
                    }
                    for (int a = 0; a < 3; ++a) {
                        double t = coef * (-d[a]) / r;  /* (x_k - x_j) / r */
                        acc[a] += t;
                        aab[a] += fabs(t);
                    }
                }
            }
        });
        for (int a = 0; a < 3; ++a) {
            if (gx) gx[3 * q + a] = acc[a];
            if (gx_abs) gx_abs[3 * q + a] = aab[a];
        }
        double rho, wc, dh, dabs;
        int64_t c;
        density_one(G, k, &rho, &wc, &dh, &c, &dabs);
        if (gh) gh[q] = Gr[k] * dh;
        if (gh_abs) gh_abs[q] = fabs(Gr[k]) * dabs;
    }
}

/* rho_i with particle k's coordinate `comp` (0..2 position, 3 smoothing length)
 * replaced by `val`; everything else as in the grid.  Used for finite
 * differences, where the perturbed value is fp64 and not representable in the
 * fp32 inputs. */
static double rho_with(const or_grid *G, int64_t i, int64_t k, int comp, double val)
{
    double hi = (i == k && comp == 3) ? val : G->h[i];
    double H = OR_GAMMA * hi;
    double xi[3] = {G->x[3 * i], G->x[3 * i + 1], G->x[3 * i + 2]};
    if (i == k && comp < 3) xi[comp] = val;
    double s = 0.0;
    FOR_STENCIL(G, i, {
        double xj[3] = {G->x[3 * j], G->x[3 * j + 1], G->x[3 * j + 2]};
        if (j == k && comp < 3) xj[comp] = val;
        double d2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            double t = xj[a] - xi[a];
            t -= G->L[a] * nearbyint(t / G->L[a]);
            d2 += t * t;
        }
        double r = sqrt(d2);
        if (r < H) {
            double w, dw;
            or_kernel(r / H, &w, &dw);
            s += G->m[j] * w;
        }
    });
    return 8.0 / (OR_PI * H * H * H) * s;
}

/* Central difference of L = sum_i (rho_i - t_i)^2 with respect to coordinate
 * `comp` of particle k (0..2 = x,y,z; 3 = h), step eps, in fp64.  Only the
 * receivers whose density can change are re-evaluated: k itself and every i
 * whose cut-off sphere, widened by eps, reaches k.  Requires eps small enough
 * that k stays within the 27-cell stencil of its own cell. */
double or_fd_loss(const or_grid *G, const double *target, int64_t k, int comp, double eps)
{
    double x0 = comp < 3 ? G->x[3 * k + comp] : G->h[k];
    double lp = 0.0, lm = 0.0;
    /* receiver k */
    {
        double rp = rho_with(G, k, k, comp, x0 + eps) - target[k];
        double rm = rho_with(G, k, k, comp, x0 - eps) - target[k];
        lp += rp * rp;
        lm += rm * rm;
    }
    if (comp < 3) {
        FOR_STENCIL(G, k, {
            if (j != k) {
                double d[3];
                min_image(G, k, j, d);
                double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                if (r < OR_GAMMA * G->h[j] + 2.0 * eps) {
                    double rp = rho_with(G, j, k, comp, x0 + eps) - target[j];
                    double rm = rho_with(G, j, k, comp, x0 - eps) - target[j];
                    lp += rp * rp;
                    lm += rm * rm;
                }
            }
        });
    }
    return (lp - lm) / (2.0 * eps);
}

/* Same central difference, one call per (k, comp) pair of the arrays. */
void or_fd_loss_many(const or_grid *G, const double *target, const int64_t *ks,
                     const int *comps, const double *eps, int64_t m, double *out)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < m; ++q) out[q] = or_fd_loss(G, target, ks[q], comps[q], eps[q]);
}

/*
 * Smoothing lengths from the density-smoothing-length relation
 *
 *   rho_i(h_i) h_i^3 = m_i eta^3,
 *
 * where rho_i(h) is the density of receiver i with its own cut-off gamma h and
 * everything else fixed (rho_i depends on no other particle's h, so the
 * particles' equations are independent).  With equal masses this is the
 * neighbour-number condition (4 pi / 3) H_i^3 wcount_i = N_ngb with
 * eta^3 = 3 N_ngb / (4 pi gamma^3).  g(h) = rho_i(h) h^3 - m_i eta^3 grows with
 * h (every kernel term w(r / gamma h) grows with h, and new terms enter at
 * w = 0), so the root is found by plain bisection in fp64 on [h_lo_i, h_hi_i].
 * The grid G must be built with h = h_hi (its stencil then holds every
 * candidate).  Returns the number of particles whose bracket holds no sign
 * change (their h_out is left at -1).
 */
static double rho_at(const double *rj, const double *mj, int64_t k, double h)
{
    double H = OR_GAMMA * h, s = 0.0;
    for (int64_t q = 0; q < k; ++q)
        if (rj[q] < H) {
            double w, dw;
            or_kernel(rj[q] / H, &w, &dw);
            s += mj[q] * w;
        }
    return 8.0 / (OR_PI * H * H * H) * s;
}

int64_t or_solve_h(const or_grid *G, double eta, const double *h_lo, double *h_out)
{
    int64_t bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : bad)
    for (int64_t i = 0; i < G->n; ++i) {
        /* the distances and masses of every candidate within the bracket */
        const double Hhi = OR_GAMMA * G->h[i];
        int64_t cap = 64, k = 0;
        double *rj = (double *)malloc(sizeof(double) * cap);
        double *mj = (double *)malloc(sizeof(double) * cap);
        FOR_STENCIL(G, i, {
            double d[3];
            min_image(G, i, j, d);
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (r < Hhi) {
                if (k == cap) {
                    cap *= 2;
                    rj = (double *)realloc(rj, sizeof(double) * cap);
                    mj = (double *)realloc(mj, sizeof(double) * cap);
                }
                rj[k] = r;
                mj[k] = G->m[j];
                ++k;
            }
        });
        const double target = G->m[i] * eta * eta * eta;
        double lo = h_lo[i], hi = G->h[i];
        double glo = rho_at(rj, mj, k, lo) * lo * lo * lo - target;
        double ghi = rho_at(rj, mj, k, hi) * hi * hi * hi - target;
        if (!(glo < 0.0 && ghi > 0.0)) {
            h_out[i] = -1.0;
            ++bad;
        } else {
            for (int it = 0; it < 200 && hi - lo > 1e-14 * hi; ++it) {
                double mid = 0.5 * (lo + hi);
                double g = rho_at(rj, mj, k, mid) * mid * mid * mid - target;
                if (g < 0.0) lo = mid; else hi = mid;
            }
            h_out[i] = 0.5 * (lo + hi);
        }
        free(rj);
        free(mj);
    }
    return bad;
}

/*
 * Lennard-Jones forces and energies over the same neighbour sets (the paper's
 * introduction: the pseudo-Verlet list serves molecular dynamics as well as
 * SPH).  For every pair with r_ij < H_i (H_i = GAMMA h_i, the receiver's
 * cut-off):
 *
 *   U(r) = 4 eps [ (sigma/r)^12 - (sigma/r)^6 ]
 *   F_i  = sum_j (24 eps / r^2) [ 2 (sigma/r)^12 - (sigma/r)^6 ] (x_i - x_j)_mi
 *   E_i  = 1/2 sum_j U(r_ij)          (so that sum_i E_i is the total energy
 *                                      when every cut-off is the same)
 *
 * f_abs and e_abs (may be NULL) receive the sums of the terms' magnitudes per
 * force component and for the energy: the scales against which the signed
 * sums are compared.
 */
void or_lj(const or_grid *G, double eps, double sigma, const int64_t *recv, int64_t nrecv,
           double *force, double *energy, double *f_abs, double *e_abs)
{
    int64_t nr = recv ? nrecv : G->n;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t q = 0; q < nr; ++q) {
        int64_t i = recv ? recv[q] : q;
        double H = OR_GAMMA * G->h[i];
        double f[3] = {0, 0, 0}, fa[3] = {0, 0, 0}, e = 0.0, ea = 0.0;
        FOR_STENCIL(G, i, {
            if (j != i) {
                double d[3];
                min_image(G, i, j, d);      /* d = x_j - x_i */
                double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                if (sqrt(r2) < H) {
                    double s2 = sigma * sigma / r2, s6 = s2 * s2 * s2, s12 = s6 * s6;
                    double c = 24.0 * eps / r2 * (2.0 * s12 - s6);
                    for (int a = 0; a < 3; ++a) {
                        f[a] -= c * d[a];
                        fa[a] += fabs(c * d[a]);
                    }
                    e += 2.0 * eps * (s12 - s6);
                    ea += fabs(2.0 * eps * (s12 - s6));
                }
            }
        });
        for (int a = 0; a < 3; ++a) {
            force[3 * q + a] = f[a];
            if (f_abs) f_abs[3 * q + a] = fa[a];
        }
        energy[q] = e;
        if (e_abs) e_abs[q] = ea;
    }
}

/* Total energy sum_i E_i with particle k's coordinate `comp` (0..2) moved by
 * delta, in fp64: for force = -dE/dx checks by central differences.  Every
 * receiver is re-evaluated (small sets only). */
double or_lj_energy_moved(const or_grid *G, double eps, double sigma, int64_t k, int comp,
                          double delta)
{
    double tot = 0.0;
#pragma omp parallel for reduction(+ : tot) schedule(dynamic, 64)
    for (int64_t i = 0; i < G->n; ++i) {
        double H = OR_GAMMA * G->h[i];
        double xi[3] = {G->x[3 * i], G->x[3 * i + 1], G->x[3 * i + 2]};
        if (i == k) xi[comp] += delta;
        double e = 0.0;
        for (int64_t j = 0; j < G->n; ++j) {
            if (j == i) continue;
            double r2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                double t = G->x[3 * j + a] + ((j == k && a == comp) ? delta : 0.0) - xi[a];
                t -= G->L[a] * nearbyint(t / G->L[a]);
                r2 += t * t;
            }
            if (sqrt(r2) < H) {
                double s2 = sigma * sigma / r2, s6 = s2 * s2 * s2;
                e += 2.0 * eps * (s6 * s6 - s6);
            }
        }
        tot += e;
    }
    return tot;
}
