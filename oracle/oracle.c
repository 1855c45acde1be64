/*
 * Plain FP64 CPU oracle of one explicit electromagnetic PIC step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can compare the HIP library against an
 * independent, slow, obviously correct implementation.  It shares no code,
 * header, table or constant with the HIP path.
 *
 * The method is the paper's (Sec. 2): the Vlasov-Maxwell system (eq. 1) is
 * sampled by macro-particles with a compact shape g (eq. 2); particles follow
 * eq. (3) advanced with leap-frog and the relativistic Boris rotation; the
 * current (eq. 4) is deposited in a charge-conserving way; E and B follow the
 * two curl equations on the Yee lattice (FDTD).  Units: c = eps0 = 1, charge
 * in units of e, mass in units of m_e, u = p/(m c), v = u/gamma.
 *
 * Everything is FP64, scalar loops, periodic (modulo) indexing, no guard
 * cells, no tiles.  Build with -O2 -ffp-contract=off.
 *
 * Conventions fixed here because the paper does not state them:
 *  - Yee staggering: Ex(i+1/2,j,k) Ey(i,j+1/2,k) Ez(i,j,k+1/2),
 *    Bx(i,j+1/2,k+1/2) By(i+1/2,j,k+1/2) Bz(i+1/2,j+1/2,k); J sits with E,
 *    rho on nodes.  In 2D the z index is dropped.
 *  - Array index [k][j][i] (x fastest) holds the component whose position is
 *    its staggered point with integer base (i,j,k).
 *  - Shapes are B-splines of order 1 (linear) or 2 (quadratic), in cell units.
 *  - A particle position is an integer cell index per dimension plus an
 *    offset in [0,1) (x = (cell + off) * dx).
 *  - Time levels: x, E, B at n; u at n-1/2 -> n+1/2; J at n+1/2.
 *  - Charge conservation follows Esirkepov, Comput. Phys. Commun. 135 (2001)
 *    144; the pusher is Boris (1970) in its relativistic form; the field
 *    solver is Yee (1966).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t dims;    /* 2 or 3 (velocities always have 3 components) */
    int32_t n[3];    /* cells per dimension; n[2] == 1 when dims == 2 */
    double dx[3];    /* cell size per dimension (dx[2] ignored in 2D) */
    double dt;       /* time step */
    int32_t order;   /* shape order: 1 = linear, 2 = quadratic */
} or_grid;

/* ------------------------------------------------------------------ */
/* Shape functions (Sec. 2: compact, positive definite g).             */
/* ------------------------------------------------------------------ */

double or_shape(int32_t order, double xi)
{
    double a = fabs(xi);
    if (order == 1) {
        return a < 1.0 ? 1.0 - a : 0.0;
    }
    if (order == 2) {
        if (a <= 0.5) return 0.75 - a * a;
        if (a < 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
        return 0.0;
    }
    return NAN;
}

static int64_t wrap(int64_t i, int64_t n)
{
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

static int64_t lin(const or_grid *g, int64_t i, int64_t j, int64_t k)
{
    return wrap(i, g->n[0]) + (int64_t)g->n[0] * (wrap(j, g->n[1]) + (int64_t)g->n[1] * wrap(k, g->n[2]));
}

static double cell_volume(const or_grid *g)
{
    return g->dims == 3 ? g->dx[0] * g->dx[1] * g->dx[2] : g->dx[0] * g->dx[1];
}

/* Stagger (in cell units) of each field component along each dimension,
 * component order Ex Ey Ez Bx By Bz. */
static const double STAG[6][3] = {
    {0.5, 0.0, 0.0}, {0.0, 0.5, 0.0}, {0.0, 0.0, 0.5},
    {0.0, 0.5, 0.5}, {0.5, 0.0, 0.5}, {0.5, 0.5, 0.0},
};

/* ------------------------------------------------------------------ */
/* Gather: field at the particle = sum over grid points of the field    */
/* weighted by the shape centred on the particle (Sec. 2).              */
/* ------------------------------------------------------------------ */

/* Field component c at one particle, summing the shape over the points
 * within two cells of the particle (the support of order <= 2 shapes). */
static double gather_one(const or_grid *g, const double *F, int c, const int32_t cell[3], const double off[3])
{
    double sum = 0.0;
    int kmax = g->dims == 3 ? 2 : 0;
    int kmin = g->dims == 3 ? -2 : 0;
    for (int dk = kmin; dk <= kmax; ++dk) {
        double wz = 1.0;
        if (g->dims == 3) wz = or_shape(g->order, ((double)(-dk) - STAG[c][2]) + off[2]);
        if (wz == 0.0) continue;
        for (int dj = -2; dj <= 2; ++dj) {
            double wy = or_shape(g->order, ((double)(-dj) - STAG[c][1]) + off[1]);
            if (wy == 0.0) continue;
            for (int di = -2; di <= 2; ++di) {
                double wx = or_shape(g->order, ((double)(-di) - STAG[c][0]) + off[0]);
                if (wx == 0.0) continue;
                int64_t idx = lin(g, (int64_t)cell[0] + di, (int64_t)cell[1] + dj,
                                  g->dims == 3 ? (int64_t)cell[2] + dk : 0);
                sum += F[idx] * (wx * wy * wz);
            }
        }
    }
    return sum;
}

/* out[c*np + p] = component c (Ex Ey Ez Bx By Bz) at particle p. */
void or_gather(const or_grid *g, const double *Ex, const double *Ey, const double *Ez,
               const double *Bx, const double *By, const double *Bz, int64_t np,
               const int32_t *ix, const int32_t *iy, const int32_t *iz,
               const double *ox, const double *oy, const double *oz, double *out)
{
    const double *F[6] = {Ex, Ey, Ez, Bx, By, Bz};
    for (int64_t p = 0; p < np; ++p) {
        int32_t cell[3] = {ix[p], iy[p], g->dims == 3 ? iz[p] : 0};
        double off[3] = {ox[p], oy[p], g->dims == 3 ? oz[p] : 0.0};
        for (int c = 0; c < 6; ++c) out[(int64_t)c * np + p] = gather_one(g, F[c], c, cell, off);
    }
}

/* Brute force: the same average taken over every grid point of the periodic
 * box with minimum-image distances (for tiny grids). */
void or_gather_bruteforce(const or_grid *g, const double *Ex, const double *Ey, const double *Ez,
                          const double *Bx, const double *By, const double *Bz, int64_t np,
                          const int32_t *ix, const int32_t *iy, const int32_t *iz,
                          const double *ox, const double *oy, const double *oz, double *out)
{
    const double *F[6] = {Ex, Ey, Ez, Bx, By, Bz};
    for (int64_t p = 0; p < np; ++p) {
        double pos[3] = {ix[p] + ox[p], iy[p] + oy[p], g->dims == 3 ? iz[p] + oz[p] : 0.0};
        for (int c = 0; c < 6; ++c) {
            double sum = 0.0;
            for (int64_t k = 0; k < g->n[2]; ++k)
                for (int64_t j = 0; j < g->n[1]; ++j)
                    for (int64_t i = 0; i < g->n[0]; ++i) {
                        int64_t node[3] = {i, j, k};
                        double w = 1.0;
                        for (int d = 0; d < g->dims; ++d) {
                            double r = pos[d] - ((double)node[d] + STAG[c][d]);
                            double L = (double)g->n[d];
                            while (r > 0.5 * L) r -= L;
                            while (r <= -0.5 * L) r += L;
                            w *= or_shape(g->order, r);
                        }
                        sum += F[c][i + g->n[0] * (j + g->n[1] * k)] * w;
                    }
            out[(int64_t)c * np + p] = sum;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Relativistic Boris rotation (leap-frog, Sec. 2 ref. [8]).            */
/* u is advanced from n-1/2 to n+1/2 in place; Ep/Bp laid out [6][np].  */
/* ------------------------------------------------------------------ */

void or_boris(int64_t np, double q, double m, double dt, const double *EB,
              double *ux, double *uy, double *uz)
{
    double h = q * dt / (2.0 * m);
    for (int64_t p = 0; p < np; ++p) {
        double E[3] = {EB[p], EB[np + p], EB[2 * np + p]};
        double B[3] = {EB[3 * np + p], EB[4 * np + p], EB[5 * np + p]};
        /* first half electric kick */
        double um[3] = {ux[p] + h * E[0], uy[p] + h * E[1], uz[p] + h * E[2]};
        double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
        /* magnetic rotation */
        double t[3] = {h * B[0] / gm, h * B[1] / gm, h * B[2] / gm};
        double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
        double s[3] = {2.0 * t[0] / (1.0 + t2), 2.0 * t[1] / (1.0 + t2), 2.0 * t[2] / (1.0 + t2)};
        double up[3] = {um[0] + (um[1] * t[2] - um[2] * t[1]),
                        um[1] + (um[2] * t[0] - um[0] * t[2]),
                        um[2] + (um[0] * t[1] - um[1] * t[0])};
        double uplus[3] = {um[0] + (up[1] * s[2] - up[2] * s[1]),
                           um[1] + (up[2] * s[0] - up[0] * s[2]),
                           um[2] + (up[0] * s[1] - up[1] * s[0])};
        /* second half electric kick */
        ux[p] = uplus[0] + h * E[0];
        uy[p] = uplus[1] + h * E[1];
        uz[p] = uplus[2] + h * E[2];
    }
}

/* ------------------------------------------------------------------ */
/* Position update x^{n+1} = x^n + dt u^{n+1/2}/gamma^{n+1/2}.          */
/* Cell/offset renormalised with floor semantics; dcell receives the    */
/* (unwrapped) cell change per dimension, |dcell| must be <= 1.         */
/* Returns the number of particles that moved more than one cell.       */
/* ------------------------------------------------------------------ */

int64_t or_move(const or_grid *g, int64_t np, const double *ux, const double *uy, const double *uz,
                int32_t *ix, int32_t *iy, int32_t *iz, double *ox, double *oy, double *oz,
                int32_t *dcell /* [3][np] */)
{
    int64_t bad = 0;
    int32_t *cells[3] = {ix, iy, iz};
    double *offs[3] = {ox, oy, oz};
    for (int64_t p = 0; p < np; ++p) {
        double u[3] = {ux[p], uy[p], uz[p]};
        double gam = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        for (int d = 0; d < 3; ++d) dcell[(int64_t)d * np + p] = 0;
        for (int d = 0; d < g->dims; ++d) {
            double disp = g->dt * (u[d] / gam) / g->dx[d];
            double o = offs[d][p] + disp;
            double f = floor(o);
            o = o - f;
            if (o >= 1.0) { o = 0.0; f += 1.0; }
            if (fabs(f) > 1.0) ++bad;
            offs[d][p] = o;
            dcell[(int64_t)d * np + p] = (int32_t)f;
            cells[d][p] = (int32_t)wrap((int64_t)cells[d][p] + (int64_t)f, g->n[d]);
        }
    }
    return bad;
}

/* ------------------------------------------------------------------ */
/* Charge-conserving current deposition (Esirkepov 2001).               */
/* Old position: cell0 + off0; new position: cell0 + dcell + off1.      */
/* J (at n+1/2, co-located with E) is incremented.                      */
/* ------------------------------------------------------------------ */

#define WIN 6 /* window per dimension: covers both supports for order <= 2 */

void or_deposit(const or_grid *g, double q, int64_t np,
                const int32_t *ix0, const int32_t *iy0, const int32_t *iz0,
                const double *ox0, const double *oy0, const double *oz0,
                const int32_t *dcell /* [3][np] */,
                const double *ox1, const double *oy1, const double *oz1,
                const double *ux, const double *uy, const double *uz, const double *w,
                double *Jx, double *Jy, double *Jz)
{
    const int32_t *c0[3] = {ix0, iy0, iz0};
    const double *o0[3] = {ox0, oy0, oz0};
    const double *o1[3] = {ox1, oy1, oz1};
    double dV = cell_volume(g);
    for (int64_t p = 0; p < np; ++p) {
        /* window starts two cells below the old cell in every dimension */
        double S0[3][WIN], DS[3][WIN];
        for (int d = 0; d < 3; ++d)
            for (int i = 0; i < WIN; ++i) { S0[d][i] = 0.0; DS[d][i] = 0.0; }
        for (int d = 0; d < g->dims; ++d) {
            double xi0 = 2.0 + o0[d][p];                                   /* old, window units */
            double xi1 = (2.0 + (double)dcell[(int64_t)d * np + p]) + o1[d][p]; /* new, window units */
            for (int i = 0; i < WIN; ++i) {
                double s0 = or_shape(g->order, xi0 - (double)i);
                double s1 = or_shape(g->order, xi1 - (double)i);
                S0[d][i] = s0;
                DS[d][i] = s1 - s0;
            }
        }
        double base[3] = {(double)c0[0][p] - 2.0, (double)c0[1][p] - 2.0,
                          g->dims == 3 ? (double)c0[2][p] - 2.0 : 0.0};
        double qw = q * w[p] / dV;
        if (g->dims == 3) {
            double W[3][WIN][WIN][WIN]; /* [component][k][j][i] */
            for (int k = 0; k < WIN; ++k)
                for (int j = 0; j < WIN; ++j)
                    for (int i = 0; i < WIN; ++i) {
                        W[0][k][j][i] = DS[0][i] * (S0[1][j] * S0[2][k] + 0.5 * DS[1][j] * S0[2][k]
                                                    + 0.5 * S0[1][j] * DS[2][k] + DS[1][j] * DS[2][k] / 3.0);
                        W[1][k][j][i] = DS[1][j] * (S0[0][i] * S0[2][k] + 0.5 * DS[0][i] * S0[2][k]
                                                    + 0.5 * S0[0][i] * DS[2][k] + DS[0][i] * DS[2][k] / 3.0);
                        W[2][k][j][i] = DS[2][k] * (S0[0][i] * S0[1][j] + 0.5 * DS[0][i] * S0[1][j]
                                                    + 0.5 * S0[0][i] * DS[1][j] + DS[0][i] * DS[1][j] / 3.0);
                    }
            double cx = -qw * g->dx[0] / g->dt, cy = -qw * g->dx[1] / g->dt, cz = -qw * g->dx[2] / g->dt;
            /* J_x(i+1/2) = J_x(i-1/2) - qw dx/dt W_x(i), starting from zero below the window */
            for (int k = 0; k < WIN; ++k)
                for (int j = 0; j < WIN; ++j) {
                    double acc = 0.0;
                    for (int i = 0; i < WIN; ++i) {
                        acc += W[0][k][j][i];
                        Jx[lin(g, (int64_t)base[0] + i, (int64_t)base[1] + j, (int64_t)base[2] + k)] += cx * acc;
                    }
                }
            for (int k = 0; k < WIN; ++k)
                for (int i = 0; i < WIN; ++i) {
                    double acc = 0.0;
                    for (int j = 0; j < WIN; ++j) {
                        acc += W[1][k][j][i];
                        Jy[lin(g, (int64_t)base[0] + i, (int64_t)base[1] + j, (int64_t)base[2] + k)] += cy * acc;
                    }
                }
            for (int j = 0; j < WIN; ++j)
                for (int i = 0; i < WIN; ++i) {
                    double acc = 0.0;
                    for (int k = 0; k < WIN; ++k) {
                        acc += W[2][k][j][i];
                        Jz[lin(g, (int64_t)base[0] + i, (int64_t)base[1] + j, (int64_t)base[2] + k)] += cz * acc;
                    }
                }
        } else {
            double Wx[WIN][WIN], Wy[WIN][WIN], Wz[WIN][WIN]; /* [j][i] */
            double gam = sqrt(1.0 + ux[p] * ux[p] + uy[p] * uy[p] + uz[p] * uz[p]);
            double vz = uz[p] / gam;
            for (int j = 0; j < WIN; ++j)
                for (int i = 0; i < WIN; ++i) {
                    Wx[j][i] = DS[0][i] * (S0[1][j] + 0.5 * DS[1][j]);
                    Wy[j][i] = DS[1][j] * (S0[0][i] + 0.5 * DS[0][i]);
                    Wz[j][i] = S0[0][i] * S0[1][j] + 0.5 * DS[0][i] * S0[1][j]
                               + 0.5 * S0[0][i] * DS[1][j] + DS[0][i] * DS[1][j] / 3.0;
                }
            double cx = -qw * g->dx[0] / g->dt, cy = -qw * g->dx[1] / g->dt;
            for (int j = 0; j < WIN; ++j) {
                double acc = 0.0;
                for (int i = 0; i < WIN; ++i) {
                    acc += Wx[j][i];
                    Jx[lin(g, (int64_t)base[0] + i, (int64_t)base[1] + j, 0)] += cx * acc;
                }
            }
            for (int i = 0; i < WIN; ++i) {
                double acc = 0.0;
                for (int j = 0; j < WIN; ++j) {
                    acc += Wy[j][i];
                    Jy[lin(g, (int64_t)base[0] + i, (int64_t)base[1] + j, 0)] += cy * acc;
                }
            }
            for (int j = 0; j < WIN; ++j)
                for (int i = 0; i < WIN; ++i)
                    Jz[lin(g, (int64_t)base[0] + i, (int64_t)base[1] + j, 0)] += qw * vz * Wz[j][i];
        }
    }
}

/* ------------------------------------------------------------------ */
/* One species through gather, Boris, move and deposit, in place.       */
/* Returns the number of particles that moved more than one cell.       */
/* ------------------------------------------------------------------ */

int64_t or_push_deposit(const or_grid *g, double q, double m, int64_t np,
                        const double *Ex, const double *Ey, const double *Ez,
                        const double *Bx, const double *By, const double *Bz,
                        int32_t *ix, int32_t *iy, int32_t *iz, double *ox, double *oy, double *oz,
                        double *ux, double *uy, double *uz, const double *w,
                        double *Jx, double *Jy, double *Jz)
{
    double *EB = (double *)malloc(sizeof(double) * 6 * (size_t)(np > 0 ? np : 1));
    int32_t *old = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)(np > 0 ? np : 1));
    double *oldo = (double *)malloc(sizeof(double) * 3 * (size_t)(np > 0 ? np : 1));
    int32_t *dc = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)(np > 0 ? np : 1));
    or_gather(g, Ex, Ey, Ez, Bx, By, Bz, np, ix, iy, iz, ox, oy, oz, EB);
    or_boris(np, q, m, g->dt, EB, ux, uy, uz);
    for (int64_t p = 0; p < np; ++p) {
        old[p] = ix[p]; old[np + p] = iy[p]; old[2 * np + p] = iz[p];
        oldo[p] = ox[p]; oldo[np + p] = oy[p]; oldo[2 * np + p] = oz[p];
    }
    int64_t bad = or_move(g, np, ux, uy, uz, ix, iy, iz, ox, oy, oz, dc);
    or_deposit(g, q, np, old, old + np, old + 2 * np, oldo, oldo + np, oldo + 2 * np, dc,
               ox, oy, oz, ux, uy, uz, w, Jx, Jy, Jz);
    free(EB); free(old); free(oldo); free(dc);
    return bad;
}

/* ------------------------------------------------------------------ */
/* Yee FDTD curl updates (Sec. 2 ref. [9]).                              */
/* ------------------------------------------------------------------ */

/* B -= f * dt * curl E, curl taken at the B points (forward differences). */
void or_yee_b(const or_grid *g, double f, const double *Ex, const double *Ey, const double *Ez,
              double *Bx, double *By, double *Bz)
{
    double c = f * g->dt;
    int three = g->dims == 3;
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i) {
                int64_t o = lin(g, i, j, k);
                double dEz_dy = (Ez[lin(g, i, j + 1, k)] - Ez[o]) / g->dx[1];
                double dEz_dx = (Ez[lin(g, i + 1, j, k)] - Ez[o]) / g->dx[0];
                double dEy_dx = (Ey[lin(g, i + 1, j, k)] - Ey[o]) / g->dx[0];
                double dEx_dy = (Ex[lin(g, i, j + 1, k)] - Ex[o]) / g->dx[1];
                double dEy_dz = three ? (Ey[lin(g, i, j, k + 1)] - Ey[o]) / g->dx[2] : 0.0;
                double dEx_dz = three ? (Ex[lin(g, i, j, k + 1)] - Ex[o]) / g->dx[2] : 0.0;
                Bx[o] -= c * (dEz_dy - dEy_dz);
                By[o] -= c * (dEx_dz - dEz_dx);
                Bz[o] -= c * (dEy_dx - dEx_dy);
            }
}

/* E += dt * (curl B - J), curl taken at the E points (backward differences). */
void or_yee_e(const or_grid *g, const double *Bx, const double *By, const double *Bz,
              const double *Jx, const double *Jy, const double *Jz,
              double *Ex, double *Ey, double *Ez)
{
    double c = g->dt;
    int three = g->dims == 3;
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i) {
                int64_t o = lin(g, i, j, k);
                double dBz_dy = (Bz[o] - Bz[lin(g, i, j - 1, k)]) / g->dx[1];
                double dBz_dx = (Bz[o] - Bz[lin(g, i - 1, j, k)]) / g->dx[0];
                double dBy_dx = (By[o] - By[lin(g, i - 1, j, k)]) / g->dx[0];
                double dBx_dy = (Bx[o] - Bx[lin(g, i, j - 1, k)]) / g->dx[1];
                double dBy_dz = three ? (By[o] - By[lin(g, i, j, k - 1)]) / g->dx[2] : 0.0;
                double dBx_dz = three ? (Bx[o] - Bx[lin(g, i, j, k - 1)]) / g->dx[2] : 0.0;
                Ex[o] += c * ((dBz_dy - dBy_dz) - Jx[o]);
                Ey[o] += c * ((dBx_dz - dBz_dx) - Jy[o]);
                Ez[o] += c * ((dBy_dx - dBx_dy) - Jz[o]);
            }
}

/* The field part of one step: B^{n+1/2}, E^{n+1}, B^{n+1}. */
void or_yee_step(const or_grid *g, double *Ex, double *Ey, double *Ez, double *Bx, double *By, double *Bz,
                 const double *Jx, const double *Jy, const double *Jz)
{
    or_yee_b(g, 0.5, Ex, Ey, Ez, Bx, By, Bz);
    or_yee_e(g, Bx, By, Bz, Jx, Jy, Jz, Ex, Ey, Ez);
    or_yee_b(g, 0.5, Ex, Ey, Ez, Bx, By, Bz);
}

/* ------------------------------------------------------------------ */
/* Open x boundary and laser source.  The paper leaves boundaries and    */
/* laser injection out (Sec. 2); the readings used here are:             */
/*  - the x faces are the node planes i = 0 and i = n0-1; the tangential */
/*    E components there (Ey, Ez) follow Mur's first-order one-way wave  */
/*    condition (G. Mur, IEEE Trans. EMC 23 (1981) 377) instead of the   */
/*    curl update; y and z stay periodic;                                */
/*  - a particle whose cell leaves [lo, hi) along x after its move is    */
/*    removed, after it has deposited that step's current;               */
/*  - the laser is a sheet of current J_y (or J_z) on the node plane i_s */
/*    whose amplitude makes the radiated plane wave of the discrete Yee  */
/*    lattice, in the steady state, exactly E0 on both sides.            */
/* ------------------------------------------------------------------ */

/* One Yee step with open x faces: the periodic step, except that Ey and Ez
 * on the planes i = 0 and i = n0-1 take E^{n+1}_face = E^n_next +
 * a (E^{n+1}_next - E^n_face), a = (dt - dx)/(dt + dx), "next" being the
 * plane one cell inside. */
void or_yee_step_open(const or_grid *g, double *Ex, double *Ey, double *Ez, double *Bx, double *By,
                      double *Bz, const double *Jx, const double *Jy, const double *Jz)
{
    const int64_t n0 = g->n[0], nyz = (int64_t)g->n[1] * g->n[2];
    const int64_t planes[4] = {0, 1, n0 - 2, n0 - 1};
    double *old = (double *)malloc(sizeof(double) * 2 * 4 * nyz);
    or_yee_b(g, 0.5, Ex, Ey, Ez, Bx, By, Bz);
    for (int64_t jk = 0; jk < nyz; ++jk)
        for (int p = 0; p < 4; ++p) {
            int64_t o = planes[p] + n0 * jk;
            old[(0 * 4 + p) * nyz + jk] = Ey[o];
            old[(1 * 4 + p) * nyz + jk] = Ez[o];
        }
    or_yee_e(g, Bx, By, Bz, Jx, Jy, Jz, Ex, Ey, Ez);
    const double a = (g->dt - g->dx[0]) / (g->dt + g->dx[0]);
    for (int64_t jk = 0; jk < nyz; ++jk) {
        double *F[2] = {Ey, Ez};
        for (int c = 0; c < 2; ++c) {
            const double *o = old + c * 4 * nyz;
            double *f = F[c];
            /* low face: the wave leaves towards -x */
            f[0 + n0 * jk] = o[1 * nyz + jk] + a * (f[1 + n0 * jk] - o[0 * nyz + jk]);
            /* high face: the wave leaves towards +x */
            f[(n0 - 1) + n0 * jk] = o[2 * nyz + jk] + a * (f[(n0 - 2) + n0 * jk] - o[3 * nyz + jk]);
        }
    }
    or_yee_b(g, 0.5, Ex, Ey, Ez, Bx, By, Bz);
    free(old);
}

/* Current-sheet amplitude that radiates a plane wave of amplitude e0 and
 * angular frequency omega to both sides on the Yee lattice (normal
 * incidence, dx = dx[0]).  From the discrete wave equation with a source
 * J on one node plane: E = -J dx^2 sin(omega dt / 2) / (dt sin(k dx)),
 * with sin(k dx / 2) = (dx / dt) sin(omega dt / 2). */
double or_laser_j0(const or_grid *g, double e0, double omega)
{
    const double dx = g->dx[0], dt = g->dt;
    const double s = sin(0.5 * omega * dt);
    const double k = 2.0 * asin(dx / dt * s) / dx;
    return -e0 * dt * sin(k * dx) / (dx * dx * s);
}

/* Add the laser sheet to J at time t (the J time level, n + 1/2):
 * J_pol(i_s, y, z) += j0 f(y, z) g(t) sin(omega (t - t0)), with
 * f = exp(-((y - yc)^2 + (z - zc)^2) / w0^2) (w0: 1/e field radius) and
 * g = exp(-2 ln 2 (t - t0)^2 / tau^2) (tau: FWHM of the intensity).
 * pol = 1 puts it on J_y (positions (i_s, j + 1/2, k)), pol = 2 on J_z
 * (positions (i_s, j, k + 1/2)). */
void or_laser_add(const or_grid *g, double *Jy, double *Jz, int32_t plane, int32_t pol, double e0,
                  double omega, double w0, double tau, double t0, double yc, double zc, double t)
{
    const double j0 = or_laser_j0(g, e0, omega);
    const double env = exp(-2.0 * log(2.0) * (t - t0) * (t - t0) / (tau * tau));
    const double carrier = sin(omega * (t - t0));
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j) {
            double y = ((double)j + (pol == 1 ? 0.5 : 0.0)) * g->dx[1];
            double z = g->dims == 3 ? ((double)k + (pol == 2 ? 0.5 : 0.0)) * g->dx[2] : 0.0;
            double r2 = (y - yc) * (y - yc) + (g->dims == 3 ? (z - zc) * (z - zc) : 0.0);
            double v = j0 * exp(-r2 / (w0 * w0)) * env * carrier;
            int64_t o = lin(g, plane, j, k);
            if (pol == 1)
                Jy[o] += v;
            else
                Jz[o] += v;
        }
}

/* Mark every particle whose x cell is outside [lo, hi) as removed (weight
 * set to 0); returns how many were marked. */
int64_t or_absorb(int64_t np, const int32_t *ix, int32_t lo, int32_t hi, double *w)
{
    int64_t removed = 0;
    for (int64_t p = 0; p < np; ++p)
        if (w[p] != 0.0 && (ix[p] < lo || ix[p] >= hi)) {
            w[p] = 0.0;
            ++removed;
        }
    return removed;
}

/* ------------------------------------------------------------------ */
/* Diagnostics.                                                          */
/* ------------------------------------------------------------------ */

/* rho on nodes: rho(node) += q w / dV * S(x - node). */
void or_rho(const or_grid *g, double q, int64_t np, const int32_t *ix, const int32_t *iy, const int32_t *iz,
            const double *ox, const double *oy, const double *oz, const double *w, double *rho)
{
    double dV = cell_volume(g);
    for (int64_t p = 0; p < np; ++p) {
        int kmin = g->dims == 3 ? -2 : 0, kmax = g->dims == 3 ? 2 : 0;
        for (int dk = kmin; dk <= kmax; ++dk) {
            double wz = g->dims == 3 ? or_shape(g->order, (double)(-dk) + oz[p]) : 1.0;
            if (wz == 0.0) continue;
            for (int dj = -2; dj <= 2; ++dj) {
                double wy = or_shape(g->order, (double)(-dj) + oy[p]);
                if (wy == 0.0) continue;
                for (int di = -2; di <= 2; ++di) {
                    double wx = or_shape(g->order, (double)(-di) + ox[p]);
                    if (wx == 0.0) continue;
                    rho[lin(g, (int64_t)ix[p] + di, (int64_t)iy[p] + dj,
                            g->dims == 3 ? (int64_t)iz[p] + dk : 0)] += q * w[p] / dV * (wx * wy * wz);
                }
            }
        }
    }
}

/* Divergence of an E-staggered vector field, landing on nodes. */
void or_div(const or_grid *g, const double *Fx, const double *Fy, const double *Fz, double *out)
{
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i) {
                int64_t o = lin(g, i, j, k);
                double d = (Fx[o] - Fx[lin(g, i - 1, j, k)]) / g->dx[0] + (Fy[o] - Fy[lin(g, i, j - 1, k)]) / g->dx[1];
                if (g->dims == 3) d += (Fz[o] - Fz[lin(g, i, j, k - 1)]) / g->dx[2];
                out[o] = d;
            }
}

/* 1/2 sum |F|^2 dV over the grid. */
double or_field_energy(const or_grid *g, const double *Fx, const double *Fy, const double *Fz)
{
    int64_t N = (int64_t)g->n[0] * g->n[1] * g->n[2];
    double s = 0.0;
    for (int64_t o = 0; o < N; ++o) s += Fx[o] * Fx[o] + Fy[o] * Fy[o] + Fz[o] * Fz[o];
    return 0.5 * s * cell_volume(g);
}

/* sum w m (gamma - 1). */
double or_kinetic_energy(double m, int64_t np, const double *ux, const double *uy, const double *uz, const double *w)
{
    double s = 0.0;
    for (int64_t p = 0; p < np; ++p) {
        double gam = sqrt(1.0 + ux[p] * ux[p] + uy[p] * uy[p] + uz[p] * uz[p]);
        s += w[p] * m * (gam - 1.0);
    }
    return s;
}
