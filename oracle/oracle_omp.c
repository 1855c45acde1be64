/*
 * All-core timing build of the FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY: used by the CPU-baseline leg of the benchmark to
 * time the oracle on every host core.  It compiles oracle.c unchanged and adds
 * one driver that splits the particles of a species into contiguous chunks,
 * one per OpenMP thread; each thread runs the oracle's own gather, Boris, move
 * and Esirkepov deposit (paper Sec. 2) on its chunk into a private current
 * grid, and the private grids are then added into J in thread order, so the
 * result does not depend on scheduling (it differs from the one-thread
 * oracle only in the order of the current sums).  The parity oracle itself
 * stays single-threaded; nothing here is used for parity.
 */
#include <omp.h>

#include "oracle.c"

int64_t or_push_deposit_omp(const or_grid *g, double q, double m, int64_t np,
                            const double *Ex, const double *Ey, const double *Ez,
                            const double *Bx, const double *By, const double *Bz,
                            int32_t *ix, int32_t *iy, int32_t *iz, double *ox, double *oy, double *oz,
                            double *ux, double *uy, double *uz, const double *w,
                            double *Jx, double *Jy, double *Jz, int32_t nthreads)
{
    const int64_t N = (int64_t)g->n[0] * g->n[1] * g->n[2];
    if (nthreads < 1) nthreads = 1;
    double *priv = (double *)calloc((size_t)nthreads * 3 * (size_t)N, sizeof(double));
    if (!priv) return -1;
    int64_t bad = 0;
#pragma omp parallel num_threads(nthreads) reduction(+ : bad)
    {
        const int t = omp_get_thread_num(), nt = omp_get_num_threads();
        const int64_t lo = np * t / nt, hi = np * (t + 1) / nt;
        double *jx = priv + (size_t)t * 3 * (size_t)N, *jy = jx + N, *jz = jy + N;
        bad += or_push_deposit(g, q, m, hi - lo, Ex, Ey, Ez, Bx, By, Bz, ix + lo, iy + lo, iz + lo, ox + lo,
                               oy + lo, oz + lo, ux + lo, uy + lo, uz + lo, w + lo, jx, jy, jz);
    }
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t o = 0; o < N; ++o) {
        for (int t = 0; t < nthreads; ++t) {
            const double *p = priv + (size_t)t * 3 * (size_t)N;
            Jx[o] += p[o];
            Jy[o] += p[N + o];
            Jz[o] += p[2 * N + o];
        }
    }
    free(priv);
    return bad;
}
