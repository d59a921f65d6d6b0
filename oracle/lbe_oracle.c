/*
 * Plain FP64 CPU stepper of the lattice Boltzmann equation for the LEE.
 *
 * TEST INFRASTRUCTURE: this file is part of the oracle.  Only the test suite, the
 * package smoke check and the benchmark's CPU-baseline leg load it.  It shares no
 * code, header or table with the GPU library.
 *
 * What one step computes, in the order the paper gives it (Section "Derivation of
 * the Lattice Boltzmann Equation", fully discrete update scheme, written in the
 * "push" form, i.e. the value leaves x and lands on x + c_i):
 *
 *   1. moments at x (monoatomic FDVM section; polyatomic form with beta in the
 *      "Generalization ... for Polyatomic Gases" section):
 *        rho'   = sum_i g_i
 *        u'     = (1/rho0) sum_i c_i g_i
 *        theta' = (1/rho0) ((gamma-1) sum_i (|c_i|^2 + beta_i)/2 g_i - theta0 rho')
 *   2. equilibrium (polyatomic ansatz; the monoatomic one is its special case):
 *        g_i^eq = f*_i (a1 rho' + a2 theta' + b c_i.u' + |c_i|^2/2 (c1 rho' + c2 theta'))
 *   3. relaxation:  g_i^* = (1 - 1/tau) g_i + (1/tau) g_i^eq
 *   4. streaming:   g_i(t+1, x + c_i) = g_i^*(x), periodic in every direction.
 *
 * Layout: g[i * N + cell], cell = x + nx * (y + ny * z), N = nx*ny*nz.
 * Unused dimensions have extent 1 and velocity component 0.
 *
 * The loop over rows is split over OpenMP threads when nthreads > 1; every (i, destination)
 * pair is written by exactly one source cell, so the threads never write the same slot.
 */
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static long wrap(long v, long n) {
    v %= n;
    return v < 0 ? v + n : v;
}

/* Collide one cell: in[Q] -> out[Q] (post-collision values, before streaming). */
static void collide_cell(int Q, const int *c, const double *fstar, const double *beta,
                         double rho0, double theta0, double gamma,
                         double a1, double a2, double b, double c1, double c2, double tau,
                         const double *in, double *out) {
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0}, e = 0.0;
    for (int i = 0; i < Q; ++i) {
        const int *ci = c + 3 * i;
        double c2i = (double)(ci[0] * ci[0] + ci[1] * ci[1] + ci[2] * ci[2]);
        rho += in[i];
        j[0] += ci[0] * in[i];
        j[1] += ci[1] * in[i];
        j[2] += ci[2] * in[i];
        e += 0.5 * (c2i + beta[i]) * in[i];
    }
    double u[3] = {j[0] / rho0, j[1] / rho0, j[2] / rho0};
    double theta = ((gamma - 1.0) * e - theta0 * rho) / rho0;
    for (int i = 0; i < Q; ++i) {
        const int *ci = c + 3 * i;
        double c2i = (double)(ci[0] * ci[0] + ci[1] * ci[1] + ci[2] * ci[2]);
        double cu = ci[0] * u[0] + ci[1] * u[1] + ci[2] * u[2];
        double geq = fstar[i] * (a1 * rho + a2 * theta + b * cu + 0.5 * c2i * (c1 * rho + c2 * theta));
        out[i] = (1.0 - 1.0 / tau) * in[i] + (1.0 / tau) * geq;
    }
}

/*
 * nsteps time steps on a periodic box.  g holds the state on entry and on return;
 * work is a second array of the same size.  Returns 0, or -1 on bad arguments.
 */
int oracle_lbe_steps(int Q, const int *c, const double *fstar, const double *beta,
                     double rho0, double theta0, double gamma,
                     double a1, double a2, double b, double c1, double c2, double tau,
                     long nx, long ny, long nz, double *g, double *work, long nsteps, int nthreads) {
    if (Q <= 0 || Q > 27 || nx <= 0 || ny <= 0 || nz <= 0 || nsteps < 0 || !(tau > 0.0)) return -1;
    const long N = nx * ny * nz;
    double *src = g, *dst = work;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    for (long s = 0; s < nsteps; ++s) {
#pragma omp parallel for collapse(2) schedule(static)
        for (long z = 0; z < nz; ++z) {
            for (long y = 0; y < ny; ++y) {
                double in[27], out[27];
                for (long x = 0; x < nx; ++x) {
                    long cell = x + nx * (y + ny * z);
                    for (int i = 0; i < Q; ++i) in[i] = src[(long)i * N + cell];
                    collide_cell(Q, c, fstar, beta, rho0, theta0, gamma, a1, a2, b, c1, c2, tau, in, out);
                    for (int i = 0; i < Q; ++i) {
                        const int *ci = c + 3 * i;
                        long xd = wrap(x + ci[0], nx), yd = wrap(y + ci[1], ny), zd = wrap(z + ci[2], nz);
                        dst[(long)i * N + xd + nx * (yd + ny * zd)] = out[i];
                    }
                }
            }
        }
        double *t = src;
        src = dst;
        dst = t;
    }
    if (src != g) memcpy(g, src, sizeof(double) * (size_t)N * (size_t)Q);
    return 0;
}

/* Number of threads OpenMP would use for the stepper (1 when built without OpenMP). */
int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
