/*
 * spfm_oracle.c -- plain, slow, FP64 CPU reference of the Sharp Phase-Field
 * Method time step (arXiv:1910.05180).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the GPU library.  It shares no
 * code with the GPU library.
 *
 * Everything here follows the paper's equations in the paper's order and
 * notation, one grid point and one direction at a time:
 *   Eq. 1  discrete free-energy density f_p with forward differences,
 *   Eq. 2  Allen-Cahn law 3 lambda Gamma d_t phi = -2 M delta_phi F,
 *   Eq. 5  grid coupling parameters a_k = tanh(2 r_k.n / lambda),
 *   Eq. 6  translationally invariant equilibrium potential g_k,
 *   Tab. 1 the 13 directions of the three neighbour shells,
 *   Eq. 3  the ideal tanh profile used for initial fields.
 * Readings where the paper is silent (time integrator, local normal, shell
 * weights, calibration) are stated where they are used.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC spfm_oracle.c -lm
 */
#include "spfm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Tab. 1, column r_k.  Row 8 is printed as [10-1] with -r = [-101]; both
 * members of the pair are used, so the choice of representative is moot. */
static const int DIR[13][3] = {
    {1, 0, 0},  {0, 1, 0},  {0, 0, 1},                                      /* shell 1 */
    {1, 1, 0},  {0, 1, 1},  {1, 0, 1}, {1, -1, 0}, {0, 1, -1}, {1, 0, -1},  /* shell 2 */
    {1, 1, 1},  {-1, 1, 1}, {1, -1, 1}, {1, 1, -1}                          /* shell 3 */
};
static const int SHELL_OF[13] = {1, 1, 1, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3};

int orc_direction(int k, int r[3]) {
    r[0] = DIR[k][0];
    r[1] = DIR[k][1];
    r[2] = DIR[k][2];
    return SHELL_OF[k];
}

/* Sec. 2.1: nu_j = 3/m_j.  Reading: m_j counts the directions of shell j
 * (3, 6, 4), so that every shell alone is a consistent Laplacian. */
double orc_nu(int shell) {
    static const double m[3] = {3.0, 6.0, 4.0};
    return 3.0 / m[shell - 1];
}

static int num_directions(int stencil) {
    return stencil == 6 ? 3 : (stencil == 18 ? 9 : 13);
}

static long lin(const orc_params *p, int x, int y, int z) {
    return ((long)z * p->ny + y) * p->nx + x;
}

static int wrap(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

/* Eq. 6.  As printed, g_k r^2/lambda^2 = x + (1-a^2)/(4a^2) ln((1-a^2)/(1-a^2 u^2))
 * with x = phi(1-phi), u = 1-2phi.  For small a^2 the logarithm's argument is
 * close to 1 and the two terms cancel.  The same expression, rewritten with
 * z = 4 a^2 x / (1 - a^2 u^2) (so that (1-a^2)/(1-a^2 u^2) = 1-z and
 * (1-a^2)/(4a^2) = x (1-z)/z), is x * T(z) with T(z) = 1 + (1-z) ln(1-z)/z,
 * whose Taylor series sum_{m>=1} z^m/(m(m+1)) is used for small z. */
double orc_g(double phi, double a, double rho, double lambda) {
    double x = phi * (1.0 - phi);
    double u = 1.0 - 2.0 * phi;
    double q = a * a;
    if (q == 0.0 || x == 0.0) return 0.0;
    double z = 4.0 * q * x / (1.0 - q * u * u);
    double T;
    if (z < 0.1) {
        double term = z, sum = 0.0;
        for (int m = 1; m < 60; ++m) {
            double t = term / ((double)m * (m + 1));
            sum += t;
            if (t < 1e-20 * sum) break;
            term *= z;
        }
        T = sum;
    } else {
        T = 1.0 + (1.0 - z) * log1p(-z) / z;
    }
    return lambda * lambda / (rho * rho) * x * T;
}

/* Derivative of Eq. 6 with respect to phi:
 * g_k' = (lambda^2/r^2) * 4 a^2 phi (1-phi)(1-2phi) / (1 - a^2 (1-2phi)^2). */
double orc_g_prime(double phi, double a, double rho, double lambda) {
    double x = phi * (1.0 - phi);
    double u = 1.0 - 2.0 * phi;
    return lambda * lambda / (rho * rho) * 4.0 * a * a * x * u / (1.0 - a * a * u * u);
}

/* Continuum-field potential g^inf = 8 phi^2 (1-phi)^2 / 3 per direction
 * (Sec. 2.1 and Tab. 2) and its derivative. */
static double g_cf(double phi) {
    double x = phi * (1.0 - phi);
    return 8.0 * x * x / 3.0;
}
static double g_cf_prime(double phi) {
    return 16.0 * phi * (1.0 - phi) * (1.0 - 2.0 * phi) / 3.0;
}

/* psi = (lambda/4) ln((1-phi)/phi) inverts Eq. 3: on the ideal profile it equals
 * p.n - c_n, a linear function of position.  Both logarithm arguments are
 * floored at eps, which keeps psi finite on bulk values phi = 0 or 1 (and on
 * the small over- and undershoots of explicit stepping). */
static double psi_of(const orc_params *p, double phi) {
    double a = 1.0 - phi, b = phi;
    if (a < p->eps) a = p->eps;
    if (b < p->eps) b = p->eps;
    return 0.25 * p->lambda * (log(a) - log(b));
}

/* Local normal of the TI_n model.  The paper defers the estimator to its
 * companion article; reading: n = grad psi / |grad psi| with central
 * differences over the six face neighbours, which is exact for an ideal planar
 * profile of any orientation and offset.  Where |grad psi| < tau (bulk, where
 * phi(1-phi) ~ 0) the normal falls back to (1,0,0). */
void orc_normal(const orc_params *p, const double *phi, int x, int y, int z, double n[3]) {
    double g[3];
    g[0] = (psi_of(p, phi[lin(p, wrap(x + 1, p->nx), y, z)]) -
            psi_of(p, phi[lin(p, wrap(x - 1, p->nx), y, z)])) / (2.0 * p->dx);
    g[1] = (psi_of(p, phi[lin(p, x, wrap(y + 1, p->ny), z)]) -
            psi_of(p, phi[lin(p, x, wrap(y - 1, p->ny), z)])) / (2.0 * p->dx);
    g[2] = (psi_of(p, phi[lin(p, x, y, wrap(z + 1, p->nz))]) -
            psi_of(p, phi[lin(p, x, y, wrap(z - 1, p->nz))])) / (2.0 * p->dx);
    double norm = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    if (norm < p->tau) {
        n[0] = 1.0; n[1] = 0.0; n[2] = 0.0;
    } else {
        n[0] = g[0] / norm; n[1] = g[1] / norm; n[2] = g[2] / norm;
    }
}

static void coupling_normal(const orc_params *p, const double *phi, int x, int y, int z,
                            double n[3]) {
    if (p->coupling == ORC_LOCAL) {
        orc_normal(p, phi, x, y, z, n);
    } else {
        double un = sqrt(p->u[0] * p->u[0] + p->u[1] * p->u[1] + p->u[2] * p->u[2]);
        n[0] = p->u[0] / un; n[1] = p->u[1] / un; n[2] = p->u[2] / un;
    }
}

/* Eq. 5: a_k(n) = tanh(2 r_k.n / lambda), r_k in physical units. */
static double coupling_a(const orc_params *p, const int r[3], const double n[3]) {
    double rn = (r[0] * n[0] + r[1] * n[1] + r[2] * n[2]) * p->dx;
    return tanh(2.0 * rn / p->lambda);
}

/* Interpolation functions of Tab. 2: h3 = phi^2 (3 - 2 phi) (all models),
 * h5 = phi^3 (10 - 15 phi + 6 phi^2) and h_Abel = phi^2 / (phi^2 + (1-phi)^2)
 * (CF comparisons, Sec. 3.1).  Written as printed; their derivatives below are
 * the textbook derivatives of these expressions. */
static double interp_h(int which, double phi) {
    switch (which) {
        case ORC_H5: return phi * phi * phi * (10.0 - 15.0 * phi + 6.0 * phi * phi);
        case ORC_HABEL: return phi * phi / (phi * phi + (1.0 - phi) * (1.0 - phi));
        default: return phi * phi * (3.0 - 2.0 * phi);
    }
}
static double interp_h_prime(int which, double phi) {
    switch (which) {
        case ORC_H5: return 30.0 * phi * phi * (1.0 - phi) * (1.0 - phi);
        case ORC_HABEL: {
            double d = phi * phi + (1.0 - phi) * (1.0 - phi);
            return 2.0 * phi * (1.0 - phi) / (d * d);
        }
        default: return 6.0 * phi * (1.0 - phi);
    }
}
double orc_interp(int which, double phi) { return interp_h(which, phi); }
double orc_interp_prime(int which, double phi) { return interp_h_prime(which, phi); }

/* d phi_p / dt from Eq. 2 with the functional derivative of Eq. 1:
 *   delta_phi F = Gamma/(C_Gamma lambda) sum_k gamma_j nu_j [ g_k'(phi_p)
 *                 - lambda^2 (phi_{p+r} - 2 phi_p + phi_{p-r}) / |r|^2 ] + mu h'(phi_p),
 *   d_t phi = -(2M / (3 lambda Gamma)) delta_phi F,
 * with h the interpolation function of the model (h3 unless chosen otherwise).  The sign of the gradient
 * term is that of the variational derivative of the forward-difference energy
 * of Eq. 1 (and of Eq. 4); the printed definition of the backward difference
 * carries the opposite sign. */
static double rate_at(const orc_params *p, const double *phi, int x, int y, int z) {
    double phi0 = phi[lin(p, x, y, z)];
    double n[3] = {1.0, 0.0, 0.0};
    if (p->coupling != ORC_CF) coupling_normal(p, phi, x, y, z, n);
    double s = 0.0;
    int nd = num_directions(p->stencil);
    for (int k = 0; k < nd; ++k) {
        int r[3];
        int j = orc_direction(k, r);
        double rho = sqrt((double)j) * p->dx;
        double w = p->gamma[j - 1] * orc_nu(j);
        double pp = phi[lin(p, wrap(x + r[0], p->nx), wrap(y + r[1], p->ny), wrap(z + r[2], p->nz))];
        double pm = phi[lin(p, wrap(x - r[0], p->nx), wrap(y - r[1], p->ny), wrap(z - r[2], p->nz))];
        double lap = p->lambda * p->lambda / (rho * rho) * (pp - 2.0 * phi0 + pm);
        double gp;
        if (p->coupling == ORC_CF) {
            gp = g_cf_prime(phi0);
        } else {
            gp = orc_g_prime(phi0, coupling_a(p, r, n), rho, p->lambda);
        }
        s += w * (gp - lap);
    }
    double dF = p->Gamma / (p->C_Gamma * p->lambda) * s + p->mu * interp_h_prime(p->interp, phi0);
    return -2.0 * p->M / (3.0 * p->lambda * p->Gamma) * dF;
}

void orc_rate(const orc_params *p, const double *phi, double *rate) {
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) rate[lin(p, x, y, z)] = rate_at(p, phi, x, y, z);
}

void orc_rate_points(const orc_params *p, const double *phi, long npts, const long *idx,
                     double *rate) {
#pragma omp parallel for schedule(static)
    for (long i = 0; i < npts; ++i) {
        long q = idx[i];
        int x = (int)(q % p->nx);
        int y = (int)((q / p->nx) % p->ny);
        int z = (int)(q / ((long)p->nx * p->ny));
        rate[i] = rate_at(p, phi, x, y, z);
    }
}

/* Reading: the explicit time integration the paper implies is forward Euler
 * with all reads from the previous time level (Jacobi). */
int orc_step(const orc_params *p, double *phi, long nsteps) {
    long n = (long)p->nx * p->ny * p->nz;
    double *rate = (double *)malloc(sizeof(double) * (size_t)n);
    if (!rate) return -1;
    for (long s = 0; s < nsteps; ++s) {
        orc_rate(p, phi, rate);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) phi[i] = phi[i] + p->dt * rate[i];
    }
    free(rate);
    return 0;
}

/* Neumaier compensated accumulation. */
typedef struct { double s, c; } acc_t;
static void acc_add(acc_t *a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}

/* Eq. 1: F = sum_p f_p dx^3 with
 * f_p = Gamma/(C_Gamma lambda) sum_k gamma_j nu_j (lambda^2/2 (d_k^+ phi)^2 + g_k(phi_p)) + mu h(phi_p). */
double orc_energy(const orc_params *p, const double *phi, int with_mu) {
    acc_t *plane = (acc_t *)calloc((size_t)p->nz, sizeof(acc_t));
    if (!plane) return NAN;
    int nd = num_directions(p->stencil);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; ++z) {
        acc_t a = {0.0, 0.0};
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                double phi0 = phi[lin(p, x, y, z)];
                double n[3] = {1.0, 0.0, 0.0};
                if (p->coupling != ORC_CF) coupling_normal(p, phi, x, y, z, n);
                double s = 0.0;
                for (int k = 0; k < nd; ++k) {
                    int r[3];
                    int j = orc_direction(k, r);
                    double rho = sqrt((double)j) * p->dx;
                    double w = p->gamma[j - 1] * orc_nu(j);
                    double pp = phi[lin(p, wrap(x + r[0], p->nx), wrap(y + r[1], p->ny),
                                        wrap(z + r[2], p->nz))];
                    double d = (pp - phi0) / rho;
                    double g = p->coupling == ORC_CF
                                   ? g_cf(phi0)
                                   : orc_g(phi0, coupling_a(p, r, n), rho, p->lambda);
                    s += w * (0.5 * p->lambda * p->lambda * d * d + g);
                }
                double f = p->Gamma / (p->C_Gamma * p->lambda) * s;
                if (with_mu) f += p->mu * interp_h(p->interp, phi0);
                acc_add(&a, f);
            }
        plane[z] = a;
    }
    acc_t tot = {0.0, 0.0};
    for (int z = 0; z < p->nz; ++z) {
        acc_add(&tot, plane[z].s);
        acc_add(&tot, plane[z].c);
    }
    free(plane);
    return (tot.s + tot.c) * p->dx * p->dx * p->dx;
}

/* Reading of the calibration (the paper only plots C_Gamma(lambda/dx) and
 * defers the procedure): C_Gamma is the value for which the discrete interface
 * energy (Eq. 1, mu = 0) of the ideal planar [100] profile equals Gamma times
 * the interface area.  Evaluated on a periodic x-line holding a slab with two
 * interfaces 20 lambda apart, with Gamma = dx = 1 and C_Gamma = 1. */
double orc_calibrate_cgamma(double lt) {
    int nx = (int)ceil(40.0 * lt);
    if (nx < 16) nx = 16;
    orc_params p;
    memset(&p, 0, sizeof p);
    p.nx = nx; p.ny = 1; p.nz = 1;
    p.dx = 1.0; p.lambda = lt; p.Gamma = 1.0; p.M = 1.0; p.mu = 0.0; p.dt = 0.0;
    p.C_Gamma = 1.0; p.stencil = 6; p.coupling = ORC_GLOBAL;
    p.u[0] = 1.0; p.gamma[0] = 1.0;
    p.eps = 1e-300; p.tau = 1e-3;
    double *phi = (double *)malloc(sizeof(double) * (size_t)nx);
    if (!phi) return NAN;
    const int hkl[3] = {1, 0, 0};
    orc_init_planar(nx, 1, 1, 1.0, lt, hkl, 0.0, phi);
    double F = orc_energy(&p, phi, 0);
    free(phi);
    return F / 2.0; /* two interfaces of unit area */
}

/* Linear stability of forward Euler about the bulk states phi = 0, 1.  With
 * the right-hand side linearised, d_t dphi = -(A lambda^2 |s(theta)| + A P(n)) dphi
 * +- 6 B dphi with A = 2M/(3 C_Gamma lambda^2) and B = 2 M mu / (3 lambda Gamma),
 * s(theta) = sum_k (w_k/|r_k|^2)(2cos(theta.r_k) - 2) the Fourier symbol of the
 * weighted second differences and P(n) = sum_k w_k g_k''(0).  For Eq. 6,
 * g_k''(0) = (lambda^2/|r_k|^2) 4 a_k^2/(1-a_k^2).  Forward Euler requires
 * dt * max|rate| <= 2.  Maxima are taken by brute-force sampling. */
double orc_stable_dt(const orc_params *p) {
    int nd = num_directions(p->stencil);
    double smax = 0.0;
    const int NT = 48;
    for (int i = 0; i <= NT; ++i)
        for (int j = 0; j <= NT; ++j)
            for (int l = 0; l <= NT; ++l) {
                double th[3] = {M_PI * i / NT, M_PI * j / NT, M_PI * l / NT};
                double s = 0.0;
                for (int k = 0; k < nd; ++k) {
                    int r[3];
                    int sh = orc_direction(k, r);
                    double rho2 = sh * p->dx * p->dx;
                    double w = p->gamma[sh - 1] * orc_nu(sh);
                    s += w / rho2 * (2.0 * cos(th[0] * r[0] + th[1] * r[1] + th[2] * r[2]) - 2.0);
                }
                if (fabs(s) > smax) smax = fabs(s);
            }
    double pmax = 0.0;
    const int NA = 90;
    for (int i = 0; i <= NA; ++i)
        for (int j = 0; j <= NA; ++j) {
            double n[3];
            if (p->coupling == ORC_GLOBAL) {
                if (i > 0 || j > 0) break;
                double un = sqrt(p->u[0] * p->u[0] + p->u[1] * p->u[1] + p->u[2] * p->u[2]);
                n[0] = p->u[0] / un; n[1] = p->u[1] / un; n[2] = p->u[2] / un;
            } else {
                double th = 0.5 * M_PI * i / NA, ph = 0.5 * M_PI * j / NA;
                n[0] = sin(th) * cos(ph); n[1] = sin(th) * sin(ph); n[2] = cos(th);
            }
            double s = 0.0;
            for (int k = 0; k < nd; ++k) {
                int r[3];
                int sh = orc_direction(k, r);
                double rho = sqrt((double)sh) * p->dx;
                double w = p->gamma[sh - 1] * orc_nu(sh);
                if (p->coupling == ORC_CF) {
                    s += w * 16.0 / 3.0;
                } else {
                    double a = coupling_a(p, r, n);
                    s += w * p->lambda * p->lambda / (rho * rho) * 4.0 * a * a / (1.0 - a * a);
                }
            }
            if (s > pmax) pmax = s;
            if (p->coupling == ORC_CF) break;
        }
    double A = 2.0 * p->M / (3.0 * p->C_Gamma * p->lambda * p->lambda);
    double B = 2.0 * p->M * p->mu / (3.0 * p->lambda * p->Gamma);
    /* the driving term's slope at the bulk states is mu h''(0) = mu h''(1) up to sign:
     * 6 for h3, 0 for h5, 2 for h_Abel */
    double hpp = p->interp == ORC_H5 ? 0.0 : (p->interp == ORC_HABEL ? 2.0 : 6.0);
    return 2.0 / (A * p->lambda * p->lambda * smax + A * pmax + hpp * fabs(B));
}

static long gcd_l(long a, long b) {
    if (a < 0) a = -a;
    if (b < 0) b = -b;
    while (b) { long t = a % b; a = b; b = t; }
    return a;
}

/* Eq. 3 on a periodic slab (reading of a planar interface in a periodic box).
 * For integer normal N the field depends only on s = p.N/|N| - c, with period
 * P = gcd_i(n_i |N_i|) dx / |N|.  One period holds a slab of phi = 1 of
 * thickness P/2 between two ideal interfaces whose normals point into phi = 0:
 *   T(s) = f(s + P/4) - f(s - P/4),  f(t) = (1 + tanh(2t/lambda))/2,
 * and the field is the sum of T over all periodic images, which is smooth and
 * exactly periodic (a single image would leave a kink of size ~exp(-P/lambda)
 * where neighbouring slabs meet).  Images are summed until the omitted ones
 * are at least 10 lambda away.  The slab centre is the box centre shifted by
 * offset along N. */
void orc_init_planar(int nx, int ny, int nz, double dx, double lambda, const int hkl[3],
                     double offset, double *phi) {
    double nn = sqrt((double)hkl[0] * hkl[0] + (double)hkl[1] * hkl[1] + (double)hkl[2] * hkl[2]);
    long g = 0;
    g = gcd_l(g, (long)nx * hkl[0]);
    g = gcd_l(g, (long)ny * hkl[1]);
    g = gcd_l(g, (long)nz * hkl[2]);
    double P = (double)g * dx / nn;
    double nv[3] = {hkl[0] / nn, hkl[1] / nn, hkl[2] / nn};
    double c = 0.5 * dx * (nx * nv[0] + ny * nv[1] + nz * nv[2]) + offset;
    int K = 2 + (int)ceil(10.0 * lambda / P);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                double s = dx * (x * nv[0] + y * nv[1] + z * nv[2]) - c;
                s -= P * nearbyint(s / P);
                double v = 0.0;
                for (int m = -K; m <= K; ++m) {
                    double t = s - m * P;
                    v += 0.5 * (tanh(2.0 * (t + 0.25 * P) / lambda) -
                                tanh(2.0 * (t - 0.25 * P) / lambda));
                }
                phi[((long)z * ny + y) * nx + x] = v;
            }
}

/* Eq. 3 around spheres, phi_i = (1 - tanh(2 (|p - c_i| - R_i)/lambda))/2 with the
 * periodic minimum-image distance, combined as phi = 1 - prod_i (1 - phi_i):
 * smooth, within [0, 1], and equal to phi_i near an isolated grain. */
void orc_init_spheres(int nx, int ny, int nz, double dx, double lambda, int n,
                      const double *centers, const double *radii, double *phi) {
    double L[3] = {nx * dx, ny * dx, nz * dx};
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                double pos[3] = {x * dx, y * dx, z * dx};
                /* 1 - prod_i (1 - phi_i) accumulated as sum_i phi_i prod_{j<i} (1 - phi_j),
                 * which keeps small tail values exact */
                double acc = 0.0, prod = 1.0;
                for (int i = 0; i < n; ++i) {
                    double r2 = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        double d = pos[a] - centers[3 * i + a];
                        d -= L[a] * nearbyint(d / L[a]);
                        r2 += d * d;
                    }
                    double v = 0.5 * (1.0 - tanh(2.0 * (sqrt(r2) - radii[i]) / lambda));
                    acc += prod * v;
                    prod *= 1.0 - v;
                }
                phi[((long)z * ny + y) * nx + x] = acc;
            }
}

/* The field of orc_init_spheres (box nx x ny x nz) evaluated at npts grid
 * coordinates given as integer triples (x, y, z), for crops of large boxes. */
void orc_spheres_at(int nx, int ny, int nz, double dx, double lambda, int n,
                    const double *centers, const double *radii, long npts, const int *xyz,
                    double *out) {
    double L[3] = {nx * dx, ny * dx, nz * dx};
#pragma omp parallel for schedule(static)
    for (long q = 0; q < npts; ++q) {
        double pos[3] = {xyz[3 * q] * dx, xyz[3 * q + 1] * dx, xyz[3 * q + 2] * dx};
        double acc = 0.0, prod = 1.0;
        for (int i = 0; i < n; ++i) {
            double r2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                double d = pos[a] - centers[3 * i + a];
                d -= L[a] * nearbyint(d / L[a]);
                r2 += d * d;
            }
            double v = 0.5 * (1.0 - tanh(2.0 * (sqrt(r2) - radii[i]) / lambda));
            acc += prod * v;
            prod *= 1.0 - v;
        }
        out[q] = acc;
    }
}

/* ---- Walls with a contact angle (Sec. 2.2, Eq. 7) ----
 * A walled axis carries one ghost layer at each end: the padded field has
 * nx + 2 (ny + 2, nz + 2) points along a walled axis, interior index i at
 * padded index i + 1.  Eq. 7 sets a ghost point b from its inward neighbour
 * b + r by the tanh addition law of the ideal profile (Eq. 3), shifting the
 * profile by |r| sin(alpha): phi_b = (1 - a) phi_{b+r} / (1 - a (2 phi_{b+r} - 1)),
 * a = tanh(2 |r| sin(alpha) / lambda).  For a planar front of normal n (into
 * phi = 0) the exact ghost value needs sin(alpha) = n . e, e the outward
 * normal of the wall: that is the meaning of sin_alpha[] below. */
double orc_wall_value(double phi_in, double a) {
    return (1.0 - a) * phi_in / (1.0 - a * (2.0 * phi_in - 1.0));
}

/* Reading: the paper states Eq. 7 for a face.  Edge and corner ghosts (needed
 * by the 18- and 26-neighbour stencils) are filled by applying Eq. 7 axis after
 * axis, x, then y, then z, each fill spanning the whole padded extent of the
 * other axes: a corner ghost is the interior value shifted by the sum of the
 * shifts of its walls, exact for the ideal front. */
void orc_fill_walls(const orc_params *p, int walls, const double sin_alpha[6], double *phi) {
    const int n[3] = {p->nx, p->ny, p->nz};
    for (int d = 0; d < 3; ++d) {
        if (!(walls & (1 << d))) continue;
        const double a_lo = tanh(2.0 * p->dx * sin_alpha[2 * d] / p->lambda);
        const double a_hi = tanh(2.0 * p->dx * sin_alpha[2 * d + 1] / p->lambda);
        const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
        for (int j = 0; j < n[d1]; ++j)
            for (int k = 0; k < n[d2]; ++k) {
                int c[3];
                c[d1] = j;
                c[d2] = k;
                c[d] = 1;
                const double in_lo = phi[lin(p, c[0], c[1], c[2])];
                c[d] = 0;
                phi[lin(p, c[0], c[1], c[2])] = orc_wall_value(in_lo, a_lo);
                c[d] = n[d] - 2;
                const double in_hi = phi[lin(p, c[0], c[1], c[2])];
                c[d] = n[d] - 1;
                phi[lin(p, c[0], c[1], c[2])] = orc_wall_value(in_hi, a_hi);
            }
    }
}

/* nsteps of: fill the walls of the padded field, then one forward-Euler step
 * of every point (the ghost values it produces are overwritten by the next
 * fill).  p holds the padded dimensions. */
int orc_step_walls(const orc_params *p, int walls, const double sin_alpha[6], double *phi,
                   long nsteps) {
    for (long s = 0; s < nsteps; ++s) {
        orc_fill_walls(p, walls, sin_alpha, phi);
        if (orc_step(p, phi, 1) != 0) return -1;
    }
    orc_fill_walls(p, walls, sin_alpha, phi);
    return 0;
}

/* One planar front of Eq. 3, phi = (1 - tanh(2 s / lambda)) / 2 with
 * s = dx (x, y, z) . n/|n| - c and c = the box centre (nx, ny, nz) dx / 2
 * projected on n/|n|, plus offset: phase 1 behind the front, n into phase 0. */
void orc_init_front(int nx, int ny, int nz, double dx, double lambda, const double n[3],
                    double offset, double *phi) {
    double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    double nv[3] = {n[0] / nn, n[1] / nn, n[2] / nn};
    double c = 0.5 * dx * (nx * nv[0] + ny * nv[1] + nz * nv[2]) + offset;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                double s = dx * (x * nv[0] + y * nv[1] + z * nv[2]) - c;
                phi[((long)z * ny + y) * nx + x] = 0.5 * (1.0 - tanh(2.0 * s / lambda));
            }
}

/* ---- Constant particle volume (Sec. 3.3) ----
 * The rate of Eq. 2 is affine in the homogeneous driving force:
 * rate_p(mu) = rate_p(0) - beta mu h'(phi_p), beta = 2M / (3 lambda Gamma).
 * Reading: the paper imposes mu(t) "such that the integral volume neither
 * shrinks nor grows"; here mu is chosen at every step so that the forward-Euler
 * update leaves sum phi unchanged: mu = sum rate(0) / (beta sum h'). */
int orc_step_constant_volume(const orc_params *p, double *phi, long nsteps, double *mu_out) {
    long n = (long)p->nx * p->ny * p->nz;
    double *rate = (double *)malloc(sizeof(double) * (size_t)n);
    if (!rate) return -1;
    orc_params q = *p;
    q.mu = 0.0;
    const double beta = 2.0 * p->M / (3.0 * p->lambda * p->Gamma);
    for (long s = 0; s < nsteps; ++s) {
        orc_rate(&q, phi, rate);
        acc_t r0 = {0.0, 0.0}, hp = {0.0, 0.0};
        for (long i = 0; i < n; ++i) {
            acc_add(&r0, rate[i]);
            acc_add(&hp, interp_h_prime(p->interp, phi[i]));
        }
        const double den = beta * (hp.s + hp.c);
        const double mu = den != 0.0 ? (r0.s + r0.c) / den : 0.0;
        if (mu_out) mu_out[s] = mu;
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i)
            phi[i] = phi[i] + p->dt * (rate[i] - beta * mu * interp_h_prime(p->interp, phi[i]));
    }
    free(rate);
    return 0;
}

/* Box particle: the product over the axes of smooth top hats of Eq. 3,
 * phi = prod_d t(x_d), t(s) = f(s - lo_d) f(hi_d - s) with f(s) = (1 + tanh(2 s / lambda)) / 2. */
void orc_init_box(int nx, int ny, int nz, double dx, double lambda, const double lo[3],
                  const double hi[3], double *phi) {
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const double pos[3] = {x * dx, y * dx, z * dx};
                double v = 1.0;
                for (int d = 0; d < 3; ++d)
                    v *= 0.25 * (1.0 + tanh(2.0 * (pos[d] - lo[d]) / lambda)) *
                         (1.0 + tanh(2.0 * (hi[d] - pos[d]) / lambda));
                phi[((long)z * ny + y) * nx + x] = v;
            }
}

/* phi = 1/2 contour points (Sec. 2.3, Eq. 8-10 at l = 1/2): on every grid edge
 * (p, p + e_d) of a periodic field whose end values bracket 1/2, the point
 * p + t e_d with t the zero of the linear interpolation of
 * psi = (lambda/4) ln((1 - phi)/phi) (R18).  Fills up to maxpts points
 * (x, y, z; unwrapped: p + t e_d may reach the box edge) and returns the count. */
long orc_contour_points(const orc_params *p, const double *phi, long maxpts, double *pts) {
    long cnt = 0;
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                const double a = phi[lin(p, x, y, z)];
                for (int d = 0; d < 3; ++d) {
                    int q[3] = {x, y, z};
                    q[d] += 1;
                    const double b = phi[lin(p, wrap(q[0], p->nx), wrap(q[1], p->ny), wrap(q[2], p->nz))];
                    if ((a - 0.5) * (b - 0.5) > 0.0 || a == b) continue;
                    const double pa = 0.25 * p->lambda * log((1.0 - a) / a);
                    const double pb = 0.25 * p->lambda * log((1.0 - b) / b);
                    const double t = pa / (pa - pb);
                    if (cnt < maxpts) {
                        double *o = pts + 3 * cnt;
                        o[0] = x * p->dx; o[1] = y * p->dx; o[2] = z * p->dx;
                        o[d] += t * p->dx;
                    }
                    ++cnt;
                }
            }
    return cnt;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
