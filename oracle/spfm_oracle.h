/*
 * spfm_oracle.h -- plain CPU FP64 reference of the Sharp Phase-Field Method
 * (SPFM) time step of Fleck, Schleifer & Zimbrod, "Frictionless motion of
 * diffuse interfaces by sharp phase-field modeling" (arXiv:1910.05180).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against the paper.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant with the GPU library.
 *
 * Conventions (all from Sec. 2.1 of the paper):
 *   - field phi[(z*ny + y)*nx + x], x fastest, periodic on every face;
 *   - phi = 1 and phi = 0 are the two phases; the unit normal n points from
 *     phi = 1 into phi = 0 (Eq. 3);
 *   - a positive driving force mu favours phase phi = 0.
 */
#ifndef SPFM_ORACLE_H
#define SPFM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_LOCAL = 0, ORC_GLOBAL = 1, ORC_CF = 2 };
enum { ORC_H3 = 0, ORC_H5 = 1, ORC_HABEL = 2 };

typedef struct {
    int nx, ny, nz;   /* grid points along x, y, z */
    double dx;        /* grid spacing */
    double lambda;    /* interface width (Eq. 1, Eq. 3) */
    double Gamma;     /* interface energy density (Eq. 1) */
    double M;         /* kinetic coefficient (Eq. 2) */
    double mu;        /* homogeneous driving force (Eq. 1) */
    double dt;        /* explicit time step */
    double C_Gamma;   /* interface energy calibration parameter (Eq. 1), > 0 */
    int stencil;      /* 6, 18 or 26 neighbours = shells 1, 1-2, 1-3 (Tab. 1) */
    int coupling;     /* ORC_LOCAL (TI_n), ORC_GLOBAL (TI_<hkl>), ORC_CF */
    double u[3];      /* ORC_GLOBAL: direction of restored invariance */
    double gamma[3];  /* shell weights gamma_1..3 (Eq. 1) */
    double eps;       /* floor of phi and 1-phi inside the normal estimator */
    double tau;       /* |grad psi| below tau -> fallback normal (1,0,0) */
    int interp;       /* interpolation function of the driving force: ORC_H3, ORC_H5, ORC_HABEL (Tab. 2) */
} orc_params;

/* Tab. 1: direction k (0..12) as an integer vector; returns its shell 1..3. */
int orc_direction(int k, int r[3]);
/* nu_j = 3/m_j with m_j the number of directions of shell j (Sec. 2.1). */
double orc_nu(int shell);
/* Eq. 6: g_k(phi) for coupling parameter a and |r_k| = rho. */
double orc_g(double phi, double a, double rho, double lambda);
/* d g_k / d phi of Eq. 6. */
double orc_g_prime(double phi, double a, double rho, double lambda);
/* Local interface normal of the TI_n model at (x,y,z). */
void orc_normal(const orc_params *p, const double *phi, int x, int y, int z, double n[3]);
/* Right-hand side d phi / dt of Eq. 2 at every point. */
void orc_rate(const orc_params *p, const double *phi, double *rate);
/* Right-hand side at npts listed linear indices. */
void orc_rate_points(const orc_params *p, const double *phi, long npts, const long *idx, double *rate);
/* nsteps forward-Euler steps, in place.  Returns 0, or -1 on allocation failure. */
int orc_step(const orc_params *p, double *phi, long nsteps);
/* Interpolation function h of Tab. 2 and its derivative. */
double orc_interp(int which, double phi);
double orc_interp_prime(int which, double phi);
/* Total free energy of Eq. 1 (with_mu = 0 gives the interface energy F_int). */
double orc_energy(const orc_params *p, const double *phi, int with_mu);
/* Interface energy calibration C_Gamma for lambda/dx (reading: discrete energy
 * of the ideal planar [100] profile equals Gamma times its area). */
double orc_calibrate_cgamma(double lambda_over_dx);
/* Largest dt for which the linearised explicit scheme is stable. */
double orc_stable_dt(const orc_params *p);
/* Eq. 3 initial fields. */
void orc_init_planar(int nx, int ny, int nz, double dx, double lambda, const int hkl[3],
                     double offset, double *phi);
void orc_init_spheres(int nx, int ny, int nz, double dx, double lambda, int n,
                      const double *centers, const double *radii, double *phi);
/* The field of orc_init_spheres at npts integer grid coordinates xyz[3*q..3*q+2]. */
void orc_spheres_at(int nx, int ny, int nz, double dx, double lambda, int n,
                    const double *centers, const double *radii, long npts, const int *xyz,
                    double *out);
/* Threads the oracle runs on. */
/* Eq. 7 for one ghost point: the ideal profile through phi_in shifted by the
 * length whose tanh(2 shift / lambda) is a. */
double orc_wall_value(double phi_in, double a);
/* Fill the ghost layers of a padded field; p holds the padded dimensions,
 * walls bit d marks axis d walled, sin_alpha[2d], [2d+1] are the low and high
 * faces of axis d (n . e_outward of the imposed front normal). */
void orc_fill_walls(const orc_params *p, int walls, const double sin_alpha[6], double *phi);
/* nsteps of (fill, forward-Euler step) on a padded field, then a final fill. */
int orc_step_walls(const orc_params *p, int walls, const double sin_alpha[6], double *phi,
                   long nsteps);
/* Single planar front of Eq. 3 (not periodic). */
void orc_init_front(int nx, int ny, int nz, double dx, double lambda, const double n[3],
                    double offset, double *phi);
/* nsteps forward-Euler steps at constant sum phi: mu chosen at every step;
 * mu_out (nsteps values) may be NULL.  Returns 0, or -1 on allocation failure. */
int orc_step_constant_volume(const orc_params *p, double *phi, long nsteps, double *mu_out);
/* Box particle [lo, hi] (coordinates in units of length) with smooth faces. */
void orc_init_box(int nx, int ny, int nz, double dx, double lambda, const double lo[3],
                  const double hi[3], double *phi);
/* phi = 1/2 contour points on the grid edges; returns their number. */
long orc_contour_points(const orc_params *p, const double *phi, long maxpts, double *pts);
int orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
