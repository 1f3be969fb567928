// Host-side parameter work of the SPFM library (no HIP calls).
#pragma once

#include "spfm_impl.h"

namespace spfm {

struct Params {
    int nx, ny, nz;
    double dx, lambda, Gamma, M, mu, dt, C_Gamma, eps, tau;
    double gamma[3];
    double u[3];
    int stencil, coupling;
    int interp = 0;   // kH3, kH5 or kHAbel
};

void default_gamma(int stencil, double g[3]);
double calibrate_cgamma(double lambda_over_dx, int coupling);
double stable_dt(int stencil, int coupling, const double u[3], const double gamma[3],
                 double lambda, double Gamma, double M, double mu, double dx, double C_Gamma,
                 int interp = 0);
template <typename T>
StepCoef<T> make_coef(const Params& p);
EnergyCoef make_energy_coef(const Params& p);

}  // namespace spfm
