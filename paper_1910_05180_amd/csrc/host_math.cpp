// Host-side parameter work of the SPFM library (no HIP calls): shell tables,
// the interface-energy calibration C_Gamma(lambda/dx), the explicit stability
// bound, and the per-step coefficients handed to the kernels.
#include "host_math.h"

#include <cmath>

namespace spfm {

namespace {

// Directions of Tab. 1 in the order the kernels walk them:
// shell 1: x, y, z; shell 2: x+y, x-y, y+z, y-z, x+z, x-z;
// shell 3: x+y+z, x+y-z, x-y+z, x-y-z.
const int kDir[13][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1},
                         {1, 1, 0}, {1, -1, 0}, {0, 1, 1}, {0, 1, -1}, {1, 0, 1}, {1, 0, -1},
                         {1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {1, -1, -1}};

int shell_of(int k) { return k < 3 ? 1 : (k < 9 ? 2 : 3); }
int ndirs(int stencil) { return stencil == 6 ? 3 : (stencil == 18 ? 9 : 13); }
// nu_j = 3 / (number of directions in shell j)
double nu_of(int shell) { return shell == 1 ? 1.0 : (shell == 2 ? 0.5 : 0.75); }

// Eq. 6 potential per unit lambda^2/r^2, G(phi; a) = g r^2 / lambda^2, in long double.
long double eq6_potential(long double phi, long double a) {
    const long double q = a * a, u = 1.0L - 2.0L * phi, w = u * u, x = phi * (1.0L - phi);
    if (q == 0.0L || x == 0.0L) return 0.0L;
    if (q > 1e-4L) return x + (1.0L - q) / (4.0L * q) * (log1pl(-q) - log1pl(-q * w));
    // ln((1-q)/(1-qw)) = -sum_m q^m (1 - w^m)/m
    long double s = 0.0L, qm = 1.0L, wm = 1.0L;
    for (int m = 1; m < 40; ++m) {
        wm *= w;
        const long double t = qm * (1.0L - wm) / m;
        s += t;
        if (fabsl(t) < 1e-30L * fabsl(s)) break;
        qm *= q;
    }
    return x - (1.0L - q) * 0.25L * s;
}

}  // namespace

void default_gamma(int stencil, double g[3]) {
    if (stencil == 6) { g[0] = 1.0; g[1] = 0.0; g[2] = 0.0; }
    else if (stencil == 18) { g[0] = 1.0 / 3.0; g[1] = 2.0 / 3.0; g[2] = 0.0; }
    else { g[0] = 14.0 / 30.0; g[1] = 12.0 / 30.0; g[2] = 4.0 / 30.0; }
}

// The discrete interface energy per unit area of the ideal planar [100] profile
// is (Gamma lambda / (C_Gamma dx)) sum_i [ (phi_{i+1} - phi_i)^2 / 2 + G(phi_i) ]
// (every direction with r.x = +-dx has a = tanh(2 dx/lambda), and the weights
// gamma_j nu_j / |r_j|^2 of those directions add up to sum_j gamma_j / dx^2 = 1/dx^2;
// the others see neither a gradient nor a potential).  C_Gamma is chosen so that
// this equals Gamma.  For TI it does not depend on the profile offset.
double calibrate_cgamma(double lt, int coupling) {
    if (coupling == kCF) return 2.0 / 3.0;
    if (!(lt > 0.0)) return NAN;
    const long double a = tanhl(2.0L / lt);
    const int N = (int)ceil(30.0 * lt) + 8;
    const long double c = 0.37L;
    long double sum = 0.0L;
    auto prof = [&](int i) { return 1.0L / (1.0L + expl(4.0L * ((long double)i - c) / lt)); };
    for (int i = -N; i <= N; ++i) {
        const long double p0 = prof(i), p1 = prof(i + 1);
        sum += 0.5L * (p1 - p0) * (p1 - p0) + eq6_potential(p0, a);
    }
    return (double)(lt * sum);
}

// Forward Euler is stable for the linearisation about the bulk states if
// dt (A lambda^2 |s|max + A Pmax + 6|B|) <= 2, with s(theta) the Fourier symbol
// sum_k W_k (2 cos(theta.r_k) - 2) of the weighted second differences and
// P(n) = sum_k w_k g_k''(0) the potential curvature at phi = 0 (or 1):
// TI: (lambda^2/|r_k|^2) 4 sinh^2(2 r_k.n / lambda); CF: 16/3 per direction.
double stable_dt(int stencil, int coupling, const double u[3], const double gamma[3],
                 double lambda, double Gamma, double M, double mu, double dx, double C_Gamma,
                 int interp) {
    const int nd = ndirs(stencil);
    double smax = 0.0;
    const int NT = 64;
    for (int i = 0; i <= NT; ++i)
        for (int j = 0; j <= NT; ++j)
            for (int l = 0; l <= NT; ++l) {
                const double th[3] = {M_PI * i / NT, M_PI * j / NT, M_PI * l / NT};
                double s = 0.0;
                for (int k = 0; k < nd; ++k) {
                    const int sh = shell_of(k);
                    const double W = gamma[sh - 1] * nu_of(sh) / (sh * dx * dx);
                    s += W * (2.0 * cos(th[0] * kDir[k][0] + th[1] * kDir[k][1] + th[2] * kDir[k][2]) - 2.0);
                }
                smax = fmax(smax, fabs(s));
            }
    auto pot = [&](const double n[3]) {
        double s = 0.0;
        for (int k = 0; k < nd; ++k) {
            const int sh = shell_of(k);
            const double w = gamma[sh - 1] * nu_of(sh);
            if (coupling == kCF) {
                s += w * 16.0 / 3.0;
            } else {
                const double rn = dx * (kDir[k][0] * n[0] + kDir[k][1] * n[1] + kDir[k][2] * n[2]);
                const double sh2 = sinh(2.0 * rn / lambda);
                s += w * lambda * lambda / (sh * dx * dx) * 4.0 * sh2 * sh2;
            }
        }
        return s;
    };
    double pmax = 0.0;
    if (coupling == kGlobal) {
        const double un = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        const double n[3] = {u[0] / un, u[1] / un, u[2] / un};
        pmax = pot(n);
    } else {
        const int NA = 120;
        for (int i = 0; i <= NA; ++i)
            for (int j = 0; j <= NA; ++j) {
                const double th = 0.5 * M_PI * i / NA, ph = 0.5 * M_PI * j / NA;
                const double n[3] = {sin(th) * cos(ph), sin(th) * sin(ph), cos(th)};
                pmax = fmax(pmax, pot(n));
            }
        const double d = 1.0 / sqrt(3.0);
        const double n111[3] = {d, d, d};
        pmax = fmax(pmax, pot(n111));
    }
    const double A = 2.0 * M / (3.0 * C_Gamma * lambda * lambda);
    const double B = 2.0 * M * mu / (3.0 * lambda * Gamma);
    // slope of mu h'(phi) at the bulk states: h'' = 6 (h3), 0 (h5), 2 (h_Abel)
    const double hpp = interp == kH5 ? 0.0 : (interp == kHAbel ? 2.0 : 6.0);
    return 2.0 / (A * lambda * lambda * smax + A * pmax + hpp * fabs(B));
}

template <typename T>
StepCoef<T> make_coef(const Params& p) {
    StepCoef<T> k{};
    k.nx = p.nx; k.ny = p.ny; k.nz = p.nz;
    const double A = 2.0 * p.M / (3.0 * p.C_Gamma * p.lambda * p.lambda);
    const double B = 2.0 * p.M * p.mu / (3.0 * p.lambda * p.Gamma);
    const int nsh = p.stencil == 6 ? 1 : (p.stencil == 18 ? 2 : 3);
    double wsum = 0.0;
    const int mcount[3] = {3, 6, 4};
    for (int j = 1; j <= 3; ++j) {
        const double W = j <= nsh ? p.gamma[j - 1] * nu_of(j) / (j * p.dx * p.dx) : 0.0;
        k.K[j - 1] = (T)(p.dt * A * p.lambda * p.lambda * W);
        if (j <= nsh) wsum += p.gamma[j - 1] * nu_of(j) * mcount[j - 1];
    }
    {
        double Kd[3];
        for (int j = 1; j <= 3; ++j)
            Kd[j - 1] = j <= nsh ? p.dt * A * p.lambda * p.lambda * p.gamma[j - 1] * nu_of(j) / (j * p.dx * p.dx) : 0.0;
        k.A1 = (T)(Kd[0] + 4.0 * Kd[1] + 4.0 * Kd[2]);
        k.A2 = (T)(Kd[1] + 2.0 * Kd[2]);
    }
    k.kcf = (T)(p.dt * A * 16.0 / 3.0 * wsum);
    const double hfac = p.interp == kH5 ? 30.0 : (p.interp == kHAbel ? 2.0 : 6.0);
    k.b = (T)(p.dt * hfac * B);
    k.kap2 = (T)(4.0 * p.dx / (p.lambda * M_LN2));
    k.kap2h = (T)(2.0 * p.dx / (p.lambda * M_LN2));
    k.eps = (T)p.eps;
    const double t = 8.0 * p.dx * p.tau / (p.lambda * M_LN2);
    k.tau2 = (T)(t * t);
    const double un = sqrt(p.u[0] * p.u[0] + p.u[1] * p.u[1] + p.u[2] * p.u[2]);
    double msum[3] = {0.0, 0.0, 0.0}, mmax = 0.0;
    for (int d = 0; d < 13; ++d) {
        double m = 0.0;
        if (p.coupling == kGlobal && un > 0.0) {
            const double rn = (kDir[d][0] * p.u[0] + kDir[d][1] * p.u[1] + kDir[d][2] * p.u[2]) / un;
            const double h = sinh(2.0 * p.dx * rn / p.lambda);   // beta/2
            m = 4.0 * h * h;                                      // 2 cosh(beta) - 2
        }
        k.mg[d] = (T)m;
        msum[shell_of(d) - 1] += m;
        if (shell_of(d) <= nsh) mmax = fmax(mmax, m);
    }
    for (int j = 0; j < 3; ++j) k.msum[j] = (T)msum[j];
    if (p.coupling == kLocal) {
        // beta_k = 4 r_k.n / lambda <= 4 dx sqrt(j) / lambda for every unit n
        const double h = sinh(2.0 * p.dx * sqrt((double)nsh) / p.lambda);
        mmax = 4.0 * h * h;
    }
    // y_k / (1 + y_k) = y_k (1 - y_k + ...): equal to y_k within an ulp once y_k < 2^-p
    const double ulp = sizeof(T) == 4 ? 0x1p-24 : 0x1p-53;
    k.xtail = (T)(mmax > 0.0 ? ulp / mmax : 0.0);
    return k;
}

EnergyCoef make_energy_coef(const Params& p) {
    EnergyCoef c{};
    const int nsh = p.stencil == 6 ? 1 : (p.stencil == 18 ? 2 : 3);
    for (int j = 1; j <= 3; ++j) c.w[j - 1] = j <= nsh ? p.gamma[j - 1] * nu_of(j) : 0.0;
    c.pref = p.Gamma / (p.C_Gamma * p.lambda);
    c.lambda = p.lambda;
    c.dx = p.dx;
    c.mu = p.mu;
    c.eps = p.eps;
    c.tau = p.tau;
    c.ndir = ndirs(p.stencil);
    c.coupling = p.coupling;
    c.interp = p.interp;
    const double un = sqrt(p.u[0] * p.u[0] + p.u[1] * p.u[1] + p.u[2] * p.u[2]);
    for (int d = 0; d < 13; ++d) {
        double rn = 0.0;
        if (p.coupling == kGlobal && un > 0.0)
            rn = (kDir[d][0] * p.u[0] + kDir[d][1] * p.u[1] + kDir[d][2] * p.u[2]) / un;
        c.ag[d] = tanh(2.0 * rn * p.dx / p.lambda);
    }
    return c;
}

template StepCoef<float> make_coef<float>(const Params&);
template StepCoef<double> make_coef<double>(const Params&);

}  // namespace spfm
