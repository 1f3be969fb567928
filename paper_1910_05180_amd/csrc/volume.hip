// Constant particle volume (Sec. 3.3) and the phi = 1/2 contour statistics
// that measure the residual anisotropy of a relaxed particle.
//
// Constant volume.  The rate of Eq. 2 is affine in the homogeneous driving
// force, rate(mu) = rate(0) - beta mu h'(phi), beta = 2M / (3 lambda Gamma).  A
// step is the ordinary step kernel with mu = 0, writing phi* = phi + dt rate(0),
// and a correction that never leaves the device: the sums of phi* - phi and
// h'(phi), g = sum(phi* - phi) / sum h'(phi), mu = g / (dt beta), and
// phi_new = phi* - g h'(phi) at every point in FP64.  Then sum phi_new = sum phi
// up to the rounding of the stored values.  The sums are exact integer sums of
// terms rounded to 2^-54 (CvAcc), so g does not depend on which pass formed
// them or how it split the points:
//   k_cv_partial  per-block partial sums (the plain kernel's path; the tiled
//                 step forms one partial per work item itself);
//   k_cv_total    one block adds many partials into one;
//   k_cv_apply    every block adds the partials (few: at most kCvDirectParts),
//                 block 0 stores g and mu in device memory, and every block
//                 applies the correction to its points.
//
// Contours.  On every grid edge (p, p + e_d) whose end values bracket 1/2 the
// contour point is p + t e_d with t the zero of the linear interpolation of
// ln((1 - phi)/phi) (Eq. 8-10 at l = 1/2).  Two passes: the barycentre
// sum phi x / sum phi, then count, sum, min and max of the distances of the
// contour points from it.
#include <algorithm>

#include "spfm_impl.h"

namespace spfm {

namespace {

struct Acc {   // TwoSum accumulator
    double s, c;
    __device__ __forceinline__ void add(double v) {
        const double t = s + v;
        const double bp = t - s;
        c += (s - (t - bp)) + (v - bp);
        s = t;
    }
    __device__ __forceinline__ void merge(double os, double oc) {
        add(os);
        c += oc;
    }
    __device__ __forceinline__ double value() const { return s + c; }
};

// Block sums of NQ (s, c) pairs plus NM min and max values, in a fixed order:
// wave butterflies, then thread 0 over the waves.  Returns on thread 0.
template <int NQ>
__device__ __forceinline__ void block_sums(Acc (&a)[NQ], double& mn, double& mx) {
    for (int m = 32; m > 0; m >>= 1) {
        for (int q = 0; q < NQ; ++q) {
            const double os = __shfl_xor(a[q].s, m), oc = __shfl_xor(a[q].c, m);
            a[q].merge(os, oc);
        }
        mn = fmin(mn, __shfl_xor(mn, m));
        mx = fmax(mx, __shfl_xor(mx, m));
    }
    __shared__ double sh[kReduceThreads / 64][2 * NQ + 2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        for (int q = 0; q < NQ; ++q) { sh[wave][2 * q] = a[q].s; sh[wave][2 * q + 1] = a[q].c; }
        sh[wave][2 * NQ] = mn;
        sh[wave][2 * NQ + 1] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kReduceThreads / 64; ++w) {
            for (int q = 0; q < NQ; ++q) a[q].merge(sh[w][2 * q], sh[w][2 * q + 1]);
            mn = fmin(mn, sh[w][2 * NQ]);
            mx = fmax(mx, sh[w][2 * NQ + 1]);
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kReduceThreads) void k_cv_partial(const T* __restrict__ phi_old,
                                                               const T* __restrict__ phi_new,
                                                               int64_t n, int interp,
                                                               unsigned long long* __restrict__ part) {
    CvAcc a{{0, 0}};
    const int64_t stride = (int64_t)gridDim.x * kReduceThreads;
    for (int64_t i = (int64_t)blockIdx.x * kReduceThreads + threadIdx.x; i < n; i += stride) {
        const double o = (double)phi_old[i];
        a.add((double)phi_new[i] - o, h_slope(interp, o));
    }
    cv_block_store<kReduceThreads>(a, part + 4 * (size_t)blockIdx.x);
}

__global__ __launch_bounds__(kReduceThreads) void k_cv_total(const unsigned long long* __restrict__ part,
                                                             int nparts,
                                                             unsigned long long* __restrict__ total) {
    CvAcc a{{0, 0}};
    for (int b = threadIdx.x; b < nparts; b += kReduceThreads) a.add_words(part + 4 * (size_t)b);
    cv_block_store<kReduceThreads>(a, total);
}

// state[0] = g (the correction per unit h'), state[1] = mu.  Every block adds
// the same integers, so every block applies the same g.
template <typename T>
__global__ __launch_bounds__(kReduceThreads) void k_cv_apply(const T* phi_new, T* phi_out,
                                                             const T* __restrict__ phi_old, int64_t n,
                                                             int interp,
                                                             const unsigned long long* __restrict__ part,
                                                             int nparts, double dt_beta,
                                                             double* __restrict__ state) {
    __shared__ unsigned long long tot[4];
    // this thread's point, loaded first so that its latency overlaps the sums
    const int64_t i = (int64_t)blockIdx.x * kReduceThreads + threadIdx.x;
    const bool in = i < n;
    const T pn = in ? phi_new[i] : T(0), po = in ? phi_old[i] : T(0);
    CvAcc a{{0, 0}};
    for (int b = threadIdx.x; b < nparts; b += kReduceThreads) a.add_words(part + 4 * (size_t)b);
    cv_block_store<kReduceThreads>(a, tot);
    __syncthreads();
    CvAcc t{{0, 0}};
    t.add_words(tot);
    const double den = CvAcc::value(t.s[1]);
    const double g = den != 0.0 ? CvAcc::value(t.s[0]) / den : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        state[0] = g;
        state[1] = dt_beta != 0.0 ? g / dt_beta : 0.0;
    }
    if (in) phi_out[i] = (T)((double)pn - g * h_slope(interp, (double)po));
}

// Pass 1 of the contour statistics: sum phi, sum phi x, sum phi y, sum phi z.
template <typename T>
__global__ __launch_bounds__(kReduceThreads) void k_moments_partial(const T* __restrict__ phi, int nx,
                                                                    int ny, int nz,
                                                                    double* __restrict__ part) {
    Acc a[4] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    double mn = 0.0, mx = 0.0;
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t stride = (int64_t)gridDim.x * kReduceThreads;
    for (int64_t i = (int64_t)blockIdx.x * kReduceThreads + threadIdx.x; i < n; i += stride) {
        const double v = (double)phi[i];
        const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((int64_t)nx * ny));
        a[0].add(v);
        a[1].add(v * x);
        a[2].add(v * y);
        a[3].add(v * z);
    }
    block_sums<4>(a, mn, mx);
    if (threadIdx.x == 0) {
        double* q = part + (size_t)blockIdx.x * 8;
        for (int k = 0; k < 4; ++k) { q[2 * k] = a[k].s; q[2 * k + 1] = a[k].c; }
    }
}

// centre[0..2] = barycentre in grid units.
__global__ __launch_bounds__(kReduceThreads) void k_moments_final(const double* __restrict__ part,
                                                                  int nparts,
                                                                  double* __restrict__ centre) {
    Acc a[4] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    double mn = 0.0, mx = 0.0;
    for (int b = threadIdx.x; b < nparts; b += kReduceThreads) {
        const double* q = part + (size_t)b * 8;
        for (int k = 0; k < 4; ++k) a[k].merge(q[2 * k], q[2 * k + 1]);
    }
    block_sums<4>(a, mn, mx);
    if (threadIdx.x == 0) {
        const double w = a[0].value();
        for (int k = 0; k < 3; ++k) centre[k] = a[k + 1].value() / w;
    }
}

// Pass 2: count, sum, min and max of the contour-point distances from the centre.
template <typename T>
__global__ __launch_bounds__(kReduceThreads) void k_contour_partial(const T* __restrict__ phi, int nx,
                                                                    int ny, int nz,
                                                                    const double* __restrict__ centre,
                                                                    double* __restrict__ part) {
    Acc a[2] = {{0.0, 0.0}, {0.0, 0.0}};   // count, sum R
    double mn = INFINITY, mx = -INFINITY;
    const double c[3] = {centre[0], centre[1], centre[2]};
    const int dims[3] = {nx, ny, nz};
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t stride = (int64_t)gridDim.x * kReduceThreads;
    for (int64_t i = (int64_t)blockIdx.x * kReduceThreads + threadIdx.x; i < n; i += stride) {
        const int p[3] = {(int)(i % nx), (int)((i / nx) % ny), (int)(i / ((int64_t)nx * ny))};
        const double va = (double)phi[i];
        for (int d = 0; d < 3; ++d) {
            int q[3] = {p[0], p[1], p[2]};
            q[d] = q[d] + 1 == dims[d] ? 0 : q[d] + 1;
            const double vb = (double)phi[((int64_t)q[2] * ny + q[1]) * nx + q[0]];
            if ((va - 0.5) * (vb - 0.5) > 0.0 || va == vb) continue;
            const double la = log((1.0 - va) / va), lb = log((1.0 - vb) / vb);
            const double t = la / (la - lb);
            double r2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                const double xk = (double)p[k] + (k == d ? t : 0.0) - c[k];
                r2 += xk * xk;
            }
            const double R = sqrt(r2);
            a[0].add(1.0);
            a[1].add(R);
            mn = fmin(mn, R);
            mx = fmax(mx, R);
        }
    }
    block_sums<2>(a, mn, mx);
    if (threadIdx.x == 0) {
        double* q = part + (size_t)blockIdx.x * 6;
        q[0] = a[0].s; q[1] = a[0].c; q[2] = a[1].s; q[3] = a[1].c; q[4] = mn; q[5] = mx;
    }
}

// out[0..3] = count, sum R, min R, max R (grid units).
__global__ __launch_bounds__(kReduceThreads) void k_contour_final(const double* __restrict__ part,
                                                                  int nparts,
                                                                  double* __restrict__ out) {
    Acc a[2] = {{0.0, 0.0}, {0.0, 0.0}};
    double mn = INFINITY, mx = -INFINITY;
    for (int b = threadIdx.x; b < nparts; b += kReduceThreads) {
        const double* q = part + (size_t)b * 6;
        a[0].merge(q[0], q[1]);
        a[1].merge(q[2], q[3]);
        mn = fmin(mn, q[4]);
        mx = fmax(mx, q[5]);
    }
    block_sums<2>(a, mn, mx);
    if (threadIdx.x == 0) {
        out[0] = a[0].value();
        out[1] = a[1].value();
        out[2] = mn;
        out[3] = mx;
    }
}

__device__ __forceinline__ double rising(double s, double four_over_lambda) {
    return 1.0 / (1.0 + exp(-four_over_lambda * s));
}

// Box particle: product over the axes of f(x - lo) f(hi - x), f the rising
// profile of Eq. 3 (f(s) = (1 + tanh(2 s / lambda)) / 2).
template <typename T>
__global__ __launch_bounds__(256) void k_init_box(T* __restrict__ phi, int nx, int ny, int nz,
                                                  double dx, double fol, double lx, double ly,
                                                  double lz, double hx, double hy, double hz) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)nx * ny * nz) return;
    const double pos[3] = {dx * (double)(i % nx), dx * (double)((i / nx) % ny),
                           dx * (double)(i / ((int64_t)nx * ny))};
    const double lo[3] = {lx, ly, lz}, hi[3] = {hx, hy, hz};
    double v = 1.0;
    for (int d = 0; d < 3; ++d) v *= rising(pos[d] - lo[d], fol) * rising(hi[d] - pos[d], fol);
    phi[i] = (T)v;
}

// ---- free energy of Eq. 1 (diagnostic, FP64) ----

// Directions r_k of Tab. 1 (one of each opposite pair), shell by shell.
__constant__ int kEdir[13][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1},
                                 {1, 1, 0}, {1, -1, 0}, {0, 1, 1}, {0, 1, -1}, {1, 0, 1}, {1, 0, -1},
                                 {1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {1, -1, -1}};

// Eq. 6 for one direction: g_k = (lambda^2 / rho^2) x T(z) with x = phi(1-phi),
// u = 1 - 2 phi, z = 4 a^2 x / (1 - a^2 u^2) and T(z) = 1 + (1-z) ln(1-z) / z,
// the printed expression with its two cancelling terms gathered (A2).  For
// z < 0.1 T is summed from its series sum_{m>=1} z^m / (m (m+1)), Horner,
// m <= 14 (truncation below 1e-17).
__device__ __forceinline__ double eq6_g(double x, double u, double a, double r2_over_l2) {
    const double q = a * a;
    if (q == 0.0 || x == 0.0) return 0.0;
    const double z = 4.0 * q * x / (1.0 - q * u * u);
    double t;
    if (z < 0.1) {
        t = 1.0 / (14.0 * 15.0);
        for (int m = 13; m >= 1; --m) t = 1.0 / (m * (m + 1.0)) + z * t;
        t *= z;
    } else {
        t = 1.0 + (1.0 - z) * log1p(-z) / z;
    }
    return x * t / r2_over_l2;
}

// Interpolation functions h(phi) of Tab. 2 for the mu h(phi) term.
__device__ __forceinline__ double interp_h(int which, double p) {
    if (which == kH5) return p * p * p * (10.0 - 15.0 * p + 6.0 * p * p);
    if (which == kHAbel) return p * p / (p * p + (1.0 - p) * (1.0 - p));
    return p * p * (3.0 - 2.0 * p);
}

// Energy density f_p of Eq. 1 at one point of the periodic grid: forward
// differences over the stencil's directions, the TI potential of Eq. 6 with
// a_k = tanh(2 r_k.n dx / lambda) (TI_n: n = grad psi / |grad psi| from
// central differences of psi = (lambda/4) ln((1-phi)/phi), both logarithm
// arguments floored at eps, n = (1,0,0) where |grad psi| < tau; TI_<hkl>: the
// fixed a_k), or the CF potential 8 x^2 / 3 per direction.
template <typename T>
__device__ double energy_density(const T* __restrict__ phi, int nx, int ny, int nz, int x, int y,
                                 int z, const EnergyCoef& c, int with_mu) {
    auto at = [&](int xx, int yy, int zz) {
        xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
        yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
        zz = zz < 0 ? zz + nz : (zz >= nz ? zz - nz : zz);
        return (double)phi[((size_t)zz * ny + yy) * nx + xx];
    };
    const double p0 = at(x, y, z);
    const double xx0 = p0 * (1.0 - p0), u = 1.0 - 2.0 * p0;
    double n[3] = {1.0, 0.0, 0.0};
    if (c.coupling == kLocal) {
        auto psi = [&](double v) {
            return 0.25 * c.lambda * (log(fmax(1.0 - v, c.eps)) - log(fmax(v, c.eps)));
        };
        const double g0 = (psi(at(x + 1, y, z)) - psi(at(x - 1, y, z))) / (2.0 * c.dx);
        const double g1 = (psi(at(x, y + 1, z)) - psi(at(x, y - 1, z))) / (2.0 * c.dx);
        const double g2 = (psi(at(x, y, z + 1)) - psi(at(x, y, z - 1))) / (2.0 * c.dx);
        const double gn = sqrt(g0 * g0 + g1 * g1 + g2 * g2);
        if (!(gn < c.tau)) {
            n[0] = g0 / gn;
            n[1] = g1 / gn;
            n[2] = g2 / gn;
        }
    }
    double s = 0.0;
    for (int k = 0; k < c.ndir; ++k) {
        const int j = k < 3 ? 1 : (k < 9 ? 2 : 3);
        const double rho2 = j * c.dx * c.dx;
        const double d = at(x + kEdir[k][0], y + kEdir[k][1], z + kEdir[k][2]) - p0;
        double g;
        if (c.coupling == kCF) {
            g = 8.0 * xx0 * xx0 / 3.0;
        } else {
            const double a = c.coupling == kGlobal
                                 ? c.ag[k]
                                 : tanh(2.0 * (kEdir[k][0] * n[0] + kEdir[k][1] * n[1] + kEdir[k][2] * n[2]) *
                                        c.dx / c.lambda);
            g = eq6_g(xx0, u, a, rho2 / (c.lambda * c.lambda));
        }
        s += c.w[j - 1] * (0.5 * c.lambda * c.lambda * d * d / rho2 + g);
    }
    double f = c.pref * s;
    if (with_mu) f += c.mu * interp_h(c.interp, p0);
    return f;
}

// Neumaier's compensated sum, and the exact combination of two (sum, error) pairs.
__device__ __forceinline__ void comp_add(double& s, double& e, double v) {
    const double t = s + v;
    e += fabs(s) >= fabs(v) ? (s - t) + v : (v - t) + s;
    s = t;
}

constexpr int kEnergyBlocks = 1024;

template <typename T>
__global__ __launch_bounds__(256) void k_energy_partial(const T* __restrict__ phi, int nx, int ny, int nz,
                                                        EnergyCoef c, int with_mu, double* __restrict__ part) {
    __shared__ double ss[256], se[256];
    double s = 0.0, e = 0.0;
    const int64_t total = (int64_t)nx * ny * nz;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((int64_t)nx * ny));
        comp_add(s, e, energy_density(phi, nx, ny, nz, x, y, z, c, with_mu));
    }
    ss[threadIdx.x] = s;
    se[threadIdx.x] = e;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            double a = ss[threadIdx.x], ea = se[threadIdx.x];
            comp_add(a, ea, ss[threadIdx.x + h]);
            ss[threadIdx.x] = a;
            se[threadIdx.x] = ea + se[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = ss[0];
        part[2 * blockIdx.x + 1] = se[0];
    }
}

// One thread: the block partials in order, compensated.
__global__ __launch_bounds__(64) void k_energy_final(const double* __restrict__ part, int nb, double dx3,
                                                     double* __restrict__ out) {
    if (threadIdx.x != 0) return;
    double s = 0.0, e = 0.0;
    for (int b = 0; b < nb; ++b) {
        comp_add(s, e, part[2 * b]);
        e += part[2 * b + 1];
    }
    out[0] = (s + e) * dx3;
}

// Radius of the phi = 1/2 surface along one ray from the centre (grid units):
// psi = ln((1-phi)/phi) of the clamped field (the inverse of Eq. 3 up to the
// factor lambda/4, which does not move its zero), trilinear between grid
// points of the periodic box, marched in steps of 1/4 from the centre to the
// first sample with psi >= 0, then bisected 44 times.  NaN where the centre is
// outside or the ray runs half the smallest box edge without crossing.  One
// thread per ray; FP64 throughout.
template <typename T>
__global__ __launch_bounds__(256) void k_ray_radii(const T* __restrict__ phi, int nx, int ny, int nz,
                                                   double cx, double cy, double cz,
                                                   const double* __restrict__ dirs, int n,
                                                   double* __restrict__ radii) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double ux = dirs[3 * i], uy = dirs[3 * i + 1], uz = dirs[3 * i + 2];
    const double norm = sqrt(ux * ux + uy * uy + uz * uz);
    ux /= norm;
    uy /= norm;
    uz /= norm;
    auto wrap = [](long v, int m) { v %= m; return (int)(v < 0 ? v + m : v); };
    auto psi_at = [&](long x, long y, long z) {
        const size_t at = ((size_t)wrap(z, nz) * ny + wrap(y, ny)) * nx + wrap(x, nx);
        const double f = fmin(fmax((double)phi[at], 1e-12), 1.0 - 1e-12);
        return log((1.0 - f) / f);
    };
    auto sample = [&](double t) {
        const double qx = cx + t * ux, qy = cy + t * uy, qz = cz + t * uz;
        const double fx = floor(qx), fy = floor(qy), fz = floor(qz);
        const double wx1 = qx - fx, wy1 = qy - fy, wz1 = qz - fz;
        const long ix = (long)fx, iy = (long)fy, iz = (long)fz;
        double val = 0.0;
        for (int dz = 0; dz < 2; ++dz) {
            const double wz = dz ? wz1 : 1.0 - wz1;
            for (int dy = 0; dy < 2; ++dy) {
                const double wy = dy ? wy1 : 1.0 - wy1;
                for (int dx = 0; dx < 2; ++dx) {
                    const double wx = dx ? wx1 : 1.0 - wx1;
                    val += wz * wy * wx * psi_at(ix + dx, iy + dy, iz + dz);
                }
            }
        }
        return val;
    };
    const double step = 0.25;
    const int kmax = (int)floor(0.5 * (double)min(nx, min(ny, nz)) / step);
    double r = __builtin_nan("");
    if (sample(0.0) < 0.0) {
        for (int k = 1; k <= kmax; ++k) {
            if (sample(k * step) >= 0.0) {
                double a = (k - 1) * step, b = k * step;
                for (int it = 0; it < 44; ++it) {
                    const double m = 0.5 * (a + b);
                    if (sample(m) >= 0.0) b = m; else a = m;
                }
                r = 0.5 * (a + b);
                break;
            }
        }
    }
    radii[i] = r;
}

}  // namespace

template <typename T>
hipError_t launch_cv_apply(const T* phi_old, T* phi_new, int64_t n, int interp, double dt_beta,
                           const unsigned long long* d_part, int nparts, unsigned long long* d_total,
                           double* d_state, hipStream_t s, T* phi_out) {
    if (nparts <= 0 || n <= 0) return hipErrorInvalidValue;
    if (nparts > kCvDirectParts) {   // one block adds them first: each apply block then reads one
        hipLaunchKernelGGL(k_cv_total, dim3(1), dim3(kReduceThreads), 0, s, d_part, nparts, d_total);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        d_part = d_total;
        nparts = 1;
    }
    hipLaunchKernelGGL((k_cv_apply<T>), dim3((unsigned)((n + kReduceThreads - 1) / kReduceThreads)),
                       dim3(kReduceThreads), 0, s, phi_new, phi_out ? phi_out : phi_new, phi_old, n, interp,
                       d_part, nparts, dt_beta, d_state);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cv_correct(const T* phi_old, T* phi_new, int64_t n, int interp, double dt_beta,
                             unsigned long long* d_part, double* d_state, hipStream_t s) {
    // about 16 points per thread of the partial pass, 64 to kReduceBlocks partials
    const int nparts = (int)std::min<int64_t>(kReduceBlocks, std::max<int64_t>(64, n / (16 * kReduceThreads)));
    hipLaunchKernelGGL((k_cv_partial<T>), dim3(nparts), dim3(kReduceThreads), 0, s, phi_old, phi_new, n,
                       interp, d_part);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_cv_apply<T>(phi_old, phi_new, n, interp, dt_beta, d_part, nparts, nullptr, d_state, s);
}

template <typename T>
hipError_t launch_energy(const T* phi, int nx, int ny, int nz, const EnergyCoef& c, int with_mu,
                         double* d_part, double* d_out, hipStream_t s) {
    hipLaunchKernelGGL((k_energy_partial<T>), dim3(kEnergyBlocks), dim3(256), 0, s, phi, nx, ny, nz, c,
                       with_mu, d_part);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(64), 0, s, d_part, kEnergyBlocks,
                       c.dx * c.dx * c.dx, d_out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ray_radii(const T* phi, int nx, int ny, int nz, const double* centre,
                           const double* d_dirs, int n, double* d_radii, hipStream_t s) {
    if (n < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_ray_radii<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, phi, nx, ny,
                       nz, centre[0], centre[1], centre[2], d_dirs, n, d_radii);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_contour_stats(const T* phi, int nx, int ny, int nz, double* d_part, double* d_out,
                                hipStream_t s) {
    // d_out[0..2]: barycentre, d_out[3..6]: count, sum R, min R, max R
    hipLaunchKernelGGL((k_moments_partial<T>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, phi,
                       nx, ny, nz, d_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_moments_final, dim3(1), dim3(kReduceThreads), 0, s, d_part, kReduceBlocks,
                       d_out);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_contour_partial<T>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, phi,
                       nx, ny, nz, d_out, d_part);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_contour_final, dim3(1), dim3(kReduceThreads), 0, s, d_part, kReduceBlocks,
                       d_out + 3);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_init_box(T* phi, int nx, int ny, int nz, double dx, double lambda,
                           const double lo[3], const double hi[3], hipStream_t s) {
    const int64_t n = (int64_t)nx * ny * nz;
    hipLaunchKernelGGL((k_init_box<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, phi, nx,
                       ny, nz, dx, 4.0 / lambda, lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]);
    return hipGetLastError();
}

template hipError_t launch_cv_correct<float>(const float*, float*, int64_t, int, double,
                                             unsigned long long*, double*, hipStream_t);
template hipError_t launch_cv_correct<double>(const double*, double*, int64_t, int, double,
                                              unsigned long long*, double*, hipStream_t);
template hipError_t launch_cv_apply<float>(const float*, float*, int64_t, int, double,
                                           const unsigned long long*, int, unsigned long long*, double*,
                                           hipStream_t, float*);
template hipError_t launch_cv_apply<double>(const double*, double*, int64_t, int, double,
                                            const unsigned long long*, int, unsigned long long*, double*,
                                            hipStream_t, double*);
template hipError_t launch_contour_stats<float>(const float*, int, int, int, double*, double*,
                                                hipStream_t);
template hipError_t launch_contour_stats<double>(const double*, int, int, int, double*, double*,
                                                 hipStream_t);
template hipError_t launch_energy<float>(const float*, int, int, int, const EnergyCoef&, int, double*,
                                        double*, hipStream_t);
template hipError_t launch_energy<double>(const double*, int, int, int, const EnergyCoef&, int, double*,
                                         double*, hipStream_t);
template hipError_t launch_ray_radii<float>(const float*, int, int, int, const double*,
                                            const double*, int, double*, hipStream_t);
template hipError_t launch_ray_radii<double>(const double*, int, int, int, const double*,
                                             const double*, int, double*, hipStream_t);
template hipError_t launch_init_box<float>(float*, int, int, int, double, double, const double*,
                                           const double*, hipStream_t);
template hipError_t launch_init_box<double>(double*, int, int, int, double, double, const double*,
                                            const double*, hipStream_t);

}  // namespace spfm
