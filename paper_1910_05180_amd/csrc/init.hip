// Initial fields from the ideal profile of Eq. 3, evaluated in FP64 on the
// device and stored in the field dtype.
//
// With the logistic form of Eq. 3, phi = L(c - s), L(t) = 1/(1 + exp(-4t/lambda)):
//  planar:  periodic slab of integer normal N.  s = p.N/|N| - c is reduced to
//           one period P and the field is the sum over periodic images m of
//           the top hat L(s_m + P/4) - L(s_m - P/4), s_m = s - mP, written
//           without cancellation as L(s_m + P/4) L(P/4 - s_m) (1 - exp(-2P/lambda)).
//  spheres: phi = 1 - prod_i (1 - phi_i), phi_i = L(R_i - |p - c_i|) with the
//           minimum-image distance, accumulated as sum_i phi_i prod_{j<i}(1 - phi_j)
//           so that small tail values keep their relative accuracy.
#include <mutex>

#include "spfm_impl.h"

namespace spfm {

// Device staging of the sphere table for the allocation-free initialisation
// (4 doubles per sphere: centre x, y, z, radius).  One copy per GPU, held
// until the process ends; every call on a GPU overwrites it.  In host code the
// array's name is not a device address: host code uses the pointer that
// sphere_scratch() obtains from the runtime for the current device.
static __device__ __align__(256) double scratch[4 * kMaxScratchSpheres];

namespace {

__device__ __forceinline__ double logistic(double t, double four_over_lambda) {
    return 1.0 / (1.0 + exp(-four_over_lambda * t));
}

template <typename T>
__global__ __launch_bounds__(256) void k_init_planar(T* __restrict__ phi, int nx, int ny, int nz,
                                                     double dx, double fol, double nvx, double nvy,
                                                     double nvz, double c, double P, double e0,
                                                     int K) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n = (int64_t)nx * ny * nz;
    if (i >= n) return;
    const int x = (int)(i % nx);
    const int y = (int)((i / nx) % ny);
    const int z = (int)(i / ((int64_t)nx * ny));
    double s = dx * ((double)x * nvx + (double)y * nvy + (double)z * nvz) - c;
    s -= P * rint(s / P);
    double v = 0.0;
    for (int m = -K; m <= K; ++m) {
        const double sm = s - m * P;
        v += logistic(sm + 0.25 * P, fol) * logistic(0.25 * P - sm, fol);
    }
    phi[i] = (T)(v * e0);
}

template <typename T>
__global__ __launch_bounds__(256) void k_init_spheres(T* __restrict__ phi, int nx, int ny, int nz,
                                                      double dx, double fol, double cutoff,
                                                      int nsph, const double* __restrict__ sph) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n = (int64_t)nx * ny * nz;
    if (i >= n) return;
    const int x = (int)(i % nx);
    const int y = (int)((i / nx) % ny);
    const int z = (int)(i / ((int64_t)nx * ny));
    const double L[3] = {nx * dx, ny * dx, nz * dx};
    const double pos[3] = {x * dx, y * dx, z * dx};
    double acc = 0.0, q = 1.0;
    for (int g = 0; g < nsph; ++g) {
        double r2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            double d = pos[a] - sph[4 * g + a];
            d -= L[a] * rint(d / L[a]);
            r2 += d * d;
        }
        const double r = sqrt(r2) - sph[4 * g + 3];
        if (r > cutoff) continue;   // profile below 1e-300: contributes nothing
        const double v = logistic(-r, fol);
        acc += q * v;
        q *= 1.0 - v;
    }
    phi[i] = (T)acc;
}

int64_t gcd64(int64_t a, int64_t b) {
    if (a < 0) a = -a;
    if (b < 0) b = -b;
    while (b) { const int64_t t = a % b; a = b; b = t; }
    return a;
}

}  // namespace

template <typename T>
hipError_t launch_init_planar(T* phi, int nx, int ny, int nz, double dx, double lambda,
                              const int hkl[3], double offset, hipStream_t s) {
    const double nn = sqrt((double)hkl[0] * hkl[0] + (double)hkl[1] * hkl[1] + (double)hkl[2] * hkl[2]);
    int64_t g = gcd64(gcd64(gcd64(0, (int64_t)nx * hkl[0]), (int64_t)ny * hkl[1]), (int64_t)nz * hkl[2]);
    const double P = (double)g * dx / nn;
    const double nv[3] = {hkl[0] / nn, hkl[1] / nn, hkl[2] / nn};
    const double c = 0.5 * dx * (nx * nv[0] + ny * nv[1] + nz * nv[2]) + offset;
    const int K = 2 + (int)ceil(10.0 * lambda / P);
    const double e0 = -expm1(-2.0 * P / lambda);
    const int64_t n = (int64_t)nx * ny * nz;
    hipLaunchKernelGGL((k_init_planar<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, phi,
                       nx, ny, nz, dx, 4.0 / lambda, nv[0], nv[1], nv[2], c, P, e0, K);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_init_spheres(T* phi, int nx, int ny, int nz, double dx, double lambda, int nsph,
                               const double* d_spheres, hipStream_t s) {
    const int64_t n = (int64_t)nx * ny * nz;
    const double cutoff = lambda * 0.25 * 700.0;   // exp(-4 r / lambda) < 1e-300
    hipLaunchKernelGGL((k_init_spheres<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       phi, nx, ny, nz, dx, 4.0 / lambda, cutoff, nsph, d_spheres);
    return hipGetLastError();
}

hipError_t sphere_scratch(double** out) {
    constexpr int kMaxDevices = 64;
    static std::mutex lock;
    static double* ptr[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> guard(lock);
    if (!ptr[dev]) {   // once per device, with that device current
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        ptr[dev] = static_cast<double*>(p);
    }
    *out = ptr[dev];
    return hipSuccess;
}

template hipError_t launch_init_planar<float>(float*, int, int, int, double, double, const int*,
                                              double, hipStream_t);
template hipError_t launch_init_planar<double>(double*, int, int, int, double, double, const int*,
                                               double, hipStream_t);
template hipError_t launch_init_spheres<float>(float*, int, int, int, double, double, int,
                                               const double*, hipStream_t);
template hipError_t launch_init_spheres<double>(double*, int, int, int, double, double, int,
                                                const double*, hipStream_t);

}  // namespace spfm
