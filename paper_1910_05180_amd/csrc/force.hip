// Force density of a field: the bracket of Eq. 4 summed over the stencil's
// directions at every point, i.e. the right-hand side of Eq. 2 without the
// driving force (the functional derivative of Eq. 1's interface terms), times
// dt A so that it shares the step's coefficients.  Summed over the system it is
// the total force on an interface (the grid-friction study of Fig. 3), with no
// forward-Euler update and no difference of two field sums in between.
//
// One thread per interior point reads its 27-point neighbourhood with periodic
// wrap (walled axes: the ghost layers hold Eq. 7 values, filled beforehand) and
// evaluates the same per-point increment as the plain step kernel.
#include "spfm_impl.h"

namespace spfm {

namespace {

__device__ __forceinline__ int wrap_f(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

template <typename T, int S, int C>
__global__ __launch_bounds__(256) void k_force_density(const T* __restrict__ phi, T* __restrict__ dens,
                                                       StepCoef<T> k, int wx, int wy, int wz) {
    const int sx = k.nx, sy = k.ny, sz = k.nz;
    const int nxi = sx - 2 * wx, nyi = sy - 2 * wy, nzi = sz - 2 * wz;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)nxi * nyi * nzi) return;
    const int x = (int)(i % nxi) + wx;
    const int y = (int)((i / nxi) % nyi) + wy;
    const int z = (int)(i / ((int64_t)nxi * nyi)) + wz;
    const int xi[3] = {wrap_f(x - 1, sx), x, wrap_f(x + 1, sx)};
    const int yi[3] = {wrap_f(y - 1, sy), y, wrap_f(y + 1, sy)};
    const int zi[3] = {wrap_f(z - 1, sz), z, wrap_f(z + 1, sz)};
    auto at = [&](int dx, int dy, int dz) -> T {
        return phi[((size_t)zi[dz + 1] * sy + yi[dy + 1]) * sx + xi[dx + 1]];
    };
    auto grad = [&](T& gx, T& gy, T& gz) {
        gx = psi2(at(1, 0, 0), k.eps) - psi2(at(-1, 0, 0), k.eps);
        gy = psi2(at(0, 1, 0), k.eps) - psi2(at(0, -1, 0), k.eps);
        gz = psi2(at(0, 0, 1), k.eps) - psi2(at(0, 0, -1), k.eps);
    };
    dens[i] = point_rate_dt<T, S, C>(at, grad, k);
}

}  // namespace

template <typename T>
hipError_t launch_force_density(const T* phi, T* dens, const StepCoef<T>& k, int walls, int stencil,
                                int coupling, hipStream_t s) {
    const int wx = walls & 1, wy = (walls >> 1) & 1, wz = (walls >> 2) & 1;
    const int64_t n = (int64_t)(k.nx - 2 * wx) * (k.ny - 2 * wy) * (k.nz - 2 * wz);
    if (n <= 0) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((n + 255) / 256));
#define SPFM_FCASE(S_, C_)                                                                        \
    if (stencil == S_ && coupling == C_) {                                                        \
        hipLaunchKernelGGL((k_force_density<T, S_, C_>), grid, dim3(256), 0, s, phi, dens, k, wx, wy, \
                           wz);                                                                   \
        return hipGetLastError();                                                                 \
    }
    SPFM_FCASE(6, kLocal) SPFM_FCASE(6, kGlobal) SPFM_FCASE(6, kCF)
    SPFM_FCASE(18, kLocal) SPFM_FCASE(18, kGlobal) SPFM_FCASE(18, kCF)
    SPFM_FCASE(26, kLocal) SPFM_FCASE(26, kGlobal) SPFM_FCASE(26, kCF)
    SPFM_FCASE(6, kCF5) SPFM_FCASE(18, kCF5) SPFM_FCASE(26, kCF5)
    SPFM_FCASE(6, kCFAbel) SPFM_FCASE(18, kCFAbel) SPFM_FCASE(26, kCFAbel)
#undef SPFM_FCASE
    return hipErrorInvalidValue;
}

template hipError_t launch_force_density<float>(const float*, float*, const StepCoef<float>&, int, int,
                                                int, hipStream_t);
template hipError_t launch_force_density<double>(const double*, double*, const StepCoef<double>&, int,
                                                 int, int, hipStream_t);

}  // namespace spfm
