// Step kernels of the SPFM GPU library (forward Euler of Eq. 2): the plain
// kernel and the dispatch of the tiled and batched steps.
//
//  k_step_plain  one thread per point; the 27-point neighbourhood is read
//                straight from global memory with periodic index wrap.
//  tiled/batched the z-marching LDS sweep of sweep.h, compiled per kernel
//                coupling in its own translation unit (step_*.hip) for every
//                tile shape the autotuner may pick.
#include <type_traits>

#include "spfm_impl.h"

namespace spfm {

namespace {

__device__ __forceinline__ int wrap_plain(int i, int n) {
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

template <typename T, int S, int C>
__global__ __launch_bounds__(256) void k_step_plain(const T* __restrict__ in, T* __restrict__ out,
                                                    StepCoef<T> k) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= k.nx || y >= k.ny) return;
    const int nx = k.nx, ny = k.ny, nz = k.nz;
    const int xi[3] = {wrap_plain(x - 1, nx), x, wrap_plain(x + 1, nx)};
    const int yi[3] = {wrap_plain(y - 1, ny), y, wrap_plain(y + 1, ny)};
    const int zi[3] = {wrap_plain(z - 1, nz), z, wrap_plain(z + 1, nz)};
    auto at = [&](int dx, int dy, int dz) -> T {
        return in[((size_t)zi[dz + 1] * ny + yi[dy + 1]) * nx + xi[dx + 1]];
    };
    auto grad = [&](T& gx, T& gy, T& gz) {
        gx = psi2(at(1, 0, 0), k.eps) - psi2(at(-1, 0, 0), k.eps);
        gy = psi2(at(0, 1, 0), k.eps) - psi2(at(0, -1, 0), k.eps);
        gz = psi2(at(0, 0, 1), k.eps) - psi2(at(0, 0, -1), k.eps);
    };
    out[((size_t)z * ny + y) * nx + x] = point_update<T, S, C>(at, grad, k);
}

template <typename T, template <typename, int, int> class Launch, typename... Args>
hipError_t dispatch(int stencil, int coupling, Args&&... args) {
#define SPFM_CASE(S_, C_)                                   \
    if (stencil == S_ && coupling == C_) {                  \
        return Launch<T, S_, C_>::run(args...);             \
    }
    SPFM_CASE(6, kLocal) SPFM_CASE(6, kGlobal) SPFM_CASE(6, kCF)
    SPFM_CASE(18, kLocal) SPFM_CASE(18, kGlobal) SPFM_CASE(18, kCF)
    SPFM_CASE(26, kLocal) SPFM_CASE(26, kGlobal) SPFM_CASE(26, kCF)
    SPFM_CASE(6, kCF5) SPFM_CASE(18, kCF5) SPFM_CASE(26, kCF5)
    SPFM_CASE(6, kCFAbel) SPFM_CASE(18, kCFAbel) SPFM_CASE(26, kCFAbel)
#undef SPFM_CASE
    return hipErrorInvalidValue;
}

template <typename T, int S, int C>
struct PlainLaunch {
    static hipError_t run(const T* in, T* out, const StepCoef<T>& k, hipStream_t s) {
        dim3 block(64, 4, 1);
        dim3 grid((k.nx + 63) / 64, (k.ny + 3) / 4, k.nz);
        hipLaunchKernelGGL((k_step_plain<T, S, C>), grid, block, 0, s, in, out, k);
        return hipGetLastError();
    }
};

}  // namespace

template <typename T>
hipError_t launch_step_plain(const T* in, T* out, const StepCoef<T>& k, int stencil, int coupling,
                             hipStream_t s) {
    return dispatch<T, PlainLaunch>(stencil, coupling, in, out, k, s);
}

template <typename T>
hipError_t launch_step_tiled(const T* in, T* out, const StepCoef<T>& k, int stencil, int coupling,
                             int tile, const TileItem* d_items, int nitems, const WallCoef<T>* d_wall,
                             unsigned long long* cv_part, const CvFuse<T>* fuse, hipStream_t s) {
    if (cv_part && d_wall) return hipErrorInvalidValue;
    switch (coupling) {
        case kLocal: return launch_tiled_coupling<T, kLocal>(in, out, k, stencil, tile, d_items, nitems, d_wall, cv_part, fuse, s);
        case kGlobal: return launch_tiled_coupling<T, kGlobal>(in, out, k, stencil, tile, d_items, nitems, d_wall, cv_part, fuse, s);
        case kCF: return launch_tiled_coupling<T, kCF>(in, out, k, stencil, tile, d_items, nitems, d_wall, cv_part, fuse, s);
        case kCF5: return launch_tiled_coupling<T, kCF5>(in, out, k, stencil, tile, d_items, nitems, d_wall, cv_part, fuse, s);
        case kCFAbel: return launch_tiled_coupling<T, kCFAbel>(in, out, k, stencil, tile, d_items, nitems, d_wall, cv_part, fuse, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step_batched(const float* buf_in, float* buf_out, const StepCoef<float>* d_coef,
                               const int64_t* d_offset, const TileItem* d_items, int nitems,
                               const WallCoef<float>* d_wall, int stencil, int coupling, int tile,
                               hipStream_t s) {
    switch (coupling) {
        case kLocal: return launch_batched_coupling<kLocal>(buf_in, buf_out, d_coef, d_offset, stencil, tile, d_items, nitems, d_wall, s);
        case kGlobal: return launch_batched_coupling<kGlobal>(buf_in, buf_out, d_coef, d_offset, stencil, tile, d_items, nitems, d_wall, s);
        case kCF: return launch_batched_coupling<kCF>(buf_in, buf_out, d_coef, d_offset, stencil, tile, d_items, nitems, d_wall, s);
        case kCF5: return launch_batched_coupling<kCF5>(buf_in, buf_out, d_coef, d_offset, stencil, tile, d_items, nitems, d_wall, s);
        case kCFAbel: return launch_batched_coupling<kCFAbel>(buf_in, buf_out, d_coef, d_offset, stencil, tile, d_items, nitems, d_wall, s);
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_step_plain<float>(const float*, float*, const StepCoef<float>&, int, int,
                                             hipStream_t);
template hipError_t launch_step_plain<double>(const double*, double*, const StepCoef<double>&, int,
                                              int, hipStream_t);
template hipError_t launch_step_tiled<float>(const float*, float*, const StepCoef<float>&, int, int,
                                             int, const TileItem*, int, const WallCoef<float>*,
                                             unsigned long long*, const CvFuse<float>*, hipStream_t);
template hipError_t launch_step_tiled<double>(const double*, double*, const StepCoef<double>&, int,
                                              int, int, const TileItem*, int, const WallCoef<double>*,
                                              unsigned long long*, const CvFuse<double>*, hipStream_t);

}  // namespace spfm
