// Contact-angle walls (Sec. 2.2, Eq. 7) and the interior <-> padded copies.
// (The tiled step kernels compute the ghosts they need as they stage them; the
// fill below serves the plain kernel.)
//
// A walled axis keeps one ghost layer at each end of the stored field.  Before
// every step the ghosts are set from the nearest interior point by the tanh
// addition law of the ideal profile: phi_g = (1 - a) phi_i / (1 - a (2 phi_i - 1))
// moves phi_i along the profile by the length d with tanh(2 d / lambda) = a.  A
// face ghost is shifted by dx sin(alpha) of its wall; an edge or corner ghost by
// the sum of the shifts of its two or three walls, in one application (the
// shifts of Eq. 7 compose by addition, so this equals applying Eq. 7 wall after
// wall).  The 27 composed coefficients are computed on the host.
//
// Every ghost thread reads one interior point and writes one ghost point, so
// the fill has no ordering between threads.
#include "spfm_impl.h"

namespace spfm {

namespace {

// Ghost point i of the stored field phi (i beyond the ghost count: nothing).
template <typename T>
__device__ __forceinline__ void fill_ghost(T* __restrict__ phi, const WallCoef<T>& w, int64_t i) {
    const int SX = w.sx, SY = w.sy, SZ = w.sz;
    const int gx = w.walls & 1, gy = (w.walls >> 1) & 1, gz = (w.walls >> 2) & 1;
    // Ghost cells in three disjoint sets: the x-ghost planes (all y, z), the
    // y-ghost planes (interior x, all z), the z-ghost planes (interior x, y).
    const int64_t n1 = gx ? 2 * (int64_t)SY * SZ : 0;
    const int64_t n2 = gy ? 2 * (int64_t)(SX - 2 * gx) * SZ : 0;
    const int64_t n3 = gz ? 2 * (int64_t)(SX - 2 * gx) * (SY - 2 * gy) : 0;
    int X, Y, Z;
    if (i < n1) {
        const int64_t q = i >> 1;
        X = (i & 1) ? SX - 1 : 0;
        Y = (int)(q % SY);
        Z = (int)(q / SY);
    } else if (i < n1 + n2) {
        const int64_t j = i - n1, q = j >> 1, nxi = SX - 2 * gx;
        Y = (j & 1) ? SY - 1 : 0;
        X = gx + (int)(q % nxi);
        Z = (int)(q / nxi);
    } else if (i < n1 + n2 + n3) {
        const int64_t j = i - n1 - n2, q = j >> 1, nxi = SX - 2 * gx;
        Z = (j & 1) ? SZ - 1 : 0;
        X = gx + (int)(q % nxi);
        Y = gy + (int)(q / nxi);
    } else {
        return;
    }
    // Nearest interior point and the walls crossed on the way to it.
    const int cx = (gx && X == 0) ? -1 : ((gx && X == SX - 1) ? 1 : 0);
    const int cy = (gy && Y == 0) ? -1 : ((gy && Y == SY - 1) ? 1 : 0);
    const int cz = (gz && Z == 0) ? -1 : ((gz && Z == SZ - 1) ? 1 : 0);
    const int64_t src = ((int64_t)(Z - cz) * SY + (Y - cy)) * SX + (X - cx);
    const int64_t dst = ((int64_t)Z * SY + Y) * SX + X;
    phi[dst] = wall_map(phi[src], w.a[(cx + 1) + 3 * (cy + 1) + 9 * (cz + 1)]);
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill_walls(T* __restrict__ phi, WallCoef<T> w) {
    fill_ghost(phi, w, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

// dst box origin (dx0, dy0, dz0) in a dst field of dims (dnx, dny), src likewise;
// n = (bx, by, bz) points copied.
template <typename T>
__global__ __launch_bounds__(256) void k_box_copy(T* __restrict__ dst, int dnx, int dny, int dx0,
                                                  int dy0, int dz0, const T* __restrict__ src,
                                                  int snx, int sny, int sx0, int sy0, int sz0,
                                                  int bx, int by, int bz) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)bx * by * bz) return;
    const int x = (int)(i % bx);
    const int y = (int)((i / bx) % by);
    const int z = (int)(i / ((int64_t)bx * by));
    dst[((int64_t)(z + dz0) * dny + (y + dy0)) * dnx + (x + dx0)] =
        src[((int64_t)(z + sz0) * sny + (y + sy0)) * snx + (x + sx0)];
}

__device__ __forceinline__ double logistic(double t, double four_over_lambda) {
    return 1.0 / (1.0 + exp(-four_over_lambda * t));
}

// Eq. 3 for one planar front: phi = L(c - s), s = dx (x, y, z) . n.
template <typename T>
__global__ __launch_bounds__(256) void k_init_front(T* __restrict__ phi, int nx, int ny, int nz,
                                                    double dx, double fol, double nvx, double nvy,
                                                    double nvz, double c) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)nx * ny * nz) return;
    const int x = (int)(i % nx);
    const int y = (int)((i / nx) % ny);
    const int z = (int)(i / ((int64_t)nx * ny));
    const double s = dx * ((double)x * nvx + (double)y * nvy + (double)z * nvz);
    phi[i] = (T)logistic(c - s, fol);
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

int64_t wall_ghosts(int sx, int sy, int sz, int walls) {
    const int gx = walls & 1, gy = (walls >> 1) & 1, gz = (walls >> 2) & 1;
    return (gx ? 2 * (int64_t)sy * sz : 0) + (gy ? 2 * (int64_t)(sx - 2 * gx) * sz : 0) +
           (gz ? 2 * (int64_t)(sx - 2 * gx) * (sy - 2 * gy) : 0);
}

template <typename T>
hipError_t launch_fill_walls(T* phi, const WallCoef<T>& w, int64_t nghost, hipStream_t s) {
    if (nghost <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_fill_walls<T>), dim3(blocks_for(nghost)), dim3(256), 0, s, phi, w);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_box_copy(T* dst, int dnx, int dny, int dx0, int dy0, int dz0, const T* src,
                           int snx, int sny, int sx0, int sy0, int sz0, int bx, int by, int bz,
                           hipStream_t s) {
    const int64_t n = (int64_t)bx * by * bz;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_box_copy<T>), dim3(blocks_for(n)), dim3(256), 0, s, dst, dnx, dny, dx0,
                       dy0, dz0, src, snx, sny, sx0, sy0, sz0, bx, by, bz);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_init_front(T* phi, int nx, int ny, int nz, double dx, double lambda,
                             const double n[3], double offset, hipStream_t s) {
    const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    const double nv[3] = {n[0] / nn, n[1] / nn, n[2] / nn};
    const double c = 0.5 * dx * (nx * nv[0] + ny * nv[1] + nz * nv[2]) + offset;
    const int64_t np = (int64_t)nx * ny * nz;
    hipLaunchKernelGGL((k_init_front<T>), dim3(blocks_for(np)), dim3(256), 0, s, phi, nx, ny, nz,
                       dx, 4.0 / lambda, nv[0], nv[1], nv[2], c);
    return hipGetLastError();
}

template hipError_t launch_fill_walls<float>(float*, const WallCoef<float>&, int64_t, hipStream_t);
template hipError_t launch_fill_walls<double>(double*, const WallCoef<double>&, int64_t, hipStream_t);
template hipError_t launch_box_copy<float>(float*, int, int, int, int, int, const float*, int, int,
                                           int, int, int, int, int, int, hipStream_t);
template hipError_t launch_box_copy<double>(double*, int, int, int, int, int, const double*, int,
                                            int, int, int, int, int, int, int, hipStream_t);
template hipError_t launch_init_front<float>(float*, int, int, int, double, double, const double*,
                                             double, hipStream_t);
template hipError_t launch_init_front<double>(double*, int, int, int, double, double, const double*,
                                              double, hipStream_t);

}  // namespace spfm
