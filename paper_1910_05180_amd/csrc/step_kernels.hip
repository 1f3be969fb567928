// Step kernels of the SPFM GPU library (forward Euler of Eq. 2, periodic grid).
//
//  k_step_plain  one thread per point; the 27-point neighbourhood is read
//                straight from global memory with periodic index wrap.
//  k_step_tiled  a 512-thread block owns a 64 x 8 column of the grid and
//                marches it along z over kTileZ planes (see tile_sweep): every
//                plane is read from HBM once with coalesced rows, one plane ahead
//                of its use, staged with its halo in LDS, and reduced by each
//                thread to a few per-plane partial sums kept in registers.  For
//                TI_n the log-ratio psi' of every staged cell is computed once.
//  k_step_batched the tiled sweep over a flat list of (grid, tile) items that
//                covers many independent grids in one launch.
#include "spfm_impl.h"

namespace spfm {

namespace {

__device__ __forceinline__ int wrap_once(int i, int n) {
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
    const int xi[3] = {wrap_once(x - 1, nx), x, wrap_once(x + 1, nx)};
    const int yi[3] = {wrap_once(y - 1, ny), y, wrap_once(y + 1, ny)};
    const int zi[3] = {wrap_once(z - 1, nz), z, wrap_once(z + 1, nz)};
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

// Per-column values a thread keeps for one plane q of its z-march.
template <typename T>
struct PlaneRegs {
    T c;        // phi at the column
    T fc;       // sum over the 4 in-plane face neighbours of (phi - c)
    T dc;       // sum over the 4 in-plane diagonal neighbours of (phi - c)
    T gx, gy;   // LOCAL: in-plane central differences of psi' at the column
    T pc;       // LOCAL: psi' at the column
};

// One block sweeps the tile [x0, x0+kTileX) x [y0, y0+kTileY) x [z0, z0+kTileZ)
// (clipped to the grid).  Each plane of the tile plus a one-cell halo is loaded
// once (coalesced rows, one plane ahead of its use) into a two-slot LDS ring,
// together with psi' of every cell for TI_n.  Every thread reads its 3x3
// in-plane neighbourhood of the newest plane once and keeps per-plane partial
// sums for planes z-1, z, z+1 in registers; with them the 26-neighbour shell
// sums of point z are
//   s1 = fc(z) + e,  s2 = dc(z) + fc(z-1) + fc(z+1) + 4e,  s3 = dc(z-1) + dc(z+1) + 4e,
//   e = (c(z-1) - c(z)) + (c(z+1) - c(z)),
// all built from differences of nearby values.
template <typename T, int S, int C>
__device__ __forceinline__ void tile_sweep(const T* __restrict__ in, T* __restrict__ out,
                                           const StepCoef<T>& k, int x0, int y0, int z0,
                                           T* __restrict__ sphi, T* __restrict__ spsi) {
    constexpr int HX = kTileX + 2, HY = kTileY + 2, HP = HX * HY;
    constexpr int NT = kTileX * kTileY;
    constexpr int NL = (HP + NT - 1) / NT;   // halo cells loaded per thread
    const int tid = threadIdx.x;
    const int tx = tid % kTileX, ty = tid / kTileX;
    const int nx = k.nx, ny = k.ny, nz = k.nz;
    const size_t plane = (size_t)nx * ny;

    // In-plane offsets of this thread's halo cells (fixed along the sweep).
    int loff[NL];
    bool lval[NL];
#pragma unroll
    for (int c = 0; c < NL; ++c) {
        const int cell = tid + c * NT;
        lval[c] = cell < HP;
        int gx = x0 - 1 + cell % HX, gy = y0 - 1 + cell / HX;
        gx %= nx; if (gx < 0) gx += nx;
        gy %= ny; if (gy < 0) gy += ny;
        loff[c] = lval[c] ? gy * nx + gx : 0;
    }
    const int zend = min(z0 + kTileZ, nz);

    auto fetch = [&](int zz, T (&v)[NL]) {
        const T* src = in + (size_t)wrap_once(zz, nz) * plane;
#pragma unroll
        for (int c = 0; c < NL; ++c) v[c] = lval[c] ? src[loff[c]] : T(0);
    };
    auto stage = [&](int slot, const T (&v)[NL]) {
        T* dphi = sphi + slot * HP;
        T* dpsi = spsi + slot * HP;
#pragma unroll
        for (int c = 0; c < NL; ++c) {
            if (lval[c]) {
                dphi[tid + c * NT] = v[c];
                if (C == kLocal) dpsi[tid + c * NT] = psi2(v[c], k.eps);
            }
        }
    };
    const int cc = (ty + 1) * HX + (tx + 1);
    auto load = [&](int slot, PlaneRegs<T>& R) {
        const T* P = sphi + slot * HP;
        const T c = P[cc];
        R.c = c;
        R.fc = ((P[cc + 1] - c) + (P[cc - 1] - c)) + ((P[cc + HX] - c) + (P[cc - HX] - c));
        if (S >= 18)
            R.dc = ((P[cc + HX + 1] - c) + (P[cc - HX - 1] - c)) +
                   ((P[cc + HX - 1] - c) + (P[cc - HX + 1] - c));
        if (C == kLocal) {
            const T* Q = spsi + slot * HP;
            R.gx = Q[cc + 1] - Q[cc - 1];
            R.gy = Q[cc + HX] - Q[cc - HX];
            R.pc = Q[cc];
        }
    };
    const bool active = (x0 + tx < nx) && (y0 + ty < ny);
    T* dst = out + (size_t)(y0 + ty) * nx + (x0 + tx);

    // Output plane z with planes z-1, z, z+1 in Rm, R0, Rp; Rp is filled here.
    // Relative plane index r = z - z0 + 1 (z0 - 1 is r = 0); plane r sits in slot r & 1.
    auto step = [&](int z, const PlaneRegs<T>& Rm, const PlaneRegs<T>& R0, PlaneRegs<T>& Rp) {
        const int r = z - z0 + 1;
        __syncthreads();   // plane r+1 staged; every read of slot (r+2) & 1 done
        const bool more = z + 1 < zend;
        T pre[NL];
        if (more) fetch(z + 2, pre);
        load((r + 1) & 1, Rp);
        if (active) {
            const T p = R0.c;
            const T e = (Rm.c - p) + (Rp.c - p);
            const T s1 = R0.fc + e;
            T s2 = T(0), s3 = T(0);
            if (S >= 18) s2 = fma(T(4), e, R0.dc + (Rm.fc + Rp.fc));
            if (S >= 26) s3 = fma(T(4), e, Rm.dc + Rp.dc);
            auto grad = [&](T& gx, T& gy, T& gz) {
                gx = R0.gx;
                gy = R0.gy;
                gz = Rp.pc - Rm.pc;
            };
            dst[(size_t)z * plane] = point_core<T, S, C>(p, s1, s2, s3, grad, k);
        }
        if (more) stage((r + 2) & 1, pre);
    };

    PlaneRegs<T> A{}, B{}, D{};
    {
        T v[NL];
        fetch(z0 - 1, v);
        stage(0, v);
        fetch(z0, v);
        stage(1, v);
        __syncthreads();
        load(0, A);
        load(1, B);
        fetch(z0 + 1, v);
        __syncthreads();
        stage(0, v);
    }
    // Unrolled by three so that the plane registers rotate without moves.
    for (int z = z0; z < zend;) {
        step(z, A, B, D);
        if (++z >= zend) break;
        step(z, B, D, A);
        if (++z >= zend) break;
        step(z, D, A, B);
        ++z;
    }
}

template <typename T>
struct Smem {
    static constexpr int HP = (kTileX + 2) * (kTileY + 2);
};

template <typename T, int S, int C>
__global__ __launch_bounds__(kTileX* kTileY) void k_step_tiled(const T* __restrict__ in,
                                                               T* __restrict__ out, StepCoef<T> k,
                                                               int ntx, int nty, int ntiles) {
    __shared__ T sphi[2 * Smem<T>::HP];
    __shared__ T spsi[C == kLocal ? 2 * Smem<T>::HP : 1];
    const int t = xcd_remap(blockIdx.x, ntiles);
    const int tx = t % ntx, ty = (t / ntx) % nty, tz = t / (ntx * nty);
    tile_sweep<T, S, C>(in, out, k, tx * kTileX, ty * kTileY, tz * kTileZ, sphi, spsi);
}

template <int S, int C>
__global__ __launch_bounds__(kTileX* kTileY) void k_step_batched(
    const float* __restrict__ buf_in, float* __restrict__ buf_out,
    const StepCoef<float>* __restrict__ coef, const int64_t* __restrict__ offset,
    const TileItem* __restrict__ items) {
    __shared__ float sphi[2 * Smem<float>::HP];
    __shared__ float spsi[C == kLocal ? 2 * Smem<float>::HP : 1];
    const TileItem it = items[blockIdx.x];
    const StepCoef<float> k = coef[it.inst];
    const int64_t off = offset[it.inst];
    tile_sweep<float, S, C>(buf_in + off, buf_out + off, k, it.x0, it.y0, it.z0, sphi, spsi);
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

template <typename T, int S, int C>
struct TiledLaunch {
    static hipError_t run(const T* in, T* out, const StepCoef<T>& k, hipStream_t s) {
        const int ntx = (k.nx + kTileX - 1) / kTileX, nty = (k.ny + kTileY - 1) / kTileY;
        const int ntz = (k.nz + kTileZ - 1) / kTileZ;
        const int64_t n = (int64_t)ntx * nty * ntz;
        if (n > 0x7fffffff) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_step_tiled<T, S, C>), dim3((unsigned)n), dim3(kTileX * kTileY), 0, s,
                           in, out, k, ntx, nty, (int)n);
        return hipGetLastError();
    }
};

template <typename T, int S, int C>
struct BatchedLaunch {
    static hipError_t run(const float* in, float* out, const StepCoef<float>* coef,
                          const int64_t* offset, const TileItem* items, int nitems, hipStream_t s) {
        if (nitems <= 0) return hipSuccess;
        hipLaunchKernelGGL((k_step_batched<S, C>), dim3(nitems), dim3(kTileX * kTileY), 0, s, in,
                           out, coef, offset, items);
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
                             hipStream_t s) {
    return dispatch<T, TiledLaunch>(stencil, coupling, in, out, k, s);
}

hipError_t launch_step_batched(const float* buf_in, float* buf_out, const StepCoef<float>* d_coef,
                               const int64_t* d_offset, const TileItem* d_items, int nitems,
                               int stencil, int coupling, hipStream_t s) {
    return dispatch<float, BatchedLaunch>(stencil, coupling, buf_in, buf_out, d_coef, d_offset,
                                          d_items, nitems, s);
}

template hipError_t launch_step_plain<float>(const float*, float*, const StepCoef<float>&, int, int,
                                             hipStream_t);
template hipError_t launch_step_plain<double>(const double*, double*, const StepCoef<double>&, int,
                                              int, hipStream_t);
template hipError_t launch_step_tiled<float>(const float*, float*, const StepCoef<float>&, int, int,
                                             hipStream_t);
template hipError_t launch_step_tiled<double>(const double*, double*, const StepCoef<double>&, int,
                                              int, hipStream_t);

}  // namespace spfm
