// Temporal blocking of the SPFM step (FP32): TB forward-Euler steps of Eq. 2
// per pass over HBM.
//
// A 512-thread block owns a 64 x 8 column of the grid and marches it along z,
// like the single-step tiled kernel, but keeps TB time levels in flight.  Level
// l (time n + l) is computed on the footprint (64 + 2(TB-l)) x (8 + 2(TB-l)):
// each level needs one ring of cells around the next, so level 0 (read from
// HBM) carries a halo of TB cells and level TB is the 64 x 8 output tile.
// Every level lives in a four-plane LDS ring (with psi' for TI_n); the output
// level goes to HBM.  HBM sees one read and one write per point per TB steps;
// the price is the recomputed rings (the footprints are larger than the tile)
// and the 27 + 6 LDS reads per point update.
//
// Scheduling.  Level l numbers its planes j = 0, 1, ... from global plane
// z0 - (TB - l); level-l plane j needs level-(l-1) planes j, j+1, j+2.  At
// iteration i of the march the block stages level-0 plane i and computes
// level-l plane i - 3l for l = 1..TB.  A plane written at iteration i is read
// from iteration i + 1 on, and its ring slot is next overwritten at iteration
// i + 4, after its last reader (iteration i + 3): one barrier per iteration
// orders everything.
//
// Every point update is point_update, the same function the plain kernel
// evaluates, on the same neighbour values, so TB fused steps reproduce TB
// plain steps bit for bit.
#include <type_traits>

#include "spfm_impl.h"

namespace spfm {

namespace {

// Output tile of the temporally blocked kernel (one 512-thread block).
constexpr int kTTileX = 64, kTTileY = 8;

template <int TB>
struct TLevels {
    static constexpr int W(int l) { return kTTileX + 2 * (TB - l); }
    static constexpr int H(int l) { return kTTileY + 2 * (TB - l); }
    static constexpr int N(int l) { return W(l) * H(l); }
    // Start of level l's four-plane ring in the LDS arrays (levels 0..TB-1).
    static constexpr int ring(int l) {
        int o = 0;
        for (int i = 0; i < l; ++i) o += 4 * N(i);
        return o;
    }
    static constexpr int total = ring(TB);
    static constexpr int R0 = (N(0) + kTTileX * kTTileY - 1) / (kTTileX * kTTileY);   // staged cells per thread
};

__device__ __forceinline__ int wrap_mod(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

template <int TB, int S, int C>
__global__ __launch_bounds__(kTTileX* kTTileY) void k_step_temporal(const float* __restrict__ in,
                                                                   float* __restrict__ out,
                                                                   StepCoef<float> k, int ntx, int nty,
                                                                   int ntiles, int zlen) {
    using L = TLevels<TB>;
    constexpr int NT = kTTileX * kTTileY;
    constexpr int R0 = L::R0;
    __shared__ float sphi[L::total];
    __shared__ float spsi[C == kLocal ? L::total : 1];

    const int t = xcd_remap(blockIdx.x, ntiles);
    const int x0 = (t % ntx) * kTTileX, y0 = ((t / ntx) % nty) * kTTileY, z0 = (t / (ntx * nty)) * zlen;
    const int nx = k.nx, ny = k.ny, nz = k.nz;
    const size_t plane = (size_t)nx * ny;
    const int plane_bytes = (int)(plane * sizeof(float));   // < 2^31, checked at create
    const int tid = threadIdx.x;
    const int nout = min(zlen, nz - z0);
    const int n0 = nout + 2 * TB;          // level-0 planes
    const int last = nout - 1 + 3 * TB;    // iteration that writes the last output plane

    // Level-0 cells of this thread (wrapped in-plane byte offsets; footprints
    // wider than the grid wrap more than once).
    int loff[R0];
#pragma unroll
    for (int r = 0; r < R0; ++r) {
        const int c = tid + r * NT;
        const int gx = wrap_mod(x0 - TB + c % L::W(0), nx), gy = wrap_mod(y0 - TB + c / L::W(0), ny);
        loff[r] = c < L::N(0) ? (gy * nx + gx) * (int)sizeof(float) : 0;
    }
    auto fetch = [&](int j, float (&v)[R0]) {
        const __amdgpu_buffer_rsrc_t src =
            plane_rsrc(in + (size_t)wrap_mod(z0 - TB + j, nz) * plane, plane_bytes);
#pragma unroll
        for (int r = 0; r < R0; ++r) v[r] = buf_load(src, loff[r], (float*)nullptr);
    };
    auto stage = [&](int j, const float (&v)[R0]) {
        float* dphi = sphi + L::ring(0) + (j & 3) * L::N(0);
        float* dpsi = spsi + L::ring(0) + (j & 3) * L::N(0);
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int c = tid + r * NT;
            if (c < L::N(0)) {
                dphi[c] = v[r];
                if (C == kLocal) dpsi[c] = psi2(v[r], k.eps);
            }
        }
    };

    // Level l, plane j (of its own numbering) from level l-1 planes j, j+1, j+2.
    auto level = [&](auto lc, int j) {
        constexpr int l = decltype(lc)::value;
        constexpr int Wm = L::W(l - 1), Nm = L::N(l - 1);
        const float* P0 = sphi + L::ring(l - 1) + (j & 3) * Nm;
        const float* P1 = sphi + L::ring(l - 1) + ((j + 1) & 3) * Nm;
        const float* P2 = sphi + L::ring(l - 1) + ((j + 2) & 3) * Nm;
        const float* Q0 = spsi + L::ring(l - 1) + (j & 3) * Nm;
        const float* Q1 = spsi + L::ring(l - 1) + ((j + 1) & 3) * Nm;
        const float* Q2 = spsi + L::ring(l - 1) + ((j + 2) & 3) * Nm;
        for (int c = tid; c < L::N(l); c += NT) {
            const int cx = c % L::W(l), cy = c / L::W(l);
            const int b = (cy + 1) * Wm + (cx + 1);
            auto at = [&](int dx, int dy, int dz) -> float {
                const float* P = dz < 0 ? P0 : (dz > 0 ? P2 : P1);
                return P[b + dy * Wm + dx];
            };
            auto grad = [&](float& gx, float& gy, float& gz) {
                gx = Q1[b + 1] - Q1[b - 1];
                gy = Q1[b + Wm] - Q1[b - Wm];
                gz = Q2[b] - Q0[b];
            };
            const float v = point_update<float, S, C>(at, grad, k);
            if constexpr (l < TB) {
                sphi[L::ring(l) + (j & 3) * L::N(l) + c] = v;
                if (C == kLocal) spsi[L::ring(l) + (j & 3) * L::N(l) + c] = psi2(v, k.eps);
            } else {
                if (x0 + cx < nx && y0 + cy < ny) {
                    const __amdgpu_buffer_rsrc_t dst =
                        plane_rsrc(out + (size_t)(z0 + j) * plane, plane_bytes);
                    buf_store(v, dst, ((y0 + cy) * nx + (x0 + cx)) * (int)sizeof(float));
                }
            }
        }
    };
    auto level_at = [&](auto lc, int i) {
        constexpr int l = decltype(lc)::value;
        if constexpr (l <= TB) {
            const int j = i - 3 * l;
            if (j >= 0 && j < nout + 2 * (TB - l)) level(lc, j);
        }
    };
    auto levels = [&](int i) {
        static_assert(TB >= 2 && TB <= 4, "2 to 4 fused steps");
        level_at(std::integral_constant<int, 1>{}, i);
        level_at(std::integral_constant<int, 2>{}, i);
        level_at(std::integral_constant<int, 3>{}, i);
        level_at(std::integral_constant<int, 4>{}, i);
    };

    // Level-0 planes are fetched two iterations before they are staged; the two
    // register sets alternate, so the march is unrolled by two.
    float pa[R0], pb[R0];
    fetch(0, pa);
    if (1 < n0) fetch(1, pb);
    auto iter = [&](int i, float (&v)[R0]) {
        __syncthreads();
        if (i < n0) {
            stage(i, v);
            if (i + 2 < n0) fetch(i + 2, v);
        }
        levels(i);
    };
    for (int i = 0; i <= last; i += 2) {
        iter(i, pa);
        if (i + 1 <= last) iter(i + 1, pb);
    }
}

template <int TB, int S, int C>
hipError_t run_temporal(const float* in, float* out, const StepCoef<float>& k, int zlen, hipStream_t s) {
    const int ntx = (k.nx + kTTileX - 1) / kTTileX, nty = (k.ny + kTTileY - 1) / kTTileY;
    const int ntz = (k.nz + zlen - 1) / zlen;
    const int64_t n = (int64_t)ntx * nty * ntz;
    if (n > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_step_temporal<TB, S, C>), dim3((unsigned)n), dim3(kTTileX * kTTileY), 0, s, in,
                       out, k, ntx, nty, (int)n, zlen);
    return hipGetLastError();
}

template <int TB>
hipError_t dispatch_temporal(const float* in, float* out, const StepCoef<float>& k, int stencil,
                             int coupling, int zlen, hipStream_t s) {
#define SPFM_CASE(S_, C_) \
    if (stencil == S_ && coupling == C_) return run_temporal<TB, S_, C_>(in, out, k, zlen, s);
    SPFM_CASE(6, kLocal) SPFM_CASE(6, kGlobal) SPFM_CASE(6, kCF)
    SPFM_CASE(18, kLocal) SPFM_CASE(18, kGlobal) SPFM_CASE(18, kCF)
    SPFM_CASE(26, kLocal) SPFM_CASE(26, kGlobal) SPFM_CASE(26, kCF)
    SPFM_CASE(6, kCF5) SPFM_CASE(18, kCF5) SPFM_CASE(26, kCF5)
    SPFM_CASE(6, kCFAbel) SPFM_CASE(18, kCFAbel) SPFM_CASE(26, kCFAbel)
#undef SPFM_CASE
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_step_temporal(const float* in, float* out, const StepCoef<float>& k, int stencil,
                                int coupling, int tsteps, int zlen, hipStream_t s) {
    if (zlen < 1) return hipErrorInvalidValue;
    switch (tsteps) {
        case 2: return dispatch_temporal<2>(in, out, k, stencil, coupling, zlen, s);
        case 3: return dispatch_temporal<3>(in, out, k, stencil, coupling, zlen, s);
        case 4: return dispatch_temporal<4>(in, out, k, stencil, coupling, zlen, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace spfm
