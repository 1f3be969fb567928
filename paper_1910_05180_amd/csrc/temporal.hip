// Temporal blocking of the SPFM step (FP32): TB forward-Euler steps of Eq. 2
// per pass over HBM.
//
// A 512-thread block owns a 64 x 8 column of the grid and marches it along z,
// like the single-step tiled sweep, but keeps TB time levels in flight.  Level
// l (time n + l) is computed on the footprint (64 + 2(TB-l)) x (8 + 2(TB-l)):
// each level needs one ring of cells around the next, so level 0 (read from
// HBM) carries a halo of TB cells and level TB is the 64 x 8 output tile.
// Levels 0 .. TB-1 live in LDS (with psi' for TI_n); the output level goes to
// HBM.  HBM sees one read and one write per point per TB steps; the price is
// the recomputed rings (the footprints are larger than the tile).
//
// Columns.  Thread t owns cell t of every level's footprint and, where the
// footprint holds more than 512 cells, cell t + 512 as well, with the cells of
// a footprint numbered strip by strip (strips 16 columns wide, row by row
// inside a strip), so that a wave's 64 cells form a 16 x 4 patch, as in the
// single-step sweep: the full coupling is voted per wave, and compact patches
// take it less often than rows of 64 would.  For each owned
// column it keeps the per-plane sums (PlaneRegs) of the three level-(l-1)
// planes its next point needs, as the single-step sweep does, so a staged
// plane is read from LDS once per column, and the point update is
// point_from_planes, the single-step sweep's, on the same values: TB fused
// steps equal TB tiled steps bit for bit.
//
// Scheduling.  Level l numbers its planes j = 0, 1, ... from global plane
// z0 - (TB - l); level-l plane j is centred on level-(l-1) plane j + 1.  At
// iteration i of the march the block stages level-0 plane i, and level l
// (l = 1..TB) reads the sums of level-(l-1) plane i - 3l + 2, written at
// iteration i - 1, and computes its plane i - 3l.  Every plane is read only in
// the iteration after it is written, so two LDS slots per level suffice, and
// one barrier per iteration orders everything.  The register sets rotate with
// period 3 (plane number mod 3), so the march is unrolled by three.
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
    // LDS row stride of every level's plane: 80 = 16 mod 64 banks puts the four
    // rows of a wave's 16 x 4 patch in distinct banks.
    static constexpr int LS = 80;
    static_assert(W(0) <= LS, "footprint rows fit the LDS row stride");
    static constexpr int P(int l) { return LS * H(l); }
    // Start of level l's two-plane ring in the LDS arrays (levels 0..TB-1).
    static constexpr int ring(int l) {
        int o = 0;
        for (int i = 0; i < l; ++i) o += 2 * P(i);
        return o;
    }
    static constexpr int total = ring(TB);
    static constexpr int R0 = (N(0) + kTTileX * kTTileY - 1) / (kTTileX * kTTileY);   // staged cells per thread
};

// Waves per SIMD the fused kernels are compiled for: TI_n with three or four
// levels keeps too many plane sums in flight for four waves.
template <int TB, int C>
struct TWaves {
    static constexpr int value = (C == kLocal && TB >= 3) ? 2 : 4;
};

// Cell k of a W x H footprint in strip order: strips of 16 columns (the
// last one narrower when 16 does not divide W), row by row inside a strip.
template <int W, int H>
__device__ __forceinline__ void strip_cell(int k, int& cx, int& cy) {
    constexpr int SW = 16, FS = W / SW, SN = SW * H;
    const int s = k / SN, r = k - s * SN;
    if constexpr (W % SW == 0) {
        cx = s * SW + r % SW;
        cy = r / SW;
    } else {
        constexpr int WS = W - FS * SW;
        if (s < FS) {
            cx = s * SW + r % SW;
            cy = r / SW;
        } else {
            cx = FS * SW + r % WS;
            cy = r / WS;
        }
    }
}

__device__ __forceinline__ int wrap_mod(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

template <int TB, int S, int C>
__global__ __launch_bounds__(kTTileX* kTTileY, (TWaves<TB, C>::value)) void k_step_temporal(
    const float* __restrict__ in, float* __restrict__ out, StepCoef<float> k, int ntx, int nty,
    int ntiles, int zlen) {
    using L = TLevels<TB>;
    constexpr int NT = kTTileX * kTTileY;
    constexpr int R0 = L::R0;
    static_assert(L::N(TB) == NT && L::N(1) <= 2 * NT, "one or two columns per thread and level");
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

    // Level-0 cells of this thread, numbered row by row for coalesced loads:
    // wrapped in-plane byte offsets (footprints wider than the grid wrap more
    // than once) and LDS positions.
    int loff[R0], soff[R0];
#pragma unroll
    for (int r = 0; r < R0; ++r) {
        const int c = tid + r * NT;
        const int cx = c % L::W(0), cy = c / L::W(0);
        const int gx = wrap_mod(x0 - TB + cx, nx), gy = wrap_mod(y0 - TB + cy, ny);
        loff[r] = c < L::N(0) ? (gy * nx + gx) * (int)sizeof(float) : 0;
        soff[r] = cy * L::LS + cx;
    }
    auto fetch = [&](int j, float (&v)[R0]) {
        const __amdgpu_buffer_rsrc_t src =
            plane_rsrc(in + (size_t)wrap_mod(z0 - TB + j, nz) * plane, plane_bytes);
#pragma unroll
        for (int r = 0; r < R0; ++r) v[r] = buf_load(src, loff[r], (float*)nullptr);
    };
    auto stage = [&](int j, const float (&v)[R0]) {
        float* dphi = sphi + L::ring(0) + (j & 1) * L::P(0);
        float* dpsi = spsi + L::ring(0) + (j & 1) * L::P(0);
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int c = tid + r * NT;
            if (c < L::N(0)) {
                dphi[soff[r]] = v[r];
                if (C == kLocal) dpsi[soff[r]] = psi2(v[r], k.eps);
            }
        }
    };

    // Plane sums of the owned columns: R[l][col][plane mod 3] for level l's
    // points (sums of level-(l-1) planes).
    PlaneRegs<float> R[TB + 1][2][3];
    // Per owned column of level l: cb = the corner of its 3 x 3 neighbourhood
    // in the level-(l-1) plane; cw = its cell in the level-l plane (l < TB) or
    // the byte offset of the output point in its z-plane (-1 outside the grid).
    int cb[TB + 1][2], cw[TB + 1][2];
    auto columns = [&](auto lc) {
        constexpr int l = decltype(lc)::value;
        constexpr int Wl = L::W(l), Hl = L::H(l), Nl = L::N(l);
#pragma unroll
        for (int cc = 0; cc < (Nl + NT - 1) / NT; ++cc) {
            const int c = tid + cc * NT;
            int cx = 0, cy = 0;
            if (c < Nl) strip_cell<Wl, Hl>(c, cx, cy);
            cb[l][cc] = cy * L::LS + cx;
            if constexpr (l < TB)
                cw[l][cc] = cy * L::LS + cx;
            else
                cw[l][cc] = (x0 + cx < nx && y0 + cy < ny) ? ((y0 + cy) * nx + (x0 + cx)) * (int)sizeof(float) : -1;
        }
    };
    columns(std::integral_constant<int, 1>{});
    columns(std::integral_constant<int, 2>{});
    if constexpr (TB >= 3) columns(std::integral_constant<int, 3>{});
    if constexpr (TB >= 4) columns(std::integral_constant<int, 4>{});

    // Level l at iteration i (i mod 3 = PH): sums of the newest level-(l-1)
    // plane, then level-l plane i - 3l.
    auto level = [&](auto lc, auto phc, int i) {
        constexpr int l = decltype(lc)::value;
        constexpr int PH = decltype(phc)::value;
        constexpr int Pm = L::P(l - 1), Nl = L::N(l);
        constexpr int NCOL = (Nl + NT - 1) / NT;
        const int pn = i - 3 * l + 2;
        const int j = i - 3 * l;
        if (pn >= 0 && pn < nout + 2 * (TB - l + 1)) {
            const float* P = sphi + L::ring(l - 1) + (pn & 1) * Pm;
            const float* Q = spsi + L::ring(l - 1) + (pn & 1) * Pm;
#pragma unroll
            for (int cc = 0; cc < NCOL; ++cc) {
                const int c = tid + cc * NT;
                if (cc == 0 || c < Nl)
                    plane_sums<float, S, C, L::LS>(P + cb[l][cc], Q + cb[l][cc], R[l][cc][(PH + 2) % 3]);
            }
        }
        if (j >= 0 && j < nout + 2 * (TB - l)) {
#pragma unroll
            for (int cc = 0; cc < NCOL; ++cc) {
                const int c = tid + cc * NT;
                if (cc == 0 || c < Nl) {
                    const float v = point_from_planes<float, S, C>(R[l][cc][PH], R[l][cc][(PH + 1) % 3],
                                                                   R[l][cc][(PH + 2) % 3], k);
                    if constexpr (l < TB) {
                        sphi[L::ring(l) + (j & 1) * L::P(l) + cw[l][cc]] = v;
                        if (C == kLocal) spsi[L::ring(l) + (j & 1) * L::P(l) + cw[l][cc]] = psi2(v, k.eps);
                    } else if (cw[l][cc] >= 0) {
                        const __amdgpu_buffer_rsrc_t dst =
                            plane_rsrc(out + (size_t)(z0 + j) * plane, plane_bytes);
                        buf_store(v, dst, cw[l][cc]);
                    }
                }
            }
        }
    };

    // Level-0 planes are fetched two iterations before they are staged, into
    // three register sets that rotate with the iteration number.
    float pf[3][R0];
    fetch(0, pf[0]);
    if (1 < n0) fetch(1, pf[1]);
    auto iter = [&](auto phc, int i) {
        constexpr int PH = decltype(phc)::value;
        static_assert(TB >= 2 && TB <= 4, "2 to 4 fused steps");
        __syncthreads();
        if (i < n0) {
            stage(i, pf[PH]);
            if (i + 2 < n0) fetch(i + 2, pf[(PH + 2) % 3]);
        }
        level(std::integral_constant<int, 1>{}, phc, i);
        level(std::integral_constant<int, 2>{}, phc, i);
        if constexpr (TB >= 3) level(std::integral_constant<int, 3>{}, phc, i);
        if constexpr (TB >= 4) level(std::integral_constant<int, 4>{}, phc, i);
    };
    using P0 = std::integral_constant<int, 0>;
    using P1 = std::integral_constant<int, 1>;
    using P2 = std::integral_constant<int, 2>;
    for (int i = 0; i <= last; i += 3) {
        iter(P0{}, i);
        if (i + 1 > last) break;
        iter(P1{}, i + 1);
        if (i + 2 > last) break;
        iter(P2{}, i + 2);
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
