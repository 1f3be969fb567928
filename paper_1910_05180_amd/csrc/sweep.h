// Tiled sweep of the single-step kernels (forward Euler of Eq. 2; periodic
// grid, or contact-angle walls on chosen axes), shared by the per-coupling
// translation units that instantiate it for every compiled tile shape.
//
//  k_step_tiled   a block owns a TX x TY tile column of the grid (one wave per
//                 16 x 4 patch) and marches it along z over the work items of a
//                 schedule (see tile_sweep): every plane is read from HBM once
//                 with coalesced rows, ahead of its use, staged with its halo in
//                 LDS, and reduced by each thread to a few per-plane partial sums
//                 kept in registers.  For TI_n the log-ratio psi' of every staged
//                 cell is computed once.  On walled grids the ghost values are
//                 computed as planes are staged.
//  k_step_batched the same sweep over a flat list of (grid, tile) items that
//                 covers many independent grids in one launch.
// The result of a point does not depend on the tile shape or on the z-chunk:
// every shape evaluates the same per-plane sums and point update.
#pragma once

#include <type_traits>

#include "spfm_impl.h"

namespace spfm {

__device__ __forceinline__ int wrap_once(int i, int n) {
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

// One block sweeps the tile [x0, x0+TX) x [y0, y0+TY) x [z0, z0+zlen)
// (clipped to the grid).  Each plane of the tile plus a one-cell halo is read
// from global memory once (coalesced rows) two iterations before it is staged
// into a four-slot LDS ring, together with psi' of every cell for TI_n.  Every
// thread reads its 3x3 in-plane neighbourhood of each plane once and keeps
// per-plane sums in registers (its value c, the sum F of its 4 face neighbours
// and the sum D of its 4 diagonal neighbours); with them the shell sums of
// second differences of point z are
//   s1 = F(z) + c(z-1) + c(z+1) - 6c(z),  s2 = D(z) + F(z-1) + F(z+1) - 12c(z),
//   s3 = D(z-1) + D(z+1) - 8c(z).  Two output planes are produced
// per iteration (one barrier per two planes, two independent points per thread).
// Planes are numbered relative to the sweep, r = 0 for z0 - 1; plane r lives in
// LDS slot r & 3.  Iterations start at r = 1 (mod 4) and alternate parity, so the
// slots each iteration touches are compile-time constants.
//
// W: the stored grid has contact-angle walls (w in device memory).  A halo cell
// on a ghost layer is then read from its interior neighbour and mapped by Eq. 7
// with the composed coefficient of its ghost class as it is staged; ghost planes
// of a walled z axis are read from their interior neighbour planes.  Points on
// ghost layers are computed too, and their values are never read.
//
// V (periodic grids): the block also sums phi* - phi and h'(phi) over its output
// points exactly (CvAcc) and stores the sums to cvp, for the constant-volume
// correction that follows the step.
// F (with V): `in` is the previous step's uncorrected phi*, and the block first
// applies that step's correction as it reads: it adds the previous step's sums
// (fz.part, the same integers in every block, so the same g) and stages
// phi* - g h'(phi_prev) with phi_prev from fz.old, exactly as the separate
// correction pass computes it; the corrected value of each output point, the
// step's input, is also written to fz.corr.
template <typename T, int S, int C, bool W, bool V, int TX, int TY, bool F = false>
__device__ __forceinline__ void tile_sweep(const T* __restrict__ in, T* __restrict__ out,
                                           const StepCoef<T>& k, int x0, int y0, int z0, int zlen,
                                           T* __restrict__ sphi, T* __restrict__ spsi,
                                           const WallCoef<T>* __restrict__ w,
                                           unsigned long long* __restrict__ cvp,
                                           const CvFuse<T>& fz = CvFuse<T>{}) {
    static_assert(!(V && W), "constant volume needs a periodic grid");
    static_assert(!F || V, "the fused correction comes with the constant-volume sums");
    // Halo plane: HY rows of HX cells, stored in LDS with row stride LX.  Each
    // wave computes a kWaveX x (64 / kWaveX) patch of the tile.
    constexpr int HX = TX + 2, HY = TY + 2, NC = HX * HY;
    constexpr int LX = lds_row(TX), HP = LX * HY;
    constexpr int NT = TX * TY;
    constexpr int WX = kWaveX, WY = 64 / kWaveX;
    static_assert(NT <= NC && NC <= 2 * NT, "the halo plane takes two load rounds");
    static_assert(TX % WX == 0 && TY % WY == 0 && LX >= HX, "wave patches tile the block");
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int tx = (wave % (TX / WX)) * WX + lane % WX;
    const int ty = (wave / (TX / WX)) * WY + lane / WX;
    const int nx = k.nx, ny = k.ny, nz = k.nz;
    const size_t plane = (size_t)nx * ny;
    const int plane_bytes = (int)(plane * sizeof(T));   // < 2^31, checked at create

    // In-plane byte offsets (fixed along the sweep) and LDS positions of this
    // thread's two halo cells; cells are numbered row by row so that loads are
    // coalesced.  The first always exists, the second only for tid + NT < NC.
    // Periodic wrap of a halo coordinate v in [-1, n + H - 2] (H = halo extent):
    // one conditional add or subtract when n >= H (the grid-wide, uniform
    // common case), a modulo for grids narrower than a tile.
    auto wrap = [](int v, int n, int H) {
        if (n >= H) {
            v = v < 0 ? v + n : v;
            return v >= n ? v - n : v;
        }
        v %= n;
        return v < 0 ? v + n : v;
    };
    // Walls: a ghost cell is read from its interior neighbour, and wa*[c] is the
    // Eq. 7 coefficient of its class on a plane of z class c - 1 (0 inside).
    const int walls = W ? w->walls : 0;
    T wa0[3] = {T(0), T(0), T(0)}, wa1[3] = {T(0), T(0), T(0)};
    auto mirror = [&](int& gx, int& gy, T (&a)[3]) {
        const int cx = (walls & 1) ? (gx == 0 ? -1 : (gx == nx - 1 ? 1 : 0)) : 0;
        const int cy = (walls & 2) ? (gy == 0 ? -1 : (gy == ny - 1 ? 1 : 0)) : 0;
        gx -= cx;
        gy -= cy;
        const int base = (cx + 1) + 3 * (cy + 1);
        a[0] = w->a[base];
        a[1] = w->a[base + 9];
        a[2] = w->a[base + 18];
    };
    int loff0, loff1, soff0, soff1;
    {
        int gx = wrap(x0 - 1 + tid % HX, nx, HX), gy = wrap(y0 - 1 + tid / HX, ny, HY);
        if (W) mirror(gx, gy, wa0);
        soff0 = (tid / HX) * LX + tid % HX;
        loff0 = (gy * nx + gx) * (int)sizeof(T);
        const int c1 = tid + NT;
        soff1 = (c1 / HX) * LX + c1 % HX;
        int hx = wrap(x0 - 1 + c1 % HX, nx, HX), hy = wrap(y0 - 1 + c1 / HX, ny, HY);
        if (W) mirror(hx, hy, wa1);
        loff1 = c1 < NC ? (hy * nx + hx) * (int)sizeof(T) : 0;
    }
    const bool has1 = tid + NT < NC;
    const int nout = min(zlen, nz - z0);   // output planes z0 .. z0+nout-1
    const int last = nout + 1;             // relative index of the last plane needed

    // Two fetched halo cells, with (W) the Eq. 7 coefficients of their classes
    // on the fetched plane, or (F) the previous step's values of the cells.
    struct Pair { T v0, v1, a0, a1; };
    __amdgpu_buffer_rsrc_t fetch_old = plane_rsrc(in, plane_bytes);   // F: fz.old, same plane
    auto fetch_at = [&](__amdgpu_buffer_rsrc_t src, int zc, Pair& v) {
        v.v0 = buf_load(src, loff0, (T*)nullptr);
        v.v1 = buf_load(src, loff1, (T*)nullptr);   // loff1 = 0 where the cell does not exist
        if (F) {
            v.a0 = buf_load(fetch_old, loff0, (T*)nullptr);
            v.a1 = buf_load(fetch_old, loff1, (T*)nullptr);
        }
        if (W) {
            v.a0 = zc == 0 ? wa0[0] : (zc == 2 ? wa0[2] : wa0[1]);
            v.a1 = zc == 0 ? wa1[0] : (zc == 2 ? wa1[2] : wa1[1]);
        }
    };
    // F: the correction g of the previous step, set before the first staging.
    double g = 0.0;
    auto correct = [&](T star, T prev) {
        return (T)((double)star - g * h_slope(kernel_interp(C), (double)prev));
    };
    auto stage_slot = [&](int slot, const Pair& v) {
        T* dphi = sphi + slot * HP;
        T* dpsi = spsi + slot * HP;
        const T u0 = W ? wall_map(v.v0, v.a0) : (F ? correct(v.v0, v.a0) : v.v0);
        dphi[soff0] = u0;
        if (C == kLocal) dpsi[soff0] = psi2(u0, k.eps);
        if (has1) {
            const T u1 = W ? wall_map(v.v1, v.a1) : (F ? correct(v.v1, v.a1) : v.v1);
            dphi[soff1] = u1;
            if (C == kLocal) dpsi[soff1] = psi2(u1, k.eps);
        }
    };
    // The 3 x 3 neighbourhood of this thread's point, from the corner cell b.
    const int b = ty * LX + tx;
    auto load_slot = [&](int slot, PlaneRegs<T>& R) {
        plane_sums<T, S, C, LX>(sphi + slot * HP + b, spsi + slot * HP + b, R);
    };
    const bool active = (x0 + tx < nx) && (y0 + ty < ny);
    const int dst_off = ((y0 + ty) * nx + (x0 + tx)) * (int)sizeof(T);
    CvAcc cv{{0, 0}};
    __amdgpu_buffer_rsrc_t out_corr = plane_rsrc(out, plane_bytes);   // F: fz.corr, same plane
    auto point = [&](__amdgpu_buffer_rsrc_t dst, const PlaneRegs<T>& Rm, const PlaneRegs<T>& R0,
                     const PlaneRegs<T>& Rp) {
        const T v = point_from_planes<T, S, C>(Rm, R0, Rp, k);
        if (active) buf_store<(C == kLocal && sizeof(T) == 4) ? kStoreThrough : 0>(v, dst, dst_off);
        if (F && active) buf_store(R0.c, out_corr, dst_off);
        if (V && active) {
            const double c = (double)R0.c;
            cv.add((double)v - c, h_slope(kernel_interp(C), c));
        }
    };
    // Descriptors of the input planes, fetched strictly in order r = 0, 1, ...
    // (plane z0 - 1 + r with periodic wrap), and of the output planes, written
    // in order z0, z0 + 1, ...: running byte pointers advanced one plane per use.
    // With a walled z axis the ghost planes 0 and nz - 1 are read from planes 1
    // and nz - 2 (z class zc = 0 and 2; 1 elsewhere).
    int fetch_z = wrap_once(z0 - 1, nz);
    const char* fetch_ptr = reinterpret_cast<const char*>(in) + (size_t)fetch_z * plane_bytes;
    auto next_in = [&](int& zc) {
        const char* ptr = fetch_ptr;
        zc = 1;
        if (W && (walls & 4)) {
            if (fetch_z == 0) { ptr += plane_bytes; zc = 0; }
            else if (fetch_z == nz - 1) { ptr -= plane_bytes; zc = 2; }
        }
        const __amdgpu_buffer_rsrc_t rs = plane_rsrc(ptr, plane_bytes);
        if (F)   // no walls here: the previous field's plane is the same plane
            fetch_old = plane_rsrc(reinterpret_cast<const char*>(fz.old) +
                                       (ptr - reinterpret_cast<const char*>(in)), plane_bytes);
        fetch_ptr += plane_bytes;
        if (++fetch_z == nz) {
            fetch_z = 0;
            fetch_ptr = reinterpret_cast<const char*>(in);
        }
        return rs;
    };
    char* out_ptr = reinterpret_cast<char*>(out) + (size_t)z0 * plane_bytes;
    auto next_out = [&]() {
        const __amdgpu_buffer_rsrc_t rs = plane_rsrc(out_ptr, plane_bytes);
        if (F)
            out_corr = plane_rsrc(reinterpret_cast<char*>(fz.corr) +
                                      (out_ptr - reinterpret_cast<char*>(out)), plane_bytes);
        out_ptr += plane_bytes;
        return rs;
    };

    // Iteration producing planes r, r+1 (slots: parity 0 reads 2, 3 and
    // writes 0, 1; parity 1 reads 0, 1 and writes 2, 3) with registers P0..P3
    // holding planes r-1 .. r+2 (P0, P1 already filled).  Planes r+3, r+4,
    // requested two iterations earlier into the set Q, are staged into the
    // slots of planes r-1, r (last read an iteration ago), and planes r+7, r+8
    // are requested into Q.  GUARD: near the end of the sweep, skip planes
    // beyond it (steady iterations need no checks).
    auto iter = [&](auto par, auto guard, int r, PlaneRegs<T>& P0, PlaneRegs<T>& P1,
                    PlaneRegs<T>& P2, PlaneRegs<T>& P3, Pair& Q0, Pair& Q1) {
        constexpr int rd = decltype(par)::value ? 0 : 2;
        constexpr int wr = decltype(par)::value ? 2 : 0;
        constexpr bool G = decltype(guard)::value;
        __syncthreads();
        if (!G || r + 1 <= last) load_slot(rd, P2);
        if (!G || r + 2 <= last) load_slot(rd + 1, P3);
        if (!G || r + 3 <= last) stage_slot(wr, Q0);
        if (!G || r + 4 <= last) stage_slot(wr + 1, Q1);
        int zc;
        if (!G || r + 7 <= last) { const auto rs = next_in(zc); fetch_at(rs, zc, Q0); }
        if (!G || r + 8 <= last) { const auto rs = next_in(zc); fetch_at(rs, zc, Q1); }
        if (!G || r <= nout) point(next_out(), P0, P1, P2);
        if (!G || r + 1 <= nout) point(next_out(), P1, P2, P3);
    };
    using P0t = std::integral_constant<int, 0>;
    using P1t = std::integral_constant<int, 1>;
    using Steady = std::false_type;
    using Guarded = std::true_type;

    PlaneRegs<T> A{}, B{}, D{}, E{};
    Pair qa0{}, qa1{}, qb0{}, qb1{};
    {
        // All prologue loads in flight at once: planes 0..3 are staged now,
        // 4, 5 and 6, 7 are staged by the first two iterations.
        Pair v[4];
        int zc;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (r <= last) { const auto rs = next_in(zc); fetch_at(rs, zc, v[r]); }
        if (4 <= last) { const auto rs = next_in(zc); fetch_at(rs, zc, qa0); }
        if (5 <= last) { const auto rs = next_in(zc); fetch_at(rs, zc, qa1); }
        if (6 <= last) { const auto rs = next_in(zc); fetch_at(rs, zc, qb0); }
        if (7 <= last) { const auto rs = next_in(zc); fetch_at(rs, zc, qb1); }
        if constexpr (F) {
            // g of the previous step while the planes are in flight: the sum
            // of its work items' sums, as the separate correction pass forms it
            __shared__ unsigned long long ftot[4];
            CvAcc a{{0, 0}};
            for (int i = tid; i < fz.nparts; i += NT) a.add_words(fz.part + 4 * (size_t)i);
            cv_block_store<NT>(a, ftot);
            __syncthreads();
            CvAcc t{{0, 0}};
            t.add_words(ftot);
            const double den = CvAcc::value(t.s[1]);
            g = den != 0.0 ? CvAcc::value(t.s[0]) / den : 0.0;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (r <= last) stage_slot(r, v[r]);
        __syncthreads();
        load_slot(0, A);
        load_slot(1, B);
    }
    // Unrolled by two so that the plane registers rotate without moves.  The
    // steady loop runs while every plane an iteration pair touches lies strictly
    // inside the sweep (no wrap, no checks).
    int r = 1;
    for (; r + 10 <= nout; r += 4) {
        iter(P0t{}, Steady{}, r, A, B, D, E, qa0, qa1);
        iter(P1t{}, Steady{}, r + 2, D, E, A, B, qb0, qb1);
    }
    for (; r <= nout; r += 4) {
        iter(P0t{}, Guarded{}, r, A, B, D, E, qa0, qa1);
        if (r + 2 > nout) break;
        iter(P1t{}, Guarded{}, r + 2, D, E, A, B, qb0, qb1);
    }
    if constexpr (V) cv_block_store<NT>(cv, cvp);
}

template <int TX, int TY>
struct Smem {
    static constexpr int NT = TX * TY;                        // threads per block
    static constexpr int HP = lds_row(TX) * (TY + 2);         // one staged plane
};

#ifndef SPFM_WAVES_F32
#define SPFM_WAVES_F32 7
#endif
// Waves per SIMD the tiled kernels are compiled for: FP32 TI_n on 16-wide
// tiles is held to 5 by its LDS (two staged arrays of row stride 48), the
// wider tiles need a few more registers than 7 waves allow (they spill at 72)
// and are compiled for 6; the FP32 couplings without psi' staging take 7; FP64
// TI_n needs more than twice as many registers (2 waves, no spills).  The
// walled variants (small grids, never many waves) are compiled for fewer waves,
// which keeps them free of spills.
// The constant-volume variants carry two 128-bit sums per thread (4 waves FP32).
template <typename T, int C = kLocal, int TX = 16>
struct WavesPerSimd {
    static constexpr int value = sizeof(T) == 4 ? (C == kLocal ? (TX == 16 ? 5 : 6) : SPFM_WAVES_F32) : 2;
    static constexpr int walled = sizeof(T) == 4 ? 4 : 2;
};
template <typename T, int C, bool W, bool V, int TX>
constexpr int waves_per_simd() {
    return W || V ? WavesPerSimd<T>::walled : WavesPerSimd<T, C, TX>::value;
}

// One block per work item of a tile schedule (see the host-side schedule
// builder): the item gives the tile column origin and its z-chunk; items with
// zlen = 0 pad the table and exit at once (with V, after storing zero sums).
// W: walled grid, coefficients at w.  V: constant-volume sums of item i to
// cvp + 4i.  F: the previous step's correction applied on reading (fz).
template <typename T, int S, int C, bool W, bool V, int TX, int TY, bool F = false>
__global__ __launch_bounds__((Smem<TX, TY>::NT), (waves_per_simd<T, C, W, V, TX>())) void k_step_tiled(
    const T* __restrict__ in, T* __restrict__ out, StepCoef<T> k, const TileItem* __restrict__ items,
    const WallCoef<T>* __restrict__ w, unsigned long long* __restrict__ cvp, CvFuse<T> fz) {
    __shared__ T sphi[4 * Smem<TX, TY>::HP];
    __shared__ T spsi[C == kLocal ? 4 * Smem<TX, TY>::HP : 1];
    const TileItem it = items[blockIdx.x];
    unsigned long long* const cvi = V ? cvp + 4 * (size_t)blockIdx.x : nullptr;
    if (it.zlen <= 0) {
        if (V && threadIdx.x < 4) cvi[threadIdx.x] = 0;
        return;
    }
    tile_sweep<T, S, C, W, V, TX, TY, F>(in, out, k, it.x0, it.y0, it.z0, it.zlen, sphi, spsi, w, cvi, fz);
}

template <int S, int C, bool W, int TX, int TY>
__global__ __launch_bounds__((Smem<TX, TY>::NT), (W ? WavesPerSimd<float>::walled : WavesPerSimd<float, C, TX>::value)) void k_step_batched(
    const float* __restrict__ buf_in, float* __restrict__ buf_out,
    const StepCoef<float>* __restrict__ coef, const int64_t* __restrict__ offset,
    const TileItem* __restrict__ items, const WallCoef<float>* __restrict__ wall) {
    __shared__ float sphi[4 * Smem<TX, TY>::HP];
    __shared__ float spsi[C == kLocal ? 4 * Smem<TX, TY>::HP : 1];
    const TileItem it = items[blockIdx.x];
    if (it.zlen <= 0) return;   // padding of the schedule
    const StepCoef<float> k = coef[it.inst];
    const int64_t off = offset[it.inst];
    tile_sweep<float, S, C, W, false, TX, TY>(buf_in + off, buf_out + off, k, it.x0, it.y0, it.z0,
                                              it.zlen, sphi, spsi, W ? wall + it.inst : nullptr, nullptr);
}


// Calls f(S, W, shape) with compile-time constants for the runtime stencil,
// walls flag and tile shape (nothing for values outside the compiled sets).
template <typename F>
void for_each_variant(int stencil, bool walled, int tile, F&& f) {
    auto by_tile = [&](auto S_, auto W_) {
        switch (tile) {
            case kTile16x8: f(S_, W_, std::integral_constant<int, kTile16x8>{}); break;
            case kTile32x8: f(S_, W_, std::integral_constant<int, kTile32x8>{}); break;
            case kTile64x8: f(S_, W_, std::integral_constant<int, kTile64x8>{}); break;
            case kTile16x16: f(S_, W_, std::integral_constant<int, kTile16x16>{}); break;
            case kTile32x16: f(S_, W_, std::integral_constant<int, kTile32x16>{}); break;
            case kTile64x16: f(S_, W_, std::integral_constant<int, kTile64x16>{}); break;
            default: break;
        }
    };
    auto by_walls = [&](auto S_) {
        if (walled) by_tile(S_, std::true_type{});
        else by_tile(S_, std::false_type{});
    };
    if (stencil == 6) by_walls(std::integral_constant<int, 6>{});
    else if (stencil == 18) by_walls(std::integral_constant<int, 18>{});
    else if (stencil == 26) by_walls(std::integral_constant<int, 26>{});
}

template <typename T, int S, int C, bool W, bool V, int TX, int TY, bool F = false>
hipError_t run_tiled(const T* in, T* out, const StepCoef<T>& k, const TileItem* items, int nitems,
                     const WallCoef<T>* wall, unsigned long long* cvp, hipStream_t s,
                     const CvFuse<T>& fz = CvFuse<T>{}) {
    hipLaunchKernelGGL((k_step_tiled<T, S, C, W, V, TX, TY, F>), dim3((unsigned)nitems), dim3(TX * TY), 0,
                       s, in, out, k, items, wall, cvp, fz);
    return hipGetLastError();
}

template <int S, int C, bool W, int TX, int TY>
hipError_t run_batched(const float* in, float* out, const StepCoef<float>* coef, const int64_t* offset,
                       const TileItem* items, int nitems, const WallCoef<float>* wall, hipStream_t s) {
    hipLaunchKernelGGL((k_step_batched<S, C, W, TX, TY>), dim3((unsigned)nitems), dim3(TX * TY), 0, s,
                       in, out, coef, offset, items, wall);
    return hipGetLastError();
}

// The tiled step of one kernel coupling C for the compiled tile shape `tile`
// (hipErrorInvalidValue for a shape not compiled for this variant).  With cvp
// (periodic grids, the untuned shape only) the constant-volume variant, with
// fuse also the correction of the previous step.
template <typename T, int C>
hipError_t launch_tiled_coupling(const T* in, T* out, const StepCoef<T>& k, int stencil, int tile,
                                 const TileItem* items, int nitems, const WallCoef<T>* wall,
                                 unsigned long long* cvp, const CvFuse<T>* fuse, hipStream_t s) {
    if (nitems <= 0) return hipErrorInvalidValue;
    if (fuse && (!cvp || fuse->nparts < 0 || fuse->nparts > kCvDirectParts)) return hipErrorInvalidValue;
    constexpr bool f32 = sizeof(T) == 4;
    hipError_t e = hipErrorInvalidValue;
    auto one = [&](auto S_, auto W_, auto T_) {
        constexpr int S = decltype(S_)::value, t = decltype(T_)::value;
        constexpr bool W = decltype(W_)::value;
        if constexpr (!W && t == default_tile(f32, C)) {
            if (cvp && fuse) {
                e = run_tiled<T, S, C, false, true, tile_tx(t), tile_ty(t), true>(in, out, k, items, nitems,
                                                                                   nullptr, cvp, s, *fuse);
                return;
            }
            if (cvp) {
                e = run_tiled<T, S, C, false, true, tile_tx(t), tile_ty(t)>(in, out, k, items, nitems,
                                                                             nullptr, cvp, s);
                return;
            }
        }
        if constexpr (tile_compiled(f32, C, W, t))
            if (!cvp)
                e = run_tiled<T, S, C, W, false, tile_tx(t), tile_ty(t)>(in, out, k, items, nitems, wall,
                                                                          nullptr, s);
    };
    for_each_variant(stencil, wall != nullptr, tile, one);
    return e;
}

template <int C>
hipError_t launch_batched_coupling(const float* in, float* out, const StepCoef<float>* coef,
                                   const int64_t* offset, int stencil, int tile, const TileItem* items,
                                   int nitems, const WallCoef<float>* wall, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipError_t e = hipErrorInvalidValue;
    auto one = [&](auto S_, auto W_, auto T_) {
        constexpr int S = decltype(S_)::value, t = decltype(T_)::value;
        constexpr bool W = decltype(W_)::value;
        if constexpr (tile_compiled(true, C, W, t))
            e = run_batched<S, C, W, tile_tx(t), tile_ty(t)>(in, out, coef, offset, items, nitems, wall, s);
    };
    for_each_variant(stencil, wall != nullptr, tile, one);
    return e;
}

}  // namespace spfm
