// Resident step for small grids (forward Euler of Eq. 2, periodic or with the
// contact-angle walls of Eq. 7): one block per grid holds the whole stored
// grid in LDS, twice (phi^n and phi^{n+1}), and takes many steps in one launch
// with block barriers only; HBM is touched once at the start and once at the
// end.  Grids of the orientation study (120 x 10 x 10 between walls) and of the
// 1D model comparison (256 x 3 x 3 slabs) are small enough, and their steps are
// otherwise bound by the latency of one launch per step.
//
// Every point is computed by the same per-plane sums and point update as the
// tiled sweep (point_from_planes), on the same neighbour values: the result of
// n resident steps equals n tiled steps bit for bit.
//  * The block's threads own columns of the grid's interior, each cut into
//    z-segments so that the columns and segments spread evenly over the
//    threads; a thread marches its segment along z keeping the per-plane sums
//    of three planes in registers, as the tiled sweep does.
//  * TI_n: psi' of every cell is refreshed once per step into a third LDS
//    array when the region's three copies fit (13653 FP32 or 6826 FP64
//    points), else each point evaluates it for the cells it needs (the column
//    cell and four in-plane face neighbours of each plane).
//  * Regions of at most two cells per thread and one work item per thread keep
//    their ghost and column indices in registers across the steps.
//  * Walls: before each step the ghost cells of the current copy are set from
//    their interior neighbours by Eq. 7 with the coefficient of their class.
//  * The output may be the input buffer (an even number of steps): a block reads
//    its whole grid before its first step and writes it after its last.
//  * Segments: a grid too large for one CU's VALU to step quickly is cut along x
//    into segments, one block each.  A block holds its segment plus a halo of h
//    columns on each open side (the grid's own walls need none) and takes at most
//    h steps: the values it has not updated, or updated from stale neighbours,
//    advance one column per step from the open sides, so after h steps its
//    segment is still exact.  The block writes back only its segment, to the
//    other buffer (every block reads its halo from the input).  Each step does
//    the same work on the same values as the tiled step, so the results are
//    the same bit for bit; the halos are computed twice, which buys many blocks
//    per grid and no synchronisation between them.
#include <atomic>

#include "spfm_impl.h"

namespace spfm {

namespace {

constexpr int kResThreads = 1024;

__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Per-plane sums of the column (x, y) on plane z of the field F (row stride sx,
// plane stride pl), with the same association as plane_sums on a staged tile:
// xm, xp, ym, yp are the wrapped (or, next to a wall, ghost) neighbour indices.
// PS: psi' of every cell is staged in Ps (same layout); else it is evaluated
// here for the cells that need it.
template <typename T, int S, int C, bool PS>
__device__ __forceinline__ void column_plane(const T* __restrict__ F, const T* __restrict__ Ps, int pl,
                                             int sx, int z, int x, int xm, int xp, int y, int ym, int yp,
                                             bool with_grad, T eps, PlaneRegs<T>& R) {
    const int q = z * pl, o0 = q + y * sx, om = q + ym * sx, op = q + yp * sx;
    const T e = F[o0 + xp], w = F[o0 + xm], n = F[op + x], s = F[om + x];
    R.c = F[o0 + x];
    R.fc = (e + w) + (n + s);
    if (S >= 18) R.dc = (F[op + xp] + F[om + xm]) + (F[op + xm] + F[om + xp]);
    if (C == kLocal) {
        if (PS) {
            R.pc = Ps[o0 + x];
            if (with_grad) {
                R.gx = Ps[o0 + xp] - Ps[o0 + xm];
                R.gy = Ps[op + x] - Ps[om + x];
            }
        } else {
            R.pc = psi2(R.c, eps);
            if (with_grad) {
                R.gx = psi2(e, eps) - psi2(w, eps);
                R.gy = psi2(n, eps) - psi2(s, eps);
            }
        }
    }
}

// PS (TI_n): a third LDS array holds psi' of every cell of the current copy,
// refreshed once per step, instead of each point evaluating it for its column
// and four in-plane neighbours on three planes.
template <typename T, int S, int C, bool W, bool PS>
__global__ __launch_bounds__(kResThreads, 1) void k_step_resident(
    const T* buf_in, T* buf_out, const StepCoef<T>* __restrict__ coef,
    const int64_t* __restrict__ offset, const WallCoef<T>* __restrict__ wall,
    const ResItem* __restrict__ items, int nsteps) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T* lds = reinterpret_cast<T*>(lds_raw);
    const int tid = threadIdx.x;
    const int g = items ? items[blockIdx.x].inst : (int)blockIdx.x;
    const StepCoef<T> k = coef[g];
    const int sx = k.nx, sy = k.ny, sz = k.nz;
    // The region this block holds: stored x in [rx0, rx0 + rw) (mod sx on a
    // periodic x axis), all y and z; it writes back x in [ox, ox + olen).
    const ResItem it = items ? items[blockIdx.x] : ResItem{g, 0, sx, 0, sx};
    const int rw = it.rw, rx0 = it.rx0;
    const bool whole = rw == sx && rx0 == 0;
    const int pl = rw * sy, cells = pl * sz;
    T* A = lds;
    T* B = lds + cells;
    T* P = lds + 2 * cells;   // PS only
    const T* in = buf_in + offset[g];
    T* out = buf_out + offset[g];
    for (int i = tid; i < cells; i += kResThreads) {
        const int lx = i % rw, row = i / rw;   // row = z sy + y
        A[i] = in[(size_t)row * sx + wrap1(rx0 + lx, sx)];
    }
    __syncthreads();   // the ghost fill reads cells that other threads loaded

    const int walls = W ? wall[g].walls : 0;
    const int wx = walls & 1, wy = (walls >> 1) & 1, wz = (walls >> 2) & 1;
    // Columns computed: the interior of a whole grid (x wraps when periodic);
    // in a segment every column with both x neighbours in the region.  The
    // outermost columns of an open side are never updated, so after n steps the
    // n columns next to it are stale: the host gives each side a halo of at
    // least nsteps columns beyond the segment written back.
    const int xa = whole ? wx : 1, xb = whole ? sx - wx : rw - 1;
    const int nxi = xb - xa, nyi = sy - 2 * wy, nzi = sz - 2 * wz;
    const int ncol = nxi * nyi;
    // z-segments per column: the count that minimises the planes a thread
    // touches, (points + 2 planes of each segment's halo) x segments per thread.
    int nseg = 1;
    {
        int best = 1 << 30;
        for (int q = 1; q <= nzi; ++q) {
            const int per = (ncol * q + kResThreads - 1) / kResThreads;
            const int cost = per * ((nzi + q - 1) / q + 2);
            if (cost < best) { best = cost; nseg = q; }
        }
    }
    const int items_n = ncol * nseg;

    // Work item t: column and z range, neighbour indices.
    struct Item {
        int x, xm, xp, y, ym, yp, za, zb;
    };
    auto item = [&](int t) {
        const int col = t % ncol, seg = t / ncol;
        Item m;
        m.x = xa + col % nxi;
        m.y = wy + col / nxi;
        m.xm = whole ? wrap1(m.x - 1, sx) : m.x - 1;
        m.xp = whole ? wrap1(m.x + 1, sx) : m.x + 1;
        m.ym = wrap1(m.y - 1, sy);
        m.yp = wrap1(m.y + 1, sy);
        m.za = wz + (seg * nzi) / nseg;
        m.zb = wz + ((seg + 1) * nzi) / nseg;
        return m;
    };
    auto march = [&](const Item& m, const T* F, T* G) {
        PlaneRegs<T> Rm{}, R0{}, Rp{};
        column_plane<T, S, C, PS>(F, P, pl, rw, wrap1(m.za - 1, sz), m.x, m.xm, m.xp, m.y, m.ym, m.yp,
                                  false, k.eps, Rm);
        column_plane<T, S, C, PS>(F, P, pl, rw, m.za, m.x, m.xm, m.xp, m.y, m.ym, m.yp, true, k.eps, R0);
        for (int z = m.za; z < m.zb; ++z) {
            column_plane<T, S, C, PS>(F, P, pl, rw, wrap1(z + 1, sz), m.x, m.xm, m.xp, m.y, m.ym, m.yp, true,
                                      k.eps, Rp);
            G[z * pl + m.y * rw + m.x] = point_from_planes<T, S, C>(Rm, R0, Rp, k);
            Rm = R0;
            R0 = Rp;
        }
    };
    // Ghost cell i: its interior neighbour and the Eq. 7 coefficient of its
    // class, or src < 0 for an interior cell.
    auto ghost = [&](int i, int& src, int& cls) {
        const int lx = i % rw, y = (i / rw) % sy, z = i / pl;
        const int x = rx0 + lx;   // a walled x axis is never wrapped
        const int cx = wx ? (x == 0 ? -1 : (x == sx - 1 ? 1 : 0)) : 0;
        const int cy = wy ? (y == 0 ? -1 : (y == sy - 1 ? 1 : 0)) : 0;
        const int cz = wz ? (z == 0 ? -1 : (z == sz - 1 ? 1 : 0)) : 0;
        src = (cx | cy | cz) ? (z - cz) * pl + (y - cy) * rw + (lx - cx) : -1;
        cls = (cx + 1) + 3 * (cy + 1) + 9 * (cz + 1);
    };
    // Regions of at most two cells per thread and one work item per thread
    // (segments, small grids) keep their cells' and item's indices in registers
    // for every step; larger ones recompute them.
    const bool few = cells <= 2 * kResThreads && items_n <= kResThreads;
    int src0 = -1, cls0 = 0, src1 = -1, cls1 = 0;
    Item m0{};
    if (few) {
        if (W) {
            ghost(tid, src0, cls0);
            if (tid + kResThreads < cells) ghost(tid + kResThreads, src1, cls1);
        }
        if (tid < items_n) m0 = item(tid);
    }

    for (int step = 0; step < nsteps; ++step) {
        // Ghosts of the current copy from their interior neighbours (Eq. 7),
        // then (PS) psi' of every cell.  A ghost's source is an interior cell,
        // which no thread writes in this phase.
        if (few) {
            if (tid < cells) {
                if (W && src0 >= 0) A[tid] = wall_map(A[src0], wall[g].a[cls0]);
                if (PS) P[tid] = psi2(A[tid], k.eps);
            }
            const int i1 = tid + kResThreads;
            if (i1 < cells) {
                if (W && src1 >= 0) A[i1] = wall_map(A[src1], wall[g].a[cls1]);
                if (PS) P[i1] = psi2(A[i1], k.eps);
            }
        } else if (W || PS) {
            for (int i = tid; i < cells; i += kResThreads) {
                if (W) {
                    int src, cls;
                    ghost(i, src, cls);
                    if (src >= 0) A[i] = wall_map(A[src], wall[g].a[cls]);
                }
                if (PS) P[i] = psi2(A[i], k.eps);
            }
        }
        __syncthreads();
        if (few) {
            if (tid < items_n) march(m0, A, B);
        } else {
            for (int t = tid; t < items_n; t += kResThreads) march(item(t), A, B);
        }
        __syncthreads();
        T* tmp = A;
        A = B;
        B = tmp;
    }
    if (whole) {
        for (int i = tid; i < cells; i += kResThreads) out[i] = A[i];
    } else {
        const int n = it.olen * sy * sz, lx0 = it.ox - rx0;
        for (int i = tid; i < n; i += kResThreads) {
            const int j = i % it.olen, row = i / it.olen;
            out[(size_t)row * sx + it.ox + j] = A[row * rw + lx0 + j];
        }
    }
}

// Lets kernel kfn take up to kResidentLdsBytes of dynamic LDS on the current
// device; set once per kernel and device (segmented runs launch often, and the
// attribute call costs host time on every launch).
template <typename K>
hipError_t allow_resident_lds(K kfn, std::atomic<unsigned>& done) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const unsigned bit = dev < 32 ? 1u << dev : 0u;
    if (bit && (done.load(std::memory_order_acquire) & bit)) return hipSuccess;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(kfn), hipFuncAttributeMaxDynamicSharedMemorySize,
                            kResidentLdsBytes);
    if (e == hipSuccess && bit) done.fetch_or(bit, std::memory_order_acq_rel);
    return e;
}

template <typename T, int S, int C>
struct ResidentLaunch {
    template <bool W, bool PS>
    static hipError_t go(const T* in, T* out, const StepCoef<T>* coef, const int64_t* offset,
                         const WallCoef<T>* wall, const ResItem* items, int nblocks, size_t lds,
                         int nsteps, hipStream_t s) {
        static std::atomic<unsigned> done{0};
        auto kfn = k_step_resident<T, S, C, W, PS>;
        const hipError_t e = allow_resident_lds(kfn, done);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kfn, dim3(nblocks), dim3(kResThreads), lds, s, in, out, coef, offset, wall, items,
                           nsteps);
        return hipGetLastError();
    }
    static hipError_t run(const T* in, T* out, const StepCoef<T>* coef, const int64_t* offset,
                          const WallCoef<T>* wall, const ResItem* items, int nblocks, int max_cells,
                          int nsteps, hipStream_t s) {
        // TI_n stages psi' in a third copy when the LDS holds it
        if constexpr (C == kLocal) {
            if (3 * (size_t)max_cells * sizeof(T) <= (size_t)kResidentLdsBytes) {
                const size_t lds = 3 * (size_t)max_cells * sizeof(T);
                return wall ? go<true, true>(in, out, coef, offset, wall, items, nblocks, lds, nsteps, s)
                            : go<false, true>(in, out, coef, offset, wall, items, nblocks, lds, nsteps, s);
            }
        }
        const size_t lds = 2 * (size_t)max_cells * sizeof(T);
        return wall ? go<true, false>(in, out, coef, offset, wall, items, nblocks, lds, nsteps, s)
                    : go<false, false>(in, out, coef, offset, wall, items, nblocks, lds, nsteps, s);
    }
};

template <typename T, typename... Args>
hipError_t resident_dispatch(int stencil, int coupling, Args... args) {
#define SPFM_RCASE(S_, C_)                                                  \
    if (stencil == S_ && coupling == C_) return ResidentLaunch<T, S_, C_>::run(args...);
    SPFM_RCASE(6, kLocal) SPFM_RCASE(6, kGlobal) SPFM_RCASE(6, kCF)
    SPFM_RCASE(18, kLocal) SPFM_RCASE(18, kGlobal) SPFM_RCASE(18, kCF)
    SPFM_RCASE(26, kLocal) SPFM_RCASE(26, kGlobal) SPFM_RCASE(26, kCF)
    SPFM_RCASE(6, kCF5) SPFM_RCASE(18, kCF5) SPFM_RCASE(26, kCF5)
    SPFM_RCASE(6, kCFAbel) SPFM_RCASE(18, kCFAbel) SPFM_RCASE(26, kCFAbel)
#undef SPFM_RCASE
    return hipErrorInvalidValue;
}

}  // namespace

int resident_max_cells(int elem_bytes) { return kResidentLdsBytes / (2 * elem_bytes); }

template <typename T>
hipError_t launch_step_resident(const T* buf_in, T* buf_out, const StepCoef<T>* d_coef,
                                const int64_t* d_offset, const WallCoef<T>* d_wall,
                                const ResItem* d_items, int nblocks, int max_cells, int nsteps,
                                int stencil, int coupling, hipStream_t s) {
    if (nblocks <= 0 || nsteps <= 0) return hipSuccess;
    if (max_cells <= 0 || max_cells > resident_max_cells((int)sizeof(T))) return hipErrorInvalidValue;
    if (d_items && buf_in == buf_out) return hipErrorInvalidValue;   // blocks read each other's halos
    return resident_dispatch<T>(stencil, coupling, buf_in, buf_out, d_coef, d_offset, d_wall, d_items,
                                nblocks, max_cells, nsteps, s);
}

template hipError_t launch_step_resident<float>(const float*, float*, const StepCoef<float>*,
                                                const int64_t*, const WallCoef<float>*, const ResItem*,
                                                int, int, int, int, int, hipStream_t);
template hipError_t launch_step_resident<double>(const double*, double*, const StepCoef<double>*,
                                                 const int64_t*, const WallCoef<double>*, const ResItem*,
                                                 int, int, int, int, int, hipStream_t);

}  // namespace spfm
