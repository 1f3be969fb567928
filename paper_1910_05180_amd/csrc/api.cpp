// C ABI of the SPFM GPU library (declared in include/spfm.h).
//
// A context owns (or adopts) two device buffers holding phi^n and phi^{n+1},
// the step coefficients, a small reduction scratch area and, on non-null
// streams, cached HIP graphs of kGraphSteps consecutive step launches (one per
// starting buffer) that spfm_step replays for long runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/spfm.h"
#include "host_math.h"

using namespace spfm;

namespace {

thread_local char g_err[512] = "";

spfm_status fail(spfm_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(SPFM_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));       \
    } while (0)

constexpr int kGraphSteps = 16;

// Dimensions of a stored grid, as the tile schedules see it.
struct GridDims {
    int nx, ny, nz;
};

constexpr int kResidentChunk = 4096;   // most steps of one whole-grid resident launch

struct Resolved {
    Params p;
    int dtype, kernel, allow_unstable;
    int tsteps;   // steps per launch (temporal blocking), 1 = one step
    int tile;     // tile shape of the tiled kernel asked for (TileShape), -1 = library choice
    int conserve_volume;   // mu chosen at every step so that sum phi is constant
    int walls;    // bit d: contact-angle walls on axis d
    double wall_sin[6];
    int sx, sy, sz;   // stored dims: the grid plus one ghost layer per end of a walled axis
    double dt_max;
    int seg_len, seg_halo;   // resident x segments asked for (batches), 0 = none
};

// Validate and resolve everything that does not touch the GPU.
spfm_status resolve(const spfm_grid* g, double lambda, double Gamma, double M, double mu,
                    int stencil, const spfm_options* opt, Resolved* r) {
    if (!g) return fail(SPFM_E_INVAL, "grid is NULL");
    spfm_options o;
    if (opt) o = *opt; else std::memset(&o, 0, sizeof o);
    // A periodic axis needs 3 points; a walled one 1 (its ghost layers complete the stencil).
    const int wmask = opt ? opt->walls : 0;
    const int emin[3] = {(wmask & 1) ? 1 : 3, (wmask & 2) ? 1 : 3, (wmask & 4) ? 1 : 3};
    if (g->nx < emin[0] || g->ny < emin[1] || g->nz < emin[2])
        return fail(SPFM_E_INVAL, "grid edges must be >= 3, or >= 1 on walled axes (got %d x %d x %d)",
                    g->nx, g->ny, g->nz);
    if (!(g->dx > 0.0) || !std::isfinite(g->dx)) return fail(SPFM_E_INVAL, "dx must be > 0");
    if (!(lambda > 0.0) || !(Gamma > 0.0) || !(M > 0.0) || !std::isfinite(lambda) ||
        !std::isfinite(Gamma) || !std::isfinite(M))
        return fail(SPFM_E_INVAL, "lambda, Gamma and M must be finite and > 0");
    if (!std::isfinite(mu)) return fail(SPFM_E_INVAL, "mu must be finite");
    if (stencil != 6 && stencil != 18 && stencil != 26)
        return fail(SPFM_E_INVAL, "stencil must be 6, 18 or 26 (got %d)", stencil);
    if (o.dtype != SPFM_F32 && o.dtype != SPFM_F64) return fail(SPFM_E_INVAL, "unknown dtype %d", o.dtype);
    if (o.walls < 0 || o.walls > 7) return fail(SPFM_E_INVAL, "walls must be a mask of axes (0..7)");
    for (int f = 0; f < 6; ++f)
        if ((o.walls >> (f / 2)) & 1)
            if (!(std::fabs(o.wall_sin[f]) <= 1.0))
                return fail(SPFM_E_INVAL, "wall_sin[%d] must be in [-1, 1]", f);
    if (o.walls && o.tsteps > 1) return fail(SPFM_E_INVAL, "walls need one step per launch (tsteps <= 1)");
    if (o.conserve_volume && (o.walls || o.tsteps > 1))
        return fail(SPFM_E_INVAL, "constant volume needs a periodic grid and one step per launch");
    // Stored dims.  The tiled kernels address one z-plane through a buffer
    // descriptor with 32-bit byte offsets.
    const int sx = g->nx + 2 * (o.walls & 1), sy = g->ny + 2 * ((o.walls >> 1) & 1),
              sz = g->nz + 2 * ((o.walls >> 2) & 1);
    const int64_t esize = o.dtype == SPFM_F64 ? 8 : 4;
    if ((int64_t)sx * sy * esize >= (int64_t)1 << 31 || (int64_t)sx * sy * sz > ((int64_t)1 << 40) ||
        sz > 65535 || sy > 4 * 65535)
        return fail(SPFM_E_INVAL,
                    "grid too large (one stored z-plane < 2^31 bytes, ny <= 262140, nz <= 65535)");
    if (o.coupling != SPFM_LOCAL && o.coupling != SPFM_GLOBAL && o.coupling != SPFM_CF)
        return fail(SPFM_E_INVAL, "unknown coupling %d", o.coupling);
    if (o.kernel < SPFM_KERNEL_AUTO || o.kernel > SPFM_KERNEL_RESIDENT)
        return fail(SPFM_E_INVAL, "unknown kernel %d", o.kernel);
    if (o.kernel == SPFM_KERNEL_RESIDENT) {
        if ((int64_t)sx * sy * sz > resident_max_cells((int)esize))
            return fail(SPFM_E_INVAL, "the resident kernel holds at most %d stored points of this dtype",
                        resident_max_cells((int)esize));
        if (o.tsteps > 1 || o.conserve_volume)
            return fail(SPFM_E_INVAL, "the resident kernel takes single steps at fixed mu");
    }
    if (o.zchunk < 0 || o.zchunk > 4096) return fail(SPFM_E_INVAL, "zchunk must be in 0..4096");
    r->seg_len = r->seg_halo = 0;
    if (o.segment[0] != 0 || o.segment[1] != 0) {
        if (o.segment[0] < 1 || o.segment[1] < 1 || o.segment[1] > 4096 ||
            o.kernel == SPFM_KERNEL_TILED || o.kernel == SPFM_KERNEL_PLAIN)
            return fail(SPFM_E_INVAL, "segment needs length >= 1, halo in 1..4096 and the resident "
                                      "kernel (or AUTO)");
        r->seg_len = o.segment[0];
        r->seg_halo = o.segment[1];
    }
    r->tile = -1;
    if (o.tile[0] != 0 || o.tile[1] != 0) {
        int t = -1;
        for (int k = 0; k < kNumTileShapes; ++k)
            if (tile_tx(k) == o.tile[0] && tile_ty(k) == o.tile[1]) t = k;
        const int kc = kernel_coupling(o.coupling, o.interp);
        if (t < 0 || !tile_compiled(o.dtype == SPFM_F32, kc, o.walls != 0, t) ||
            o.kernel == SPFM_KERNEL_PLAIN || o.kernel == SPFM_KERNEL_RESIDENT ||
            (o.conserve_volume && t != default_tile(o.dtype == SPFM_F32, kc)))
            return fail(SPFM_E_INVAL,
                        "tile %d x %d is not compiled for this dtype, coupling and walls (or kernel; "
                        "constant volume: the default shape only), see spfm_options.tile",
                        o.tile[0], o.tile[1]);
        r->tile = t;
    }
    if (o.tsteps < 0 || o.tsteps > 4) return fail(SPFM_E_INVAL, "tsteps must be in 0..4");
    if (o.tsteps > 1 && (o.dtype != SPFM_F32 || o.kernel == SPFM_KERNEL_PLAIN))
        return fail(SPFM_E_INVAL, "tsteps > 1 needs dtype F32 and the tiled kernel");
    const double un = std::sqrt(o.u[0] * o.u[0] + o.u[1] * o.u[1] + o.u[2] * o.u[2]);
    if (o.coupling == SPFM_GLOBAL && !(un > 0.0 && std::isfinite(un)))
        return fail(SPFM_E_INVAL, "GLOBAL coupling needs a nonzero direction u");
    if (o.dtype == SPFM_F32 && lambda < 0.3 * g->dx)
        return fail(SPFM_E_INVAL, "F32 needs lambda >= 0.3 dx (got lambda/dx = %g)", lambda / g->dx);
    if ((o.d_phi[0] == nullptr) != (o.d_phi[1] == nullptr))
        return fail(SPFM_E_INVAL, "give both d_phi buffers or neither");
    if (o.d_phi[0] && o.d_phi[0] == o.d_phi[1]) return fail(SPFM_E_INVAL, "d_phi buffers must differ");
    Params& p = r->p;
    p.nx = g->nx; p.ny = g->ny; p.nz = g->nz;
    p.dx = g->dx; p.lambda = lambda; p.Gamma = Gamma; p.M = M; p.mu = mu;
    p.stencil = stencil; p.coupling = o.coupling;
    for (int i = 0; i < 3; ++i) p.u[i] = o.u[i];
    if (o.gamma[0] == 0.0 && o.gamma[1] == 0.0 && o.gamma[2] == 0.0) {
        default_gamma(stencil, p.gamma);
    } else {
        for (int i = 0; i < 3; ++i) {
            if (!(o.gamma[i] >= 0.0) || !std::isfinite(o.gamma[i]))
                return fail(SPFM_E_INVAL, "shell weights must be finite and >= 0");
            p.gamma[i] = o.gamma[i];
        }
    }
    p.C_Gamma = o.C_Gamma > 0.0 ? o.C_Gamma : calibrate_cgamma(lambda / g->dx, o.coupling);
    if (!(p.C_Gamma > 0.0) || !std::isfinite(p.C_Gamma)) return fail(SPFM_E_INVAL, "bad C_Gamma");
    p.eps = o.eps > 0.0 ? o.eps : (o.dtype == SPFM_F32 ? 1e-30 : 1e-300);
    p.tau = o.tau > 0.0 ? o.tau : 1e-3;
    p.dt = o.dt > 0.0 ? o.dt : 0.1 * g->dx * g->dx / (M * Gamma);
    if (!std::isfinite(p.dt)) return fail(SPFM_E_INVAL, "dt must be finite");
    r->dtype = o.dtype;
    r->kernel = o.kernel == SPFM_KERNEL_AUTO ? SPFM_KERNEL_TILED : o.kernel;
    r->allow_unstable = o.allow_unstable;
    r->tsteps = o.tsteps > 1 ? o.tsteps : 1;
    r->walls = o.walls;
    r->conserve_volume = o.conserve_volume ? 1 : 0;
    for (int f = 0; f < 6; ++f) r->wall_sin[f] = ((o.walls >> (f / 2)) & 1) ? o.wall_sin[f] : 0.0;
    r->sx = sx; r->sy = sy; r->sz = sz;
    if (o.interp < kH3 || o.interp > kHAbel) return fail(SPFM_E_INVAL, "unknown interp %d", o.interp);
    if (o.interp != kH3 && o.coupling != kCF)
        return fail(SPFM_E_INVAL, "h5 and h_Abel go with the CF coupling (Tab. 2)");
    p.interp = o.interp;
    r->dt_max = stable_dt(stencil, o.coupling, p.u, p.gamma, lambda, Gamma, M, mu, g->dx, p.C_Gamma,
                          p.interp);
    if (!o.allow_unstable && p.dt > r->dt_max)
        return fail(SPFM_E_UNSTABLE, "dt = %g exceeds the explicit stability bound %g", p.dt, r->dt_max);
    return SPFM_OK;
}

size_t elem_size(int dtype) { return dtype == SPFM_F64 ? 8 : 4; }

// Reduction scratch: per-block partials and the pinned host copy of the result.
struct Reducer {
    double* d_partials = nullptr;
    ReduceOut* d_out = nullptr;
    ReduceOut* h_out = nullptr;
    spfm_status init() {
        HIP_TRY(hipMalloc(&d_partials, sizeof(double) * kReduceBlocks * kPartialStride));
        HIP_TRY(hipMalloc(&d_out, sizeof(ReduceOut)));
        HIP_TRY(hipHostMalloc(&h_out, sizeof(ReduceOut), hipHostMallocDefault));
        return SPFM_OK;
    }
    void release() {
        if (d_partials) (void)hipFree(d_partials);
        if (d_out) (void)hipFree(d_out);
        if (h_out) (void)hipHostFree(h_out);
        d_partials = nullptr; d_out = nullptr; h_out = nullptr;
    }
    // Reduce n values of dtype at d_phi into *h_out (synchronises s).
    spfm_status run(const void* d_phi, int dtype, int64_t n, hipStream_t s) {
        hipError_t e = dtype == SPFM_F64
                           ? launch_reduce<double>((const double*)d_phi, n, d_partials, d_out, s)
                           : launch_reduce<float>((const float*)d_phi, n, d_partials, d_out, s);
        if (e != hipSuccess) return fail(SPFM_E_HIP, "reduction launch: %s", hipGetErrorString(e));
        HIP_TRY(hipMemcpyAsync(h_out, d_out, sizeof(ReduceOut), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        return SPFM_OK;
    }
};

// Interface bookkeeping of the diagnostics.
struct Tracker {
    int kind = 0;            // 0 none, 1 planar slab, 2 single sphere
    double V1_ref = 0.0, A_ref = 0.0;
    bool ref_pending = false;
    bool have_last = false;
    double last_pos = 0.0, last_time = 0.0;
    void reset(int k, double area) {
        kind = k; A_ref = area; ref_pending = (k == 1); have_last = false;
    }
    void fill(spfm_diag* d, const ReduceOut& r, double dx, double lambda, int64_t step, double dt) {
        const double dv = dx * dx * dx;
        d->step = step;
        d->time = step * dt;
        d->sum_phi = r.sum_phi;
        d->sum_x = r.sum_x;
        d->phase_volume = r.sum_phi * dv;
        d->interface_area = 4.0 / lambda * r.sum_x * dv;
        d->phi_min = r.phi_min;
        d->phi_max = r.phi_max;
        d->diverged = (int32_t)std::min<unsigned long long>(r.bad, 0x7fffffffULL);
        if (kind == 1 && ref_pending) { V1_ref = d->phase_volume; ref_pending = false; }
        double pos = NAN;
        if (kind == 1) {
            pos = (d->phase_volume - V1_ref) / A_ref;
        } else if (kind == 2) {
            // (4 pi / 3)(R^3 + R pi^2 lambda^2 / 16) = V1, Newton from the sharp radius
            const double V = d->phase_volume, c = M_PI * M_PI * lambda * lambda / 16.0;
            double R = std::cbrt(3.0 * V / (4.0 * M_PI));
            for (int it = 0; it < 60 && R > 0.0; ++it)
                R -= (4.0 * M_PI / 3.0 * (R * R * R + R * c) - V) / (4.0 * M_PI / 3.0 * (3.0 * R * R + c));
            pos = R;
        }
        d->interface_position = pos;
        d->velocity = (have_last && d->time != last_time) ? (pos - last_pos) / (d->time - last_time) : NAN;
        if (d->time != last_time || !have_last) {
            last_pos = pos; last_time = d->time; have_last = true;
        }
    }
};

double slab_area(int nx, int ny, int nz, double dx, const int32_t hkl[3]) {
    auto gcd = [](int64_t a, int64_t b) {
        a = a < 0 ? -a : a; b = b < 0 ? -b : b;
        while (b) { int64_t t = a % b; a = b; b = t; }
        return a;
    };
    const double nn = std::sqrt((double)hkl[0] * hkl[0] + (double)hkl[1] * hkl[1] + (double)hkl[2] * hkl[2]);
    const int64_t g = gcd(gcd(gcd(0, (int64_t)nx * hkl[0]), (int64_t)ny * hkl[1]), (int64_t)nz * hkl[2]);
    const double P = (double)g * dx / nn;
    return 2.0 * (double)nx * ny * nz * dx * dx * dx / P;
}

// Wall coefficients of a resolved grid: stored dims, walled axes and the
// composed Eq. 7 coefficient of every ghost class (the shifts of the walls
// crossed from the ghost to its interior point add up).
template <typename T>
WallCoef<T> wall_coef(const Resolved& r) {
    WallCoef<T> w;
    w.sx = r.sx;
    w.sy = r.sy;
    w.sz = r.sz;
    w.walls = r.walls;
    for (int cz = -1; cz <= 1; ++cz)
        for (int cy = -1; cy <= 1; ++cy)
            for (int cx = -1; cx <= 1; ++cx) {
                const int c[3] = {cx, cy, cz};
                double sh = 0.0;
                for (int d = 0; d < 3; ++d)
                    if (c[d] != 0) sh += r.wall_sin[2 * d + (c[d] > 0 ? 1 : 0)];
                w.a[(cx + 1) + 3 * (cy + 1) + 9 * (cz + 1)] = (T)std::tanh(2.0 * r.p.dx * sh / r.p.lambda);
            }
    return w;
}

// Copies between a dense grid-shaped array and the interior of a stored field
// (walls on the axes of the mask: one ghost layer at each end).
template <typename T>
hipError_t copy_to_interior(T* stored, const T* dense, const Resolved& r, hipStream_t s) {
    const Params& p = r.p;
    return launch_box_copy<T>(stored, r.sx, r.sy, r.walls & 1, (r.walls >> 1) & 1, (r.walls >> 2) & 1,
                              dense, p.nx, p.ny, 0, 0, 0, p.nx, p.ny, p.nz, s);
}
template <typename T>
hipError_t copy_from_interior(T* dense, const T* stored, const Resolved& r, hipStream_t s) {
    const Params& p = r.p;
    return launch_box_copy<T>(dense, p.nx, p.ny, 0, 0, 0, stored, r.sx, r.sy, r.walls & 1,
                              (r.walls >> 1) & 1, (r.walls >> 2) & 1, p.nx, p.ny, p.nz, s);
}

// Area of a planar front of normal n in a box: the cross-section normal to the
// axis the front crosses (largest |n_d|) divided by that component of n / |n|.
double front_area(const Params& p, const double n[3]) {
    const double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    int d = 0;
    for (int k = 1; k < 3; ++k)
        if (std::fabs(n[k]) > std::fabs(n[d])) d = k;
    const int ext[3] = {p.nx, p.ny, p.nz};
    return (double)ext[(d + 1) % 3] * ext[(d + 2) % 3] * p.dx * p.dx / (std::fabs(n[d]) / nn);
}

// Replays of kGraphSteps launches captured from a step function, one graph per
// starting buffer (exec[0..1]; the fused constant-volume steps of a context use
// exec[2..3]); invalidated whenever the coefficients change.
struct GraphCache {
    hipGraphExec_t exec[4] = {nullptr, nullptr, nullptr, nullptr};
    void clear() {
        for (auto& e : exec) {
            if (e) (void)hipGraphExecDestroy(e);
            e = nullptr;
        }
    }
};

}  // namespace

struct spfm_ctx {
    Resolved r;
    int device = 0;           // the device current at create (the buffers live there)
    hipStream_t stream = nullptr;
    void* buf[2] = {nullptr, nullptr};
    bool owns = false;
    int cur = 0;
    int64_t nsteps = 0;
    StepCoef<float> kf;
    StepCoef<double> kd;
    Reducer red;
    Tracker track;
    GraphCache graphs;

    WallCoef<float> wf;
    WallCoef<double> wd;
    int64_t nghost = 0;
    // Device copy of the wall coefficients of the stored dtype (walls only), read
    // by the tiled kernels, which compute the ghosts they need themselves.
    void* d_wall = nullptr;
    // Constant volume: coefficients without the driving force, and device
    // scratch for the reductions (kReduceBlocks x 8 partials, then g, mu, then
    // the 7 contour results).
    StepCoef<float> kf0;
    StepCoef<double> kd0;
    double* d_scratch = nullptr;
    double* d_part() const { return d_scratch; }
    double* d_state() const { return d_scratch + (size_t)kReduceBlocks * 8; }
    double* d_contour() const { return d_state() + 2; }
    static constexpr size_t kScratchDoubles = (size_t)kReduceBlocks * 8 + 2 + 7;

    // Grid points (the interior when there are walls) and the stored field.
    int64_t points() const { return (int64_t)r.p.nx * r.p.ny * r.p.nz; }
    size_t bytes() const { return (size_t)points() * elem_size(r.dtype); }
    size_t stored_bytes() const { return (size_t)r.sx * r.sy * r.sz * elem_size(r.dtype); }
    // Copy between a dense grid-shaped array and the interior of a stored field.
    hipError_t to_interior(void* stored, const void* dense) {
        return r.dtype == SPFM_F64
                   ? copy_to_interior<double>((double*)stored, (const double*)dense, r, stream)
                   : copy_to_interior<float>((float*)stored, (const float*)dense, r, stream);
    }
    hipError_t from_interior(void* dense, const void* stored) {
        return r.dtype == SPFM_F64
                   ? copy_from_interior<double>((double*)dense, (const double*)stored, r, stream)
                   : copy_from_interior<float>((float*)dense, (const float*)stored, r, stream);
    }
    // A grid-dense array of the current field: the live buffer itself, or (with
    // walls) its interior packed into the other buffer, which the next step
    // overwrites anyway.
    hipError_t dense_field(const void** out) {
        if (!r.walls) { *out = buf[cur]; return hipSuccess; }
        *out = buf[1 - cur];
        return from_interior(buf[1 - cur], buf[cur]);
    }

    // Resident kernel: the step coefficients of the stored dtype and the grid's
    // offset (0) in device memory, uploaded before a launch when changed.
    void* d_coef = nullptr;
    int64_t* d_off = nullptr;
    bool coef_dirty = true;
    hipError_t launch_resident(int from, int to, int nsteps) {
        const int S = r.p.stencil, C = kernel_coupling(r.p.coupling, r.p.interp);
        const int cells = r.sx * r.sy * r.sz;
        const bool f64 = r.dtype == SPFM_F64;
        if (coef_dirty) {
            const hipError_t e = hipMemcpyAsync(d_coef, f64 ? (const void*)&kd : (const void*)&kf,
                                                f64 ? sizeof kd : sizeof kf, hipMemcpyHostToDevice, stream);
            if (e != hipSuccess) return e;
            coef_dirty = false;
        }
        return f64 ? launch_step_resident<double>((const double*)buf[from], (double*)buf[to],
                                                  (const StepCoef<double>*)d_coef, d_off,
                                                  (const WallCoef<double>*)d_wall, nullptr, 1, cells,
                                                  nsteps, S, C, stream)
                   : launch_step_resident<float>((const float*)buf[from], (float*)buf[to],
                                                 (const StepCoef<float>*)d_coef, d_off,
                                                 (const WallCoef<float>*)d_wall, nullptr, 1, cells,
                                                 nsteps, S, C, stream);
    }
    // Resident launches: up to kResidentChunk steps, in place for even counts.
    int resident_chunk() const { return kResidentChunk; }
    bool resident_in_place() const { return true; }

    int zlen = kTileZ;        // planes per block of the tiled kernel (the leading chunks)
    int tile = kTile64x8;     // tile shape of the tiled kernel (TileShape)
    bool tune_z = false;      // SPFM_KERNEL_AUTO without zchunk: time z-chunks at the first step
    bool tune_tile = false;   // SPFM_KERNEL_AUTO without tile: time tile shapes at the first step
    bool tuned = false;
    // Work items of the tiled kernel (tile_schedule of the stored grid for zlen).
    TileItem* d_items = nullptr;
    int nitems = 0;
    size_t items_cap = 0;
    // Constant volume with the tiled kernel: the step's exact sums, 4 words per
    // work item, in two sets (consecutive steps of the fused form), then 4
    // words for their total (2 items_cap + 1 entries); and the second pair of
    // field buffers of the fused form, allocated at its first use.
    unsigned long long* d_cvpart = nullptr;
    void* xbuf[2] = {nullptr, nullptr};
    // One grid: tile rows are dealt to the XCDs round robin.
    static constexpr bool kSpreadRows = true;

    // Steps per launch of launch_unit.
    int unit() const { return r.tsteps; }
    // r.tsteps steps from buf[from] into buf[1 - from] in one launch.
    hipError_t launch_unit(int from) {
        if (r.tsteps == 1) return launch_one(from);
        return launch_step_temporal((const float*)buf[from], (float*)buf[1 - from], kf, r.p.stencil,
                                    kernel_coupling(r.p.coupling, r.p.interp), r.tsteps, zlen, stream);
    }
    hipError_t launch_one(int from) {
        if (r.kernel == SPFM_KERNEL_RESIDENT) return launch_resident(from, 1 - from, 1);
        const void* in = buf[from];
        void* out = buf[1 - from];
        const int S = r.p.stencil, C = kernel_coupling(r.p.coupling, r.p.interp);
        if (r.walls && r.kernel == SPFM_KERNEL_PLAIN) {   // ghost layers of the input from Eq. 7
            const hipError_t e = r.dtype == SPFM_F64
                                     ? launch_fill_walls<double>((double*)buf[from], wd, nghost, stream)
                                     : launch_fill_walls<float>((float*)buf[from], wf, nghost, stream);
            if (e != hipSuccess) return e;
        }
        const StepCoef<double>& cd = r.conserve_volume ? kd0 : kd;
        const StepCoef<float>& cf = r.conserve_volume ? kf0 : kf;
        // constant volume, tiled: the step also forms the sums of its work items
        unsigned long long* cvp = r.conserve_volume ? d_cvpart : nullptr;
        hipError_t e;
        if (r.dtype == SPFM_F64) {
            e = r.kernel == SPFM_KERNEL_PLAIN
                    ? launch_step_plain<double>((const double*)in, (double*)out, cd, S, C, stream)
                    : launch_step_tiled<double>((const double*)in, (double*)out, cd, S, C, tile,
                                                d_items, nitems, (const WallCoef<double>*)d_wall, cvp,
                                                nullptr, stream);
        } else {
            e = r.kernel == SPFM_KERNEL_PLAIN
                    ? launch_step_plain<float>((const float*)in, (float*)out, cf, S, C, stream)
                    : launch_step_tiled<float>((const float*)in, (float*)out, cf, S, C, tile, d_items,
                                               nitems, (const WallCoef<float>*)d_wall, cvp, nullptr, stream);
        }
        if (e != hipSuccess || !r.conserve_volume) return e;
        // the step ran without the driving force; add the one that keeps sum phi
        const double dt_beta = r.p.dt * 2.0 * r.p.M / (3.0 * r.p.lambda * r.p.Gamma);
        const bool f64 = r.dtype == SPFM_F64;
        if (r.kernel == SPFM_KERNEL_PLAIN) {
            unsigned long long* part = reinterpret_cast<unsigned long long*>(d_part());
            return f64 ? launch_cv_correct<double>((const double*)in, (double*)out, points(), r.p.interp,
                                                   dt_beta, part, d_state(), stream)
                       : launch_cv_correct<float>((const float*)in, (float*)out, points(), r.p.interp,
                                                  dt_beta, part, d_state(), stream);
        }
        unsigned long long* total = d_cvpart + 8 * items_cap;
        return f64 ? launch_cv_apply<double>((const double*)in, (double*)out, points(), r.p.interp, dt_beta,
                                             d_cvpart, nitems, total, d_state(), stream)
                   : launch_cv_apply<float>((const float*)in, (float*)out, points(), r.p.interp, dt_beta,
                                            d_cvpart, nitems, total, d_state(), stream);
    }
    // New step coefficients from r; drops the cached graphs, so no replay may
    // still be queued (callers synchronise the stream first).
    void refresh_coef() {
        kf = make_coef<float>(r.p);
        kd = make_coef<double>(r.p);
        kf.nx = kd.nx = r.sx;   // the kernels sweep the stored grid
        kf.ny = kd.ny = r.sy;
        kf.nz = kd.nz = r.sz;
        Params p0 = r.p;
        p0.mu = 0.0;
        kf0 = make_coef<float>(p0);
        kd0 = make_coef<double>(p0);
        kf0.nx = kd0.nx = r.sx;
        kf0.ny = kd0.ny = r.sy;
        kf0.nz = kd0.nz = r.sz;
        wf = wall_coef<float>(r);
        wd = wall_coef<double>(r);
        nghost = wall_ghosts(r.sx, r.sy, r.sz, r.walls);
        coef_dirty = true;
        graphs.clear();
    }
};

struct spfm_batch {
    int n = 0;
    std::vector<Resolved> r;
    std::vector<int64_t> offset;   // element offset of each grid in the buffers
    int64_t total = 0;              // allocated elements (with padding)
    int64_t points = 0;
    hipStream_t stream = nullptr;
    float* buf[2] = {nullptr, nullptr};
    int cur = 0;
    int64_t nsteps = 0;
    StepCoef<float>* d_coef = nullptr;
    int64_t* d_offset = nullptr;
    // Work items of the batched kernel: tile_schedule of the stored grids for
    // leading z-chunks of zlen planes, with tile width tx; with SPFM_KERNEL_AUTO
    // and no zchunk the length is timed at the first step.
    TileItem* d_items = nullptr;
    int nitems = 0;
    size_t items_cap = 0;
    std::vector<GridDims> dims;
    int tile = kTile16x8, zlen = kTileZ;
    bool tune_z = false, tune_tile = false, tuned = false;
    bool walled_f32 = false;
    // Many grids, often larger than the last-level cache together: tile rows
    // are dealt to the XCDs in contiguous groups.
    static constexpr bool kSpreadRows = false;
    int stencil = 26, coupling = 0;
    // Walls (the same axes on every grid): per-grid coefficients on the device,
    // read by the batched kernel, which computes the ghosts it needs itself.
    int walls = 0;
    WallCoef<float>* d_wall = nullptr;
    Reducer red;
    std::vector<Tracker> track;
    GraphCache graphs;

    // Resident kernel (every stored grid fits the LDS of one workgroup): one
    // launch takes many steps of all grids; max_cells is the largest stored grid.
    // With x segments (seg_len > 0): the nres blocks of d_res, each region at
    // most res_cells points, at most seg_halo steps per launch, out of place.
    bool resident = false;
    int max_cells = 0;
    bool tune_res = false, res_tuned = false;   // AUTO: time tiled, whole and segmented at the first step
    int seg_len = 0, seg_halo = 0;
    ResItem* d_res = nullptr;
    size_t res_cap = 0;
    int nres = 0, res_cells = 0;
    hipError_t launch_resident(int from, int to, int nsteps) {
        if (seg_len > 0)
            return launch_step_resident<float>(buf[from], buf[to], d_coef, d_offset, walls ? d_wall : nullptr,
                                               d_res, nres, res_cells, nsteps, stencil, coupling, stream);
        return launch_step_resident<float>(buf[from], buf[to], d_coef, d_offset, walls ? d_wall : nullptr,
                                           nullptr, n, max_cells, nsteps, stencil, coupling, stream);
    }
    // Whole grids (run_resident); segments run through run_steps (launch_unit).
    int resident_chunk() const { return kResidentChunk; }
    bool resident_in_place() const { return true; }

    // Steps per unit launch: one, or a halo's worth for resident segments, whose
    // launches then run like tiled ones (graph replays, out of place).
    bool segmented() const { return resident && seg_len > 0; }
    int unit() const { return segmented() ? seg_halo : 1; }
    hipError_t launch_unit(int from) {
        return segmented() ? launch_resident(from, 1 - from, seg_halo) : launch_one(from);
    }
    hipError_t launch_one(int from) {
        if (resident) return launch_resident(from, 1 - from, 1);
        return launch_step_batched(buf[from], buf[1 - from], d_coef, d_offset, d_items, nitems,
                                   walls ? d_wall : nullptr, stencil, coupling, tile, stream);
    }
    // Grid i as a dense array: its region of the current buffer, or (with walls)
    // its interior packed into its region of the other buffer, which the next
    // step overwrites anyway.
    hipError_t dense_grid(int i, const float** out) {
        if (!walls) { *out = buf[cur] + offset[i]; return hipSuccess; }
        *out = buf[1 - cur] + offset[i];
        return copy_from_interior<float>(buf[1 - cur] + offset[i], buf[cur] + offset[i], r[i], stream);
    }
    // Where a dense initial field of grid i is written before to_grid.
    float* dense_target(int i) { return (walls ? buf[1 - cur] : buf[cur]) + offset[i]; }
    hipError_t to_grid(int i) {
        if (!walls) return hipSuccess;
        return copy_to_interior<float>(buf[cur] + offset[i], buf[1 - cur] + offset[i], r[i], stream);
    }
};

namespace {

// z-chunks of one tile column of a single-step sweep: the first nz - tail
// planes in the fewest chunks of at most zb planes, of equal length to within
// one (phase 0), then the last `tail` planes in chunks that halve from zb / 2
// down to 8 planes (4 when zb < 16), two of each size (phases 1, 2, ... in
// order).  Each chunk stages two planes beyond its own, so the shortest tail
// chunks cost the most per point: on a 256^3 grid with zb = 32, ending at 8
// instead of 4 planes (16 chunks per column instead of 21) ran the step 1-1.5%
// faster, the drain at the end of the step no worse.
struct ZChunk {
    int z0, len, phase;
};
std::vector<ZChunk> guided_chunks(int nz, int zb, int tail) {
    std::vector<ZChunk> out;
    tail = std::max(0, std::min(nz, tail));
    const int lead = nz - tail, nlead = (lead + zb - 1) / zb;
    for (int i = 0, z = 0; i < nlead; ++i) {
        const int len = lead / nlead + (i < lead % nlead ? 1 : 0);
        out.push_back(ZChunk{z, len, 0});
        z += len;
    }
    int z = lead, phase = 1;
    const int smin = zb >= 16 ? 8 : 4;
    for (int size = std::max(zb / 2, smin); z < nz; size = std::max(size / 2, smin))
        for (int rep = 0; rep < 2 && z < nz; ++rep) {
            const int len = std::min(size, nz - z);
            out.push_back(ZChunk{z, len, phase++});
            z += len;
        }
    return out;
}

// Tail planes of a column of nz planes: the short chunks at the end of a step
// hold about 1.4 rounds of the work the GPU keeps resident (256 CUs x 4 SIMDs
// x 7 waves x 64 lanes, each lane owning one column point, times 32 planes),
// and at most 35% of the step (the fastest of 15%, 25%, 35%, 50% and 70% on a
// 256^3 grid).
int tail_planes(int nz, int64_t total_points) {
    const double resident = 256.0 * 4 * 7 * 64 * 32;
    const double f = std::min(0.35, 1.4 * resident / (double)std::max<int64_t>(total_points, 1));
    return std::min(nz, (int)std::lround(f * nz));
}

// Planes per block: the longest z-chunk (kTileZ for single steps, 2 kTileZ for
// fused ones, halved down to zmin) that still gives at least min_threads
// threads for tiles tx x ty over all grids, counting the guided chunks of the
// single-step schedule (guided) or uniform chunks (the temporal kernel); then
// halved on, down to 2 planes, while there are fewer than min_threads / 4
// (grids far too small to fill the GPU: a 60^3 step takes 12.8 us with chunks
// of 2 or 4 planes against 14.2 with 8).  A
// fused chunk also computes 2 T - 2 extra planes of its intermediate levels
// and reads 2 T extra input planes, which longer chunks amortise (CF, 3 fused
// steps on the 512^3 grains: 752 GLUPS with 64 planes, 710 with 32).  Grids too
// small to fill the GPU get shorter chunks: more blocks, each with a shorter
// dependent chain of plane loads.
int default_zlen(const std::vector<GridDims>& grids, int tx, int ty, bool guided,
                 int64_t min_threads, int zmin, int zfloor = 2) {
    int64_t total = 0;
    for (const GridDims& d : grids) total += (int64_t)d.nx * d.ny * d.nz;
    auto threads = [&](int zb) {
        int64_t t = 0;
        for (const GridDims& d : grids) {
            const int64_t cols = (int64_t)((d.nx + tx - 1) / tx) * ((d.ny + ty - 1) / ty);
            const int64_t ch = guided ? (int64_t)guided_chunks(d.nz, zb, tail_planes(d.nz, total)).size()
                                      : (d.nz + zb - 1) / zb;
            t += cols * ch * tx * ty;
        }
        return t;
    };
    int z = guided ? kTileZ : 2 * kTileZ;
    while (z > zmin && threads(z) < min_threads) z /= 2;
    while (guided && z > zfloor && threads(z) < min_threads / 4) z /= 2;
    return z;
}

// Work items of the tiled step over one or more grids (TileItem.inst = grid
// index), in dispatch order (block b runs on XCD b mod 8).  Every tile row (a
// grid and a row of ty tiles, through all x and z) belongs to one XCD, so its
// halo rows and z-chunk boundaries meet in one L2.  Rows are dealt to the XCDs
// round robin (spread: an interface concentrated in one part of a grid, like a
// centred grain, is shared by all XCDs) or in contiguous groups of equal point
// counts (so that neighbouring rows also share an L2, which pays when the
// fields do not fit the last-level cache).  Each XCD's list holds its rows' tile
// columns cut along z by guided_chunks (tails from tail_planes of the total
// point count): all phase-0 chunks first (grid by grid, z chunk by z chunk),
// then the tail chunks phase by phase, so the blocks dispatched last are short
// and the SIMDs run out of work together instead of idling behind a few long
// blocks at the end of the step.  Shorter XCD lists are padded with empty items
// (zlen 0).
std::vector<TileItem> tile_schedule(const std::vector<GridDims>& grids, int tx, int ty, int zb,
                                    bool spread) {
    struct Row {
        int inst, y0, xcd;
    };
    std::vector<Row> rows;
    int64_t total = 0;
    for (int g = 0; g < (int)grids.size(); ++g)
        for (int y0 = 0; y0 < grids[g].ny; y0 += ty) {
            rows.push_back(Row{g, y0, 0});
            total += (int64_t)grids[g].nx * grids[g].nz * std::min(ty, grids[g].ny - y0);
        }
    int64_t acc = 0;
    for (size_t r = 0; r < rows.size(); ++r) {
        const GridDims& d = grids[rows[r].inst];
        const int64_t w = (int64_t)d.nx * d.nz * std::min(ty, d.ny - rows[r].y0);
        // contiguous: the group whose share of the points holds the row's midpoint
        rows[r].xcd = spread ? (int)(r % kNumXcd)
                             : (int)std::min<int64_t>(kNumXcd - 1, (2 * acc + w) * kNumXcd / (2 * total));
        acc += w;
    }
    const size_t ng = grids.size();
    std::vector<std::vector<int>> y0s(kNumXcd * ng);   // row origins of grid g on XCD k
    for (const Row& row : rows) y0s[row.xcd * ng + row.inst].push_back(row.y0);
    std::vector<std::vector<ZChunk>> zc(ng);
    int nphase = 0;
    for (size_t g = 0; g < ng; ++g) {
        zc[g] = guided_chunks(grids[g].nz, zb, tail_planes(grids[g].nz, total));
        for (const ZChunk& c : zc[g]) nphase = std::max(nphase, c.phase + 1);
    }
    std::vector<std::vector<TileItem>> per(kNumXcd);
    for (int k = 0; k < kNumXcd; ++k)
        for (int ph = 0; ph < nphase; ++ph)
            for (size_t g = 0; g < ng; ++g) {
                if (y0s[k * ng + g].empty()) continue;
                for (const ZChunk& c : zc[g]) {
                    if (c.phase != ph) continue;
                    for (const int y0 : y0s[k * ng + g])
                        for (int x0 = 0; x0 < grids[g].nx; x0 += tx)
                            per[k].push_back(TileItem{(int)g, x0, y0, c.z0, c.len});
                }
            }
    size_t m = 0;
    for (const auto& v : per) m = std::max(m, v.size());
    std::vector<TileItem> out(m * kNumXcd, TileItem{0, 0, 0, 0, 0});
    for (int k = 0; k < kNumXcd; ++k)
        for (size_t i = 0; i < per[k].size(); ++i) out[i * kNumXcd + k] = per[k][i];
    return out;
}

// Builds and uploads the work items of a context or batch for leading
// z-chunks of zb planes (after the stream has drained: no launch may still read
// the old table); captured graphs hold the old table and are dropped.
template <typename Obj>
spfm_status set_schedule(Obj* o, const std::vector<GridDims>& dims, int tile, int zb) {
    HIP_TRY(hipStreamSynchronize(o->stream));
    const std::vector<TileItem> items = tile_schedule(dims, tile_tx(tile), tile_ty(tile), zb, Obj::kSpreadRows);
    if (items.size() > 0x7fffffff) return fail(SPFM_E_INVAL, "too many tiles");
    if (items.size() > o->items_cap) {
        if (o->d_items) (void)hipFree(o->d_items);
        o->d_items = nullptr;
        o->items_cap = 0;
        if (hipMalloc(&o->d_items, items.size() * sizeof(TileItem)) != hipSuccess) {
            (void)hipGetLastError();
            o->d_items = nullptr;
            return fail(SPFM_E_NOMEM, "device allocation of the tile schedule failed");
        }
        if constexpr (std::is_same<Obj, spfm_ctx>::value) {
            if (o->r.conserve_volume) {   // the step's constant-volume sums, then their total
                if (o->d_cvpart) (void)hipFree(o->d_cvpart);
                o->d_cvpart = nullptr;
                if (hipMalloc(&o->d_cvpart, (2 * items.size() + 1) * 4 * sizeof(unsigned long long)) !=
                    hipSuccess) {
                    (void)hipGetLastError();
                    o->d_cvpart = nullptr;
                    (void)hipFree(o->d_items);
                    o->d_items = nullptr;
                    return fail(SPFM_E_NOMEM, "device allocation of the constant-volume sums failed");
                }
            }
        }
        o->items_cap = items.size();
    }
    HIP_TRY(hipMemcpyAsync(o->d_items, items.data(), items.size() * sizeof(TileItem),
                           hipMemcpyHostToDevice, o->stream));
    HIP_TRY(hipStreamSynchronize(o->stream));
    o->nitems = (int)items.size();
    o->zlen = zb;
    o->tile = tile;
    o->graphs.clear();
    return SPFM_OK;
}
spfm_status set_schedule(spfm_ctx* c, int tile, int zb) {
    return set_schedule(c, {GridDims{c->r.sx, c->r.sy, c->r.sz}}, tile, zb);
}
spfm_status set_schedule(spfm_batch* b, int tile, int zb) { return set_schedule(b, b->dims, tile, zb); }

// SPFM_KERNEL_AUTO: time the step for the candidate (tile shape, z-chunk)
// pairs on the current field, reading the current buffer and writing the other
// one, which the next step overwrites anyway.  The untuned pair (the current
// one: the default shape and the size rule's length) is kept unless one of
// the three fastest other pairs beats it by at least 1% in final rounds that
// time the four against each other: the first steps of a process run while
// the clocks still ramp up, and the clocks follow the load of the previous
// launches.  When the size rule has already shortened the chunks below full
// (zlen < zfull), the work cannot fill the GPU, a launch takes about as long
// as the host needs to issue it, and timing single launches would measure the
// host: the untuned pair is kept.  The result of a step does not depend on the
// tile shape or the chunk length.
struct TuneCand {
    int tile, z;
};
template <typename Obj>
spfm_status tune_schedule(Obj* o, const std::vector<TuneCand>& cand, int zfull) {
    o->tuned = true;
    const TuneCand rule{o->tile, o->zlen};
    if (rule.z < zfull || cand.size() < 2) return SPFM_OK;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return fail(SPFM_E_HIP, "hipEventCreate"); }
    // One sample of candidate ci: nw untimed launches, then n timed ones.
    auto sample = [&](size_t ci, int nw, int n, float& ms) -> spfm_status {
        const spfm_status s2 = set_schedule(o, cand[ci].tile, cand[ci].z);   // zlen also steers the temporal kernel
        if (s2 != SPFM_OK) return s2;
        hipError_t e = hipSuccess;
        for (int i = 0; i < nw + n && e == hipSuccess; ++i) {
            if (i == nw) e = hipEventRecord(e0, o->stream);
            if (e == hipSuccess) e = o->launch_unit(o->cur);
        }
        if (e == hipSuccess) e = hipEventRecord(e1, o->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        return e == hipSuccess ? SPFM_OK : fail(SPFM_E_HIP, "autotune: %s", hipGetErrorString(e));
    };
    std::vector<float> best(cand.size(), 1e30f);
    spfm_status st = SPFM_OK;
    // Sweep 0 is untimed (it warms clocks and caches) and sets nt from the
    // untuned pair's time, so that a sample spans about 1.5 ms (5 to 64
    // launches: short launches alone are timed mostly by their issue jitter).
    // Sweeps 1-3 give each candidate nt untimed launches, so that the clocks
    // settle to its own load, then nt timed ones; odd sweeps run the list
    // backwards, so a candidate does not always follow the same one.  The best
    // of the timed sweeps counts.
    int nt = 5;
    const size_t nc = cand.size();
    for (int sweep = 0; sweep < 4 && st == SPFM_OK; ++sweep) {
        for (size_t j = 0; j < nc && st == SPFM_OK; ++j) {
            const size_t ci = (sweep & 1) ? nc - 1 - j : j;
            float ms = 0.0f;
            st = sample(ci, sweep == 0 ? 2 : nt, nt, ms);
            if (st != SPFM_OK) break;
            if (sweep > 0) best[ci] = std::min(best[ci], ms);
            else if (ci == 0 && ms > 0.0f) nt = std::min(64, std::max(5, (int)std::ceil(1.5f * nt / ms)));
        }
    }
    // The three fastest other pairs and the untuned one (cand[0]) then run four
    // rounds, each in a rotated order, every sample again after as many
    // untimed launches; the fastest total replaces the untuned pair only if it
    // is at least 1% lower.  Single samples of pairs within a few percent of
    // each other rank them only roughly: the clocks drift, and the order of the
    // sweeps shifts a sample by about a percent.
    std::vector<size_t> fin{0};
    {
        std::vector<size_t> order;
        for (size_t ci = 1; ci < nc; ++ci) order.push_back(ci);
        std::sort(order.begin(), order.end(), [&](size_t a, size_t b) { return best[a] < best[b]; });
        for (size_t j = 0; j < order.size() && j < 3; ++j) fin.push_back(order[j]);
    }
    std::vector<double> tot(fin.size(), 0.0);
    for (int round = 0; round < 4 && st == SPFM_OK; ++round) {
        for (size_t j = 0; j < fin.size() && st == SPFM_OK; ++j) {
            const size_t f = (j + (size_t)round) % fin.size();
            float ms = 0.0f;
            st = sample(fin[f], nt, nt, ms);
            tot[f] += ms;
        }
    }
    size_t bi = 0, wf = 1;
    for (size_t f = 2; f < fin.size(); ++f)
        if (tot[f] < tot[wf]) wf = f;
    if (tot[wf] <= 0.99 * tot[0]) bi = fin[wf];
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != SPFM_OK) {
        (void)set_schedule(o, rule.tile, rule.z);
        return st;
    }
    return set_schedule(o, cand[bi].tile, cand[bi].z);
}

// Candidate pairs: every compiled tile shape (when the shape is tuned) with
// every chunk length up to twice the deepest grid (when the length is tuned);
// the untuned pair first.
std::vector<TuneCand> tune_candidates(int tile, int zlen, bool tune_tile, bool tune_z, bool f32, int C,
                                      bool walled, const int* zs, int nzs, int depth) {
    std::vector<TuneCand> out{TuneCand{tile, zlen}};
    for (int t = 0; t < kNumTileShapes; ++t) {
        if (!(t == tile || (tune_tile && tile_compiled(f32, C, walled, t)))) continue;
        for (int i = 0; i < nzs; ++i) {
            const int z = zs[i];
            if (!(z == zlen || tune_z) || (i > 0 && z > 2 * depth)) continue;
            if (t == tile && z == zlen) continue;
            out.push_back(TuneCand{t, z});
        }
    }
    return out;
}

spfm_status autotune(spfm_ctx* c) {
    c->tuned = true;
    if (c->r.kernel != SPFM_KERNEL_TILED) return SPFM_OK;
    static const int zs[4] = {8, 16, 32, 64};
    const bool f32 = c->r.dtype == SPFM_F32;
    const int C = kernel_coupling(c->r.p.coupling, c->r.p.interp);
    // fused steps (tsteps > 1) run the temporal kernel's own tile; only its chunk is timed
    const bool tt = c->tune_tile && c->r.tsteps == 1;
    return tune_schedule(c, tune_candidates(c->tile, c->zlen, tt, c->tune_z, f32, C, c->r.walls != 0, zs, 4,
                                            c->r.p.nz),
                         c->r.tsteps > 1 ? 2 * kTileZ : kTileZ);
}

// Batches: chunks from 4 planes are timed (the size rule goes down to 2 for
// batches far too small to fill the GPU, where the tuner keeps the rule's length).
spfm_status autotune(spfm_batch* b) {
    static const int zs[5] = {4, 8, 16, 32, 64};
    int nz = 1;
    for (const GridDims& d : b->dims) nz = std::max(nz, d.nz);
    return tune_schedule(b, tune_candidates(b->tile, b->zlen, b->tune_tile, b->tune_z, true, b->coupling,
                                            b->walls != 0, zs, 5, nz),
                         kTileZ);
}

template <typename Obj>
spfm_status run_steps(Obj* o, int64_t n) {
    if (n < 0) return fail(SPFM_E_INVAL, "negative step count");
    int64_t left = n;
    const int u = o->unit();   // steps per unit launch
    const int64_t per_graph = (int64_t)kGraphSteps * u;
    if (o->stream != nullptr && n >= 2 * per_graph) {
        for (int from = 0; from < 2; ++from) {
            if (o->graphs.exec[from]) continue;
            hipGraph_t g = nullptr;
            HIP_TRY(hipStreamBeginCapture(o->stream, hipStreamCaptureModeRelaxed));
            hipError_t le = hipSuccess;
            for (int s = 0; s < kGraphSteps && le == hipSuccess; ++s) le = o->launch_unit((from + s) & 1);
            hipError_t ce = hipStreamEndCapture(o->stream, &g);
            if (le != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return fail(SPFM_E_HIP, "step launch during capture: %s", hipGetErrorString(le));
            }
            if (ce != hipSuccess) return fail(SPFM_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(ce));
            hipError_t ie = hipGraphInstantiate(&o->graphs.exec[from], g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ie != hipSuccess) {
                o->graphs.exec[from] = nullptr;
                return fail(SPFM_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ie));
            }
        }
        while (left >= per_graph) {
            HIP_TRY(hipGraphLaunch(o->graphs.exec[o->cur], o->stream));
            left -= per_graph;   // kGraphSteps launches (even): the current buffer is unchanged
            o->nsteps += per_graph;
        }
    }
    // Remaining steps: whole units, then single steps.
    for (; left > 0; left -= (left >= u ? u : 1)) {
        const bool whole = left >= u;
        hipError_t e = whole ? o->launch_unit(o->cur) : o->launch_one(o->cur);
        if (e != hipSuccess) return fail(SPFM_E_HIP, "step launch: %s", hipGetErrorString(e));
        o->cur ^= 1;
        o->nsteps += whole ? u : 1;
    }
    return SPFM_OK;
}

// Resident kernel on whole grids: n steps in launches of at most
// resident_chunk() steps each; a launch of an odd count writes the other
// buffer, of an even count (in place) the same one.
constexpr int64_t kResidentAutoCells = 4096;   // largest stored grid AUTO steps resident untuned
template <typename Obj>
spfm_status run_resident(Obj* o, int64_t n) {
    if (n < 0) return fail(SPFM_E_INVAL, "negative step count");
    while (n > 0) {
        const int chunk = (int)std::min<int64_t>(n, o->resident_chunk());
        const int to = ((chunk & 1) || !o->resident_in_place()) ? 1 - o->cur : o->cur;
        const hipError_t e = o->launch_resident(o->cur, to, chunk);
        if (e != hipSuccess) return fail(SPFM_E_HIP, "resident step launch: %s", hipGetErrorString(e));
        o->cur = to;
        o->nsteps += chunk;
        n -= chunk;
    }
    return SPFM_OK;
}

// Resident segments: every grid's x axis cut into pieces of seg_len stored
// columns (on a walled axis its interior, the ghost columns joining the end
// pieces), each held with `halo` more columns on its open sides.  A grid whose
// middle piece with its halos would span the grid stays whole.  Returns the
// largest region in points.
int64_t resident_items(const std::vector<GridDims>& dims, int walls, int seg_len, int halo,
                       std::vector<ResItem>& out) {
    out.clear();
    int64_t cells = 0;
    const int wx = walls & 1;
    for (int g = 0; g < (int)dims.size(); ++g) {
        const GridDims& d = dims[g];
        const int xa = wx, xb = d.nx - wx;
        const int64_t col = (int64_t)d.ny * d.nz;
        if (seg_len <= 0 || (int64_t)seg_len + 2 * (int64_t)halo >= xb - xa) {
            out.push_back(ResItem{g, 0, d.nx, 0, d.nx});
            cells = std::max(cells, d.nx * col);
            continue;
        }
        for (int s0 = xa; s0 < xb; s0 += seg_len) {
            int ox = s0, oe = std::min(s0 + seg_len, xb);
            if (wx && s0 == xa) ox = 0;
            if (wx && oe == xb) oe = d.nx;
            int rx0 = ox - halo, re = oe + halo;
            if (wx) {
                rx0 = std::max(rx0, 0);
                re = std::min(re, d.nx);
            }
            out.push_back(ResItem{g, rx0, re - rx0, ox, oe - ox});
            cells = std::max(cells, (int64_t)(re - rx0) * col);
        }
    }
    return cells;
}

// Uploads the segments of (seg_len, halo) for the resident kernel of a batch
// (seg_len 0: whole grids), after the stream has drained.
spfm_status set_resident_segments(spfm_batch* b, int seg_len, int halo) {
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->graphs.clear();   // captured launches of the previous configuration
    if (seg_len <= 0) {
        b->seg_len = b->seg_halo = b->nres = b->res_cells = 0;
        return SPFM_OK;
    }
    std::vector<ResItem> items;
    const int64_t cells = resident_items(b->dims, b->walls, seg_len, halo, items);
    if (cells > resident_max_cells((int)sizeof(float)))
        return fail(SPFM_E_INVAL, "a segment holds more than %d points", resident_max_cells((int)sizeof(float)));
    if (items.size() > b->res_cap) {
        if (b->d_res) (void)hipFree(b->d_res);
        b->d_res = nullptr;
        b->res_cap = 0;
        if (hipMalloc(&b->d_res, items.size() * sizeof(ResItem)) != hipSuccess) {
            (void)hipGetLastError();
            b->d_res = nullptr;
            return fail(SPFM_E_NOMEM, "device allocation of the resident segments failed");
        }
        b->res_cap = items.size();
    }
    HIP_TRY(hipMemcpyAsync(b->d_res, items.data(), items.size() * sizeof(ResItem), hipMemcpyHostToDevice,
                           b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->seg_len = seg_len;
    b->seg_halo = halo;
    b->nres = (int)items.size();
    b->res_cells = (int)cells;
    return SPFM_OK;
}

// SPFM_KERNEL_AUTO on a batch whose grids fit the resident kernel: at the
// first step, time the tiled kernel (its untuned schedule), whole grids, and x
// segments of 4 to 64 columns with halos of 4 to 32 (those that cut some grid),
// each over about 64 steps read from the current buffer and written to the
// other one (the field does not change); keep the fastest, or the size rule's
// choice (whole grids up to kResidentAutoCells stored points, else tiled)
// unless another is at least 2% faster.  Two sweeps, the first untimed.
spfm_status autotune_resident(spfm_batch* b) {
    b->res_tuned = true;
    struct Cand {
        bool res;
        int seg, halo;
    };
    std::vector<Cand> cand{Cand{b->resident, 0, 0}, Cand{!b->resident, 0, 0}};
    static const int segs[5] = {4, 8, 16, 32, 64}, halos[4] = {4, 8, 16, 32};
    std::vector<ResItem> tmp;
    for (const int sl : segs)
        for (const int h : halos) {
            const int64_t cells = resident_items(b->dims, b->walls, sl, h, tmp);
            if (tmp.size() > (size_t)b->n && cells <= resident_max_cells((int)sizeof(float)))
                cand.push_back(Cand{true, sl, h});
        }
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return fail(SPFM_E_HIP, "hipEventCreate"); }
    std::vector<float> best(cand.size(), 1e30f);
    spfm_status st = SPFM_OK;
    for (int sweep = 0; sweep < 2 && st == SPFM_OK; ++sweep) {
        for (size_t ci = 0; ci < cand.size() && st == SPFM_OK; ++ci) {
            const Cand& c = cand[ci];
            b->resident = c.res;
            st = set_resident_segments(b, c.seg, c.halo);
            if (st != SPFM_OK) break;
            // steps per launch and launches: about 64 steps
            const int spl = !c.res ? 1 : (c.seg > 0 ? c.halo : 16);
            const int nl = std::max(1, 64 / spl);
            hipError_t e = hipSuccess;
            auto launch = [&]() {
                return c.res ? b->launch_resident(b->cur, 1 - b->cur, spl) : b->launch_one(b->cur);
            };
            e = launch();
            if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
            for (int i = 0; i < nl && e == hipSuccess; ++i) e = launch();
            if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) { st = fail(SPFM_E_HIP, "resident autotune: %s", hipGetErrorString(e)); break; }
            if (sweep > 0) best[ci] = std::min(best[ci], ms / (float)(nl * spl));
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    size_t bi = 0;
    for (size_t ci = 1; ci < cand.size(); ++ci)
        if (best[ci] < best[bi]) bi = ci;
    if (best[0] <= 1.02f * best[bi]) bi = 0;
    if (st != SPFM_OK) bi = 0;
    b->resident = cand[bi].res;
    const spfm_status st2 = set_resident_segments(b, cand[bi].seg, cand[bi].halo);
    return st != SPFM_OK ? st : st2;
}

spfm_status copy_in(void* dst, const void* src, size_t bytes, int src_on_device, hipStream_t s) {
    if (!src) return fail(SPFM_E_INVAL, "source is NULL");
    HIP_TRY(hipMemcpyAsync(dst, src, bytes, src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    if (!src_on_device) HIP_TRY(hipStreamSynchronize(s));
    return SPFM_OK;
}

spfm_status copy_out(void* dst, const void* src, size_t bytes, int dst_on_device, hipStream_t s) {
    if (!dst) return fail(SPFM_E_INVAL, "destination is NULL");
    HIP_TRY(hipMemcpyAsync(dst, src, bytes, dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    if (!dst_on_device) HIP_TRY(hipStreamSynchronize(s));
    return SPFM_OK;
}

spfm_status check_spheres(int32_t n, const double* centers, const double* radii) {
    if (n < 0 || (n > 0 && (!centers || !radii))) return fail(SPFM_E_INVAL, "bad sphere list");
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < 4; ++a)
            if (!std::isfinite(a < 3 ? centers[3 * i + a] : radii[i]))
                return fail(SPFM_E_INVAL, "non-finite sphere %d", i);
    return SPFM_OK;
}

// The field of n spheres from the device table d_sph (4 doubles per sphere),
// enqueued on the context stream; synchronises before returning, so the table
// may be reused afterwards.
spfm_status init_spheres_from(spfm_ctx* c, int32_t n, const double* d_sph) {
    const Params& p = c->r.p;
    void* dst = c->r.walls ? c->buf[1 - c->cur] : c->buf[c->cur];
    hipError_t e = c->r.dtype == SPFM_F64
                       ? launch_init_spheres<double>((double*)dst, p.nx, p.ny, p.nz, p.dx, p.lambda, n,
                                                     d_sph, c->stream)
                       : launch_init_spheres<float>((float*)dst, p.nx, p.ny, p.nz, p.dx, p.lambda, n,
                                                    d_sph, c->stream);
    if (e == hipSuccess && c->r.walls) e = c->to_interior(c->buf[c->cur], dst);
    const hipError_t se = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(SPFM_E_HIP, "sphere init: %s", hipGetErrorString(e));
    if (se != hipSuccess) return fail(SPFM_E_HIP, "sphere init sync: %s", hipGetErrorString(se));
    c->nsteps = 0;
    c->track.reset(n == 1 ? 2 : 0, 0.0);
    return SPFM_OK;
}

}  // namespace

extern "C" {

spfm_status spfm_create(const spfm_grid* grid, double lambda, double Gamma, double M, double mu,
                        int stencil, const spfm_options* opt, spfm_ctx** out) {
    if (!out) return fail(SPFM_E_INVAL, "out is NULL");
    *out = nullptr;
    Resolved r;
    spfm_status st = resolve(grid, lambda, Gamma, M, mu, stencil, opt, &r);
    if (st != SPFM_OK) return st;
    spfm_ctx* c = new (std::nothrow) spfm_ctx;
    if (!c) return fail(SPFM_E_NOMEM, "host allocation failed");
    c->r = r;
    if (r.seg_len > 0) {
        delete c;
        return fail(SPFM_E_INVAL, "segment is an option of batches");
    }
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(SPFM_E_HIP, "hipGetDevice failed");
    }
    c->stream = opt ? (hipStream_t)opt->stream : nullptr;
    const bool autok = !opt || opt->kernel == SPFM_KERNEL_AUTO;
    // constant volume: no timing (it would time the separate correction
    // launches, not the fused steps); the size rule keeps at least 4 planes per
    // chunk, since every fused block adds the previous step's sums of all
    // work items (60^3: 4 planes 10.5 us per step, 2 planes 11.2, 8 planes 12.3)
    c->tune_z = autok && !(opt && opt->zchunk > 0) && !r.conserve_volume;
    // constant volume: the untuned tile shape (the step's sums are compiled for it alone)
    c->tune_tile = autok && r.tile < 0 && !r.conserve_volume;
    const bool f32 = r.dtype == SPFM_F32;
    const bool temporal = r.tsteps > 1;
    c->tile = r.tile >= 0 ? r.tile : default_tile(f32, kernel_coupling(r.p.coupling, r.p.interp));
    const int tx = temporal ? 64 : tile_tx(c->tile), ty = temporal ? 8 : tile_ty(c->tile);   // temporal: 64 x 8
    c->zlen = (opt && opt->zchunk > 0)
                  ? opt->zchunk
                  : default_zlen({GridDims{r.sx, r.sy, r.sz}}, tx, ty, !temporal,
                                 temporal ? (int64_t)1 << 20 : (int64_t)1 << 19, 8,
                                 r.conserve_volume ? 4 : 2);
    const size_t bytes = c->stored_bytes();
    if (opt && opt->d_phi[0]) {
        c->buf[0] = opt->d_phi[0];
        c->buf[1] = opt->d_phi[1];
        c->owns = false;
    } else {
        c->owns = true;
        if (hipMalloc(&c->buf[0], bytes) != hipSuccess || hipMalloc(&c->buf[1], bytes) != hipSuccess) {
            (void)hipGetLastError();
            spfm_destroy(c);
            return fail(SPFM_E_NOMEM, "device allocation of 2 x %zu bytes failed", bytes);
        }
        if (hipMemsetAsync(c->buf[0], 0, bytes, c->stream) != hipSuccess) {
            spfm_destroy(c);
            return fail(SPFM_E_HIP, "hipMemsetAsync failed");
        }
    }
    st = c->red.init();
    if (st != SPFM_OK) { spfm_destroy(c); return st; }
    if (hipMalloc(&c->d_scratch, sizeof(double) * spfm_ctx::kScratchDoubles) != hipSuccess) {
        (void)hipGetLastError();
        spfm_destroy(c);
        return fail(SPFM_E_NOMEM, "device allocation of the reduction scratch failed");
    }
    c->refresh_coef();
    if (r.kernel == SPFM_KERNEL_RESIDENT) {
        const size_t cb = r.dtype == SPFM_F64 ? sizeof(StepCoef<double>) : sizeof(StepCoef<float>);
        const int64_t zero = 0;
        if (hipMalloc(&c->d_coef, cb) != hipSuccess || hipMalloc(&c->d_off, sizeof(int64_t)) != hipSuccess) {
            (void)hipGetLastError();
            spfm_destroy(c);
            return fail(SPFM_E_NOMEM, "device allocation of the resident step tables failed");
        }
        if (hipMemcpy(c->d_off, &zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess) {
            spfm_destroy(c);
            return fail(SPFM_E_HIP, "upload of the resident step tables failed");
        }
    }
    if (r.walls && (r.kernel == SPFM_KERNEL_TILED || r.kernel == SPFM_KERNEL_RESIDENT)) {
        const bool f64 = r.dtype == SPFM_F64;
        const size_t wb = f64 ? sizeof(WallCoef<double>) : sizeof(WallCoef<float>);
        if (hipMalloc(&c->d_wall, wb) != hipSuccess) {
            (void)hipGetLastError();
            c->d_wall = nullptr;
            spfm_destroy(c);
            return fail(SPFM_E_NOMEM, "device allocation of the wall coefficients failed");
        }
        const void* src = f64 ? (const void*)&c->wd : (const void*)&c->wf;
        if (hipMemcpy(c->d_wall, src, wb, hipMemcpyHostToDevice) != hipSuccess) {
            spfm_destroy(c);
            return fail(SPFM_E_HIP, "upload of the wall coefficients failed");
        }
    }
    if (r.kernel == SPFM_KERNEL_TILED) {   // single tiled steps (also the remainder of fused ones)
        st = set_schedule(c, c->tile, c->zlen);
        if (st != SPFM_OK) { spfm_destroy(c); return st; }
    }
    *out = c;
    return SPFM_OK;
}

void spfm_destroy(spfm_ctx* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream); else (void)hipDeviceSynchronize();
    c->graphs.clear();
    c->red.release();
    if (c->d_scratch) (void)hipFree(c->d_scratch);
    if (c->d_items) (void)hipFree(c->d_items);
    if (c->d_cvpart) (void)hipFree(c->d_cvpart);
    for (void* x : c->xbuf)
        if (x) (void)hipFree(x);
    if (c->d_wall) (void)hipFree(c->d_wall);
    if (c->d_coef) (void)hipFree(c->d_coef);
    if (c->d_off) (void)hipFree(c->d_off);
    if (c->owns) {
        if (c->buf[0]) (void)hipFree(c->buf[0]);
        if (c->buf[1]) (void)hipFree(c->buf[1]);
    }
    delete c;
}

spfm_status spfm_set_field(spfm_ctx* c, const void* src, int src_on_device) {
    if (!c) return fail(SPFM_E_INVAL, "ctx is NULL");
    // With walls the grid-shaped input goes through the other buffer into the interior.
    void* dst = c->r.walls ? c->buf[1 - c->cur] : c->buf[c->cur];
    spfm_status st = copy_in(dst, src, c->bytes(), src_on_device, c->stream);
    if (st != SPFM_OK) return st;
    if (c->r.walls) HIP_TRY(c->to_interior(c->buf[c->cur], dst));
    c->nsteps = 0;
    c->track.reset(0, 0.0);
    return SPFM_OK;
}

spfm_status spfm_get_field(spfm_ctx* c, void* dst, int dst_on_device) {
    if (!c) return fail(SPFM_E_INVAL, "ctx is NULL");
    const void* src = nullptr;
    HIP_TRY(c->dense_field(&src));
    return copy_out(dst, src, c->bytes(), dst_on_device, c->stream);
}

spfm_status spfm_field_ptr(spfm_ctx* c, void** d_ptr) {
    if (!c || !d_ptr) return fail(SPFM_E_INVAL, "NULL argument");
    *d_ptr = c->buf[c->cur];
    return SPFM_OK;
}

spfm_status spfm_init_planar(spfm_ctx* c, const int32_t hkl[3], double offset) {
    if (!c || !hkl) return fail(SPFM_E_INVAL, "NULL argument");
    if (hkl[0] == 0 && hkl[1] == 0 && hkl[2] == 0) return fail(SPFM_E_INVAL, "hkl must not be zero");
    if (!std::isfinite(offset)) return fail(SPFM_E_INVAL, "offset must be finite");
    const Params& p = c->r.p;
    const int h[3] = {hkl[0], hkl[1], hkl[2]};
    void* dst = c->r.walls ? c->buf[1 - c->cur] : c->buf[c->cur];
    hipError_t e = c->r.dtype == SPFM_F64
                       ? launch_init_planar<double>((double*)dst, p.nx, p.ny, p.nz, p.dx,
                                                    p.lambda, h, offset, c->stream)
                       : launch_init_planar<float>((float*)dst, p.nx, p.ny, p.nz, p.dx,
                                                   p.lambda, h, offset, c->stream);
    if (e == hipSuccess && c->r.walls) e = c->to_interior(c->buf[c->cur], dst);
    if (e != hipSuccess) return fail(SPFM_E_HIP, "init launch: %s", hipGetErrorString(e));
    c->nsteps = 0;
    c->track.reset(1, slab_area(p.nx, p.ny, p.nz, p.dx, hkl));
    return SPFM_OK;
}

spfm_status spfm_init_spheres(spfm_ctx* c, int32_t n, const double* centers, const double* radii) {
    if (!c) return fail(SPFM_E_INVAL, "ctx is NULL");
    spfm_status st = check_spheres(n, centers, radii);
    if (st != SPFM_OK) return st;
    std::vector<double> h((size_t)std::max(n, 1) * 4, 0.0);
    for (int i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) h[4 * i + a] = centers[3 * i + a];
        h[4 * i + 3] = radii[i];
    }
    double* d = nullptr;
    HIP_TRY(hipMalloc(&d, sizeof(double) * h.size()));
    hipError_t e = hipMemcpyAsync(d, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(d);
        return fail(SPFM_E_HIP, "sphere upload: %s", hipGetErrorString(e));
    }
    st = init_spheres_from(c, n, d);
    (void)hipFree(d);
    return st;
}

spfm_status spfm_init_spheres_noalloc(spfm_ctx* c, int32_t n, const double* centers,
                                      const double* radii) {
    if (!c) return fail(SPFM_E_INVAL, "ctx is NULL");
    spfm_status st = check_spheres(n, centers, radii);
    if (st != SPFM_OK) return st;
    if (n > kMaxScratchSpheres)
        return fail(SPFM_E_INVAL, "at most %d spheres without allocation (got %d)", kMaxScratchSpheres, n);
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != c->device)
        return fail(SPFM_E_STATE, "the context lives on device %d; device %d is current", c->device, dev);
    double* d = nullptr;
    HIP_TRY(sphere_scratch(&d));
    if (n > 0) {
        // pack (x, y, z) and R of each sphere into rows of 4 doubles, straight
        // from the caller's arrays
        HIP_TRY(hipMemcpy2DAsync(d, 4 * sizeof(double), centers, 3 * sizeof(double), 3 * sizeof(double),
                                 (size_t)n, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipMemcpy2DAsync(d + 3, 4 * sizeof(double), radii, sizeof(double), sizeof(double),
                                 (size_t)n, hipMemcpyHostToDevice, c->stream));
    }
    return init_spheres_from(c, n, d);
}

spfm_status spfm_init_front(spfm_ctx* c, const double n[3], double offset) {
    if (!c || !n) return fail(SPFM_E_INVAL, "NULL argument");
    const double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    if (!(nn > 0.0) || !std::isfinite(nn)) return fail(SPFM_E_INVAL, "n must be finite and nonzero");
    if (!std::isfinite(offset)) return fail(SPFM_E_INVAL, "offset must be finite");
    for (int d = 0; d < 3; ++d)
        if (n[d] != 0.0 && !((c->r.walls >> d) & 1))
            return fail(SPFM_E_INVAL, "a front varying along axis %d needs walls on that axis", d);
    const Params& p = c->r.p;
    void* dst = c->r.walls ? c->buf[1 - c->cur] : c->buf[c->cur];
    hipError_t e = c->r.dtype == SPFM_F64
                       ? launch_init_front<double>((double*)dst, p.nx, p.ny, p.nz, p.dx, p.lambda,
                                                   n, offset, c->stream)
                       : launch_init_front<float>((float*)dst, p.nx, p.ny, p.nz, p.dx, p.lambda, n,
                                                  offset, c->stream);
    if (e == hipSuccess && c->r.walls) e = c->to_interior(c->buf[c->cur], dst);
    if (e != hipSuccess) return fail(SPFM_E_HIP, "front init: %s", hipGetErrorString(e));
    // Position along n: the phase volume change over the front's area.
    c->nsteps = 0;
    c->track.reset(1, front_area(p, n));
    return SPFM_OK;
}

spfm_status spfm_init_box(spfm_ctx* c, const double lo[3], const double hi[3]) {
    if (!c || !lo || !hi) return fail(SPFM_E_INVAL, "NULL argument");
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(lo[d]) || !std::isfinite(hi[d]) || !(hi[d] > lo[d]))
            return fail(SPFM_E_INVAL, "box must have finite lo < hi");
    const Params& p = c->r.p;
    void* dst = c->r.walls ? c->buf[1 - c->cur] : c->buf[c->cur];
    hipError_t e = c->r.dtype == SPFM_F64
                       ? launch_init_box<double>((double*)dst, p.nx, p.ny, p.nz, p.dx, p.lambda, lo, hi,
                                                 c->stream)
                       : launch_init_box<float>((float*)dst, p.nx, p.ny, p.nz, p.dx, p.lambda, lo, hi,
                                                c->stream);
    if (e == hipSuccess && c->r.walls) e = c->to_interior(c->buf[c->cur], dst);
    if (e != hipSuccess) return fail(SPFM_E_HIP, "box init: %s", hipGetErrorString(e));
    c->nsteps = 0;
    c->track.reset(0, 0.0);
    return SPFM_OK;
}

spfm_status spfm_contour_stats(spfm_ctx* c, spfm_contour* out) {
    if (!c || !out) return fail(SPFM_E_INVAL, "NULL argument");
    if (c->r.walls) return fail(SPFM_E_STATE, "contour statistics need a periodic grid");
    const Params& p = c->r.p;
    hipError_t e = c->r.dtype == SPFM_F64
                       ? launch_contour_stats<double>((const double*)c->buf[c->cur], p.nx, p.ny, p.nz,
                                                      c->d_part(), c->d_contour(), c->stream)
                       : launch_contour_stats<float>((const float*)c->buf[c->cur], p.nx, p.ny, p.nz,
                                                     c->d_part(), c->d_contour(), c->stream);
    if (e != hipSuccess) return fail(SPFM_E_HIP, "contour statistics: %s", hipGetErrorString(e));
    double h[7];
    HIP_TRY(hipMemcpyAsync(h, c->d_contour(), sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int k = 0; k < 3; ++k) out->centre[k] = h[k] * p.dx;
    out->points = (int64_t)h[3];
    out->R_mean = h[3] > 0.0 ? h[4] / h[3] * p.dx : NAN;
    out->R_min = h[3] > 0.0 ? h[5] * p.dx : NAN;
    out->R_max = h[3] > 0.0 ? h[6] * p.dx : NAN;
    out->eps_eff = h[3] > 0.0 ? (out->R_max - out->R_min) / (2.0 * out->R_mean) : NAN;
    return SPFM_OK;
}

spfm_status spfm_ray_radii(spfm_ctx* c, const double centre[3], int32_t n, const double* dirs,
                           double* radii) {
    if (!c || !centre || !dirs || !radii) return fail(SPFM_E_INVAL, "NULL argument");
    if (n < 1) return fail(SPFM_E_INVAL, "n must be positive");
    if (c->r.walls) return fail(SPFM_E_STATE, "ray radii need a periodic grid");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(centre[k])) return fail(SPFM_E_INVAL, "centre not finite");
    for (int32_t i = 0; i < n; ++i) {
        const double* d = dirs + 3 * (size_t)i;
        const double nn = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (!std::isfinite(nn) || nn == 0.0) return fail(SPFM_E_INVAL, "ray %d: zero or non-finite direction", i);
    }
    const Params& p = c->r.p;
    const double cg[3] = {centre[0] / p.dx, centre[1] / p.dx, centre[2] / p.dx};
    double* d = nullptr;
    if (hipMalloc(&d, sizeof(double) * 4 * (size_t)n) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SPFM_E_NOMEM, "device allocation for %d rays failed", n);
    }
    hipError_t e = hipMemcpyAsync(d, dirs, sizeof(double) * 3 * (size_t)n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = c->r.dtype == SPFM_F64
                ? launch_ray_radii<double>((const double*)c->buf[c->cur], p.nx, p.ny, p.nz, cg, d, n,
                                           d + 3 * (size_t)n, c->stream)
                : launch_ray_radii<float>((const float*)c->buf[c->cur], p.nx, p.ny, p.nz, cg, d, n,
                                          d + 3 * (size_t)n, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(radii, d + 3 * (size_t)n, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost,
                           c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(SPFM_E_HIP, "ray radii: %s", hipGetErrorString(e));
    for (int32_t i = 0; i < n; ++i) radii[i] *= p.dx;
    return SPFM_OK;
}

spfm_status spfm_energy(spfm_ctx* c, int with_mu, double* out) {
    if (!c || !out) return fail(SPFM_E_INVAL, "NULL argument");
    if (c->r.walls) return fail(SPFM_E_STATE, "the energy needs a periodic grid");
    const Params& p = c->r.p;
    const EnergyCoef ec = make_energy_coef(p);
    // partials (2 per block of the energy kernel) and the total in the reduction scratch
    static_assert(2 * 1024 + 1 <= kReduceBlocks * 8, "energy partials fit the scratch");
    double* d_total = c->d_part() + 2 * 1024;
    const hipError_t e = c->r.dtype == SPFM_F64
                             ? launch_energy<double>((const double*)c->buf[c->cur], p.nx, p.ny, p.nz, ec,
                                                     with_mu ? 1 : 0, c->d_part(), d_total, c->stream)
                             : launch_energy<float>((const float*)c->buf[c->cur], p.nx, p.ny, p.nz, ec,
                                                    with_mu ? 1 : 0, c->d_part(), d_total, c->stream);
    if (e != hipSuccess) return fail(SPFM_E_HIP, "energy: %s", hipGetErrorString(e));
    HIP_TRY(hipMemcpyAsync(out, d_total, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SPFM_OK;
}

spfm_status spfm_force(spfm_ctx* c, double* out) {
    if (!c || !out) return fail(SPFM_E_INVAL, "NULL argument");
    const Params& p = c->r.p;
    const int S = p.stencil, C = kernel_coupling(p.coupling, p.interp);
    const bool f64 = c->r.dtype == SPFM_F64;
    void* field = c->buf[c->cur];
    void* dens = c->buf[1 - c->cur];   // dead between steps
    hipError_t e = hipSuccess;
    if (c->r.walls)   // the ghost layers of the current field from Eq. 7
        e = f64 ? launch_fill_walls<double>((double*)field, c->wd, c->nghost, c->stream)
                : launch_fill_walls<float>((float*)field, c->wf, c->nghost, c->stream);
    if (e == hipSuccess)
        e = f64 ? launch_force_density<double>((const double*)field, (double*)dens, c->kd0, c->r.walls, S, C,
                                               c->stream)
                : launch_force_density<float>((const float*)field, (float*)dens, c->kf0, c->r.walls, S, C,
                                              c->stream);
    if (e != hipSuccess) return fail(SPFM_E_HIP, "force: %s", hipGetErrorString(e));
    spfm_status st = c->red.run(dens, c->r.dtype, c->points(), c->stream);
    if (st != SPFM_OK) return st;
    // the density is dt A times the bracket of Eq. 4 summed over directions
    const double A = 2.0 * p.M / (3.0 * p.C_Gamma * p.lambda * p.lambda);
    *out = c->red.h_out->sum_phi / (p.dt * A);
    return SPFM_OK;
}

// Constant volume with the tiled kernel, one launch per step: the first launch
// steps buf[c0] into buf[1 - c0] and forms the sums; every later one applies
// the previous step's correction as it reads its input (CvFuse) and writes
// phi* and that corrected input into the other pair of the four buffers; one
// correction pass ends the call, into the buffer a launch per step would have
// left current.  The fields and mu equal those of the separate step and
// correction launches bit for bit.  The middle launches replay captured
// graphs of kGraphSteps launches (an even count: every graph starts at the
// same pair), one per starting buffer.
spfm_status run_cv_fused(spfm_ctx* c, int64_t n) {
    if (n < 0) return fail(SPFM_E_INVAL, "negative step count");
    if (n == 0) return SPFM_OK;
    const bool f64 = c->r.dtype == SPFM_F64;
    if (!c->xbuf[0]) {
        const size_t bytes = (size_t)c->points() * (f64 ? sizeof(double) : sizeof(float));
        for (void*& x : c->xbuf) {
            if (hipMalloc(&x, bytes) != hipSuccess) {
                (void)hipGetLastError();
                for (void*& y : c->xbuf) {
                    if (y) (void)hipFree(y);
                    y = nullptr;
                }
                return fail(SPFM_E_NOMEM, "device allocation of the constant-volume buffers failed");
            }
        }
    }
    const int c0 = c->cur;
    void* const star[2] = {c->buf[1 - c0], c->xbuf[0]};   // pair 0 (buf[1 - c0], buf[c0]), pair 1
    void* const prev[2] = {c->buf[c0], c->xbuf[1]};
    unsigned long long* const part[2] = {c->d_cvpart, c->d_cvpart + 4 * c->items_cap};
    const int S = c->r.p.stencil, C = kernel_coupling(c->r.p.coupling, c->r.p.interp);
    // launch kk: kk = 0 from buf[c0] into pair 0; kk >= 1 from pair (kk - 1) & 1 into pair kk & 1
    auto launch = [&](int64_t kk) -> hipError_t {
        const int i = (int)((kk + 1) & 1), o = (int)(kk & 1);
        const void* in = kk == 0 ? c->buf[c0] : star[i];
        if (f64) {
            const CvFuse<double> fz{(const double*)prev[i], (double*)prev[o], part[i], c->nitems};
            return launch_step_tiled<double>((const double*)in, (double*)star[o], c->kd0, S, C, c->tile,
                                             c->d_items, c->nitems, nullptr, part[o], kk == 0 ? nullptr : &fz,
                                             c->stream);
        }
        const CvFuse<float> fz{(const float*)prev[i], (float*)prev[o], part[i], c->nitems};
        return launch_step_tiled<float>((const float*)in, (float*)star[o], c->kf0, S, C, c->tile, c->d_items,
                                        c->nitems, nullptr, part[o], kk == 0 ? nullptr : &fz, c->stream);
    };
    hipError_t e = launch(0);
    if (e != hipSuccess) return fail(SPFM_E_HIP, "step launch: %s", hipGetErrorString(e));
    int64_t kk = 1;
    GraphCache& gc = c->graphs;
    if (c->stream != nullptr && n - 1 >= 2 * (int64_t)kGraphSteps) {
        hipGraphExec_t& ex = gc.exec[2 + c0];
        if (!ex) {
            hipGraph_t g = nullptr;
            HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
            hipError_t le = hipSuccess;
            for (int s = 0; s < kGraphSteps && le == hipSuccess; ++s) le = launch(1 + s);
            const hipError_t ce = hipStreamEndCapture(c->stream, &g);
            if (le != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return fail(SPFM_E_HIP, "step launch during capture: %s", hipGetErrorString(le));
            }
            if (ce != hipSuccess) return fail(SPFM_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(ce));
            const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ie != hipSuccess) {
                ex = nullptr;
                return fail(SPFM_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ie));
            }
        }
        for (; n - kk >= kGraphSteps; kk += kGraphSteps) HIP_TRY(hipGraphLaunch(ex, c->stream));
    }
    for (; kk < n; ++kk) {
        e = launch(kk);
        if (e != hipSuccess) return fail(SPFM_E_HIP, "step launch: %s", hipGetErrorString(e));
    }
    const int o = (int)((n - 1) & 1);
    void* const dst = c->buf[c0 ^ (int)(n & 1)];
    const double dt_beta = c->r.p.dt * 2.0 * c->r.p.M / (3.0 * c->r.p.lambda * c->r.p.Gamma);
    unsigned long long* const total = c->d_cvpart + 8 * c->items_cap;
    e = f64 ? launch_cv_apply<double>((const double*)prev[o], (double*)star[o], c->points(), c->r.p.interp,
                                      dt_beta, part[o], c->nitems, total, c->d_state(), c->stream,
                                      (double*)dst)
            : launch_cv_apply<float>((const float*)prev[o], (float*)star[o], c->points(), c->r.p.interp,
                                     dt_beta, part[o], c->nitems, total, c->d_state(), c->stream, (float*)dst);
    if (e != hipSuccess) return fail(SPFM_E_HIP, "constant-volume correction: %s", hipGetErrorString(e));
    c->cur = c0 ^ (int)(n & 1);
    c->nsteps += n;
    return SPFM_OK;
}

spfm_status spfm_set_mu(spfm_ctx* c, double mu) {
    if (!c) return fail(SPFM_E_INVAL, "ctx is NULL");
    if (!std::isfinite(mu)) return fail(SPFM_E_INVAL, "mu must be finite");
    Params p = c->r.p;
    p.mu = mu;
    const double dtm = stable_dt(p.stencil, p.coupling, p.u, p.gamma, p.lambda, p.Gamma, p.M, mu, p.dx,
                                 p.C_Gamma, p.interp);
    if (!c->r.allow_unstable && p.dt > dtm)
        return fail(SPFM_E_UNSTABLE, "dt = %g exceeds the explicit stability bound %g", p.dt, dtm);
    // Enqueued steps (and replays of the cached graphs, which hold the old
    // coefficients) finish first: the graphs are destroyed below.
    HIP_TRY(c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize());
    c->r.p = p;
    c->r.dt_max = dtm;
    c->refresh_coef();
    return SPFM_OK;
}

spfm_status spfm_step(spfm_ctx* c, int64_t n) {
    if (!c) return fail(SPFM_E_INVAL, "ctx is NULL");
    if (c->r.kernel == SPFM_KERNEL_RESIDENT) return run_resident(c, n);
    if (n > 0 && (c->tune_z || c->tune_tile) && !c->tuned) {
        spfm_status st = autotune(c);
        if (st != SPFM_OK) return st;
        c->graphs.clear();
    }
    if (c->r.conserve_volume && c->r.kernel != SPFM_KERNEL_PLAIN && c->nitems <= kCvDirectParts)
        return run_cv_fused(c, n);
    return run_steps(c, n);
}

spfm_status spfm_diagnostics(spfm_ctx* c, spfm_diag* out) {
    if (!c || !out) return fail(SPFM_E_INVAL, "NULL argument");
    const void* field = nullptr;
    HIP_TRY(c->dense_field(&field));
    spfm_status st = c->red.run(field, c->r.dtype, c->points(), c->stream);
    if (st != SPFM_OK) return st;
    c->track.fill(out, *c->red.h_out, c->r.p.dx, c->r.p.lambda, c->nsteps, c->r.p.dt);
    out->mu = c->r.p.mu;
    if (c->r.conserve_volume) {
        if (c->nsteps == 0) {
            out->mu = NAN;   // no step taken yet
        } else {
            HIP_TRY(hipMemcpyAsync(&out->mu, c->d_state() + 1, sizeof(double), hipMemcpyDeviceToHost,
                                   c->stream));
            HIP_TRY(hipStreamSynchronize(c->stream));
        }
    }
    if (out->diverged) return fail(SPFM_E_DIVERGED, "%d points are non-finite or |phi| > 2", out->diverged);
    return SPFM_OK;
}

spfm_status spfm_get_info(const spfm_ctx* c, spfm_info* o) {
    if (!c || !o) return fail(SPFM_E_INVAL, "NULL argument");
    const Params& p = c->r.p;
    o->lambda = p.lambda; o->Gamma = p.Gamma; o->M = p.M; o->mu = p.mu; o->dt = p.dt; o->dx = p.dx;
    o->C_Gamma = p.C_Gamma; o->eps = p.eps; o->tau = p.tau;
    for (int i = 0; i < 3; ++i) o->gamma[i] = p.gamma[i];
    o->dt_max = c->r.dt_max;
    o->stencil = p.stencil; o->coupling = p.coupling; o->dtype = c->r.dtype; o->kernel = c->r.kernel;
    o->zchunk = c->zlen;
    o->tile_x = c->r.kernel == SPFM_KERNEL_TILED ? tile_tx(c->tile) : 0;
    o->tile_y = c->r.kernel == SPFM_KERNEL_TILED ? tile_ty(c->tile) : 0;
    o->tsteps = c->r.tsteps;
    o->walls = c->r.walls;
    o->interp = c->r.p.interp;
    o->conserve_volume = c->r.conserve_volume;
    return SPFM_OK;
}

// ---------------------------------------------------------------- batch ----

void spfm_batch_destroy(spfm_batch* b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream); else (void)hipDeviceSynchronize();
    b->graphs.clear();
    b->red.release();
    if (b->buf[0]) (void)hipFree(b->buf[0]);
    if (b->buf[1]) (void)hipFree(b->buf[1]);
    if (b->d_coef) (void)hipFree(b->d_coef);
    if (b->d_offset) (void)hipFree(b->d_offset);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_res) (void)hipFree(b->d_res);
    if (b->d_wall) (void)hipFree(b->d_wall);
    delete b;
}

spfm_status spfm_batch_create(int32_t n, const spfm_grid* grids, const double* lambda,
                              const double* Gamma, const double* M, const double* mu, int stencil,
                              const spfm_options* opt, spfm_batch** out) {
    if (!out) return fail(SPFM_E_INVAL, "out is NULL");
    *out = nullptr;
    if (n <= 0 || !grids || !lambda || !Gamma || !M || !mu) return fail(SPFM_E_INVAL, "bad batch arrays");
    spfm_options o;
    if (opt) o = *opt; else std::memset(&o, 0, sizeof o);
    if (o.dtype != SPFM_F32) return fail(SPFM_E_INVAL, "batches run in F32");
    if (o.d_phi[0] || o.d_phi[1]) return fail(SPFM_E_INVAL, "batches allocate their own buffers");
    if (o.C_Gamma > 0.0) return fail(SPFM_E_INVAL, "batches calibrate C_Gamma per grid");
    if (o.kernel == SPFM_KERNEL_PLAIN) return fail(SPFM_E_INVAL, "batches use the tiled or resident kernel");
    if (o.tsteps > 1) return fail(SPFM_E_INVAL, "batches step one step per launch (tsteps <= 1)");
    if (o.conserve_volume) return fail(SPFM_E_INVAL, "batches keep mu fixed (conserve_volume = 0)");
    spfm_batch* b = new (std::nothrow) spfm_batch;
    if (!b) return fail(SPFM_E_NOMEM, "host allocation failed");
    b->n = n;
    b->stencil = stencil;
    b->coupling = kernel_coupling(o.coupling, o.interp);
    b->stream = (hipStream_t)o.stream;
    b->walls = o.walls;
    b->r.resize(n);
    b->track.resize(n);
    b->offset.resize(n);
    std::vector<StepCoef<float>> coef(n);
    std::vector<WallCoef<float>> wall(o.walls ? n : 0);
    std::vector<GridDims> dims(n);
    int64_t off = 0;
    for (int i = 0; i < n; ++i) {
        spfm_options oi = o;   // per-grid wall angles, when given
        if (o.walls && o.batch_wall_sin)
            for (int f = 0; f < 6; ++f) oi.wall_sin[f] = o.batch_wall_sin[6 * i + f];
        spfm_status st = resolve(&grids[i], lambda[i], Gamma[i], M[i], mu[i], stencil, &oi, &b->r[i]);
        if (st != SPFM_OK) {
            spfm_batch_destroy(b);
            char tmp[512];
            std::snprintf(tmp, sizeof tmp, "grid %d: %s", i, g_err);
            std::snprintf(g_err, sizeof g_err, "%s", tmp);
            return st;
        }
        const Resolved& ri = b->r[i];
        const Params& p = ri.p;
        coef[i] = make_coef<float>(p);
        coef[i].nx = ri.sx;   // the kernels sweep the stored grid
        coef[i].ny = ri.sy;
        coef[i].nz = ri.sz;
        b->offset[i] = off;
        b->points += (int64_t)p.nx * p.ny * p.nz;
        const int64_t ns = (int64_t)ri.sx * ri.sy * ri.sz;
        off += (ns + 63) / 64 * 64;   // keep every grid 256-byte aligned
        dims[i] = GridDims{ri.sx, ri.sy, ri.sz};
        if (o.walls) wall[i] = wall_coef<float>(ri);
    }
    b->dims = dims;
    // The resident kernel when every stored grid fits one workgroup's LDS: asked
    // for, or chosen by AUTO (unless a z-chunk for the tiled kernel was given)
    // for grids of at most kResidentAutoCells stored points.  One workgroup runs
    // on one CU, so a step of a larger grid takes longer there than the launch of
    // one tiled step of the whole batch: 7 walled 120 x 10 x 10 TI_n grids (17568
    // stored points each) took 28.5 us per step resident against 7.1 us tiled,
    // 12 periodic 256 x 3 x 3 slabs 1.7 us against 3.2 us.
    int64_t largest = 0;
    for (const GridDims& d : dims) largest = std::max<int64_t>(largest, (int64_t)d.nx * d.ny * d.nz);
    const bool fits = largest <= resident_max_cells((int)sizeof(float));
    b->max_cells = fits ? (int)largest : 0;
    const int seg_asked = b->r[0].seg_len;   // the same options resolve every grid alike
    if ((o.kernel == SPFM_KERNEL_RESIDENT || seg_asked > 0) && !fits) {
        spfm_batch_destroy(b);
        return fail(SPFM_E_INVAL, "the resident kernel holds at most %d stored points per grid",
                    resident_max_cells((int)sizeof(float)));
    }
    const int asked_tile = b->r[0].tile;   // the same options resolve every grid alike
    const bool autok = o.kernel == SPFM_KERNEL_AUTO && o.zchunk <= 0 && asked_tile < 0;
    b->resident = o.kernel == SPFM_KERNEL_RESIDENT || seg_asked > 0 || (autok && largest <= kResidentAutoCells);
    b->tune_res = autok && seg_asked == 0 && fits;
    b->tile = asked_tile >= 0 ? asked_tile : default_tile(true, b->coupling);
    b->tune_z = o.kernel == SPFM_KERNEL_AUTO && o.zchunk <= 0;
    b->tune_tile = o.kernel == SPFM_KERNEL_AUTO && asked_tile < 0;
    const int zb = o.zchunk > 0 ? o.zchunk
                                : default_zlen(dims, tile_tx(b->tile), tile_ty(b->tile), true, (int64_t)1 << 19, 4);
    b->total = off;
    const size_t bytes = (size_t)off * sizeof(float);
    if (hipMalloc(&b->buf[0], bytes) != hipSuccess || hipMalloc(&b->buf[1], bytes) != hipSuccess ||
        hipMalloc(&b->d_coef, sizeof(StepCoef<float>) * n) != hipSuccess ||
        hipMalloc(&b->d_offset, sizeof(int64_t) * n) != hipSuccess ||
        (o.walls && hipMalloc(&b->d_wall, sizeof(WallCoef<float>) * n) != hipSuccess)) {
        (void)hipGetLastError();
        spfm_batch_destroy(b);
        return fail(SPFM_E_NOMEM, "device allocation failed");
    }
    spfm_status st = b->red.init();
    if (st != SPFM_OK) { spfm_batch_destroy(b); return st; }
    if (hipMemcpy(b->d_coef, coef.data(), sizeof(StepCoef<float>) * n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->d_offset, b->offset.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice) != hipSuccess ||
        (o.walls && hipMemcpy(b->d_wall, wall.data(), sizeof(WallCoef<float>) * n,
                              hipMemcpyHostToDevice) != hipSuccess) ||
        hipMemset(b->buf[0], 0, bytes) != hipSuccess || hipMemset(b->buf[1], 0, bytes) != hipSuccess) {
        spfm_batch_destroy(b);
        return fail(SPFM_E_HIP, "batch upload failed");
    }
    st = set_schedule(b, b->tile, zb);
    if (st == SPFM_OK && seg_asked > 0) st = set_resident_segments(b, seg_asked, b->r[0].seg_halo);
    if (st != SPFM_OK) { spfm_batch_destroy(b); return st; }
    *out = b;
    return SPFM_OK;
}

spfm_status spfm_batch_init_planar(spfm_batch* b, const int32_t* hkl, const double* offset) {
    if (!b || !hkl || !offset) return fail(SPFM_E_INVAL, "NULL argument");
    for (int i = 0; i < b->n; ++i) {
        const int32_t* h = hkl + 3 * i;
        if (h[0] == 0 && h[1] == 0 && h[2] == 0) return fail(SPFM_E_INVAL, "grid %d: hkl is zero", i);
        if (!std::isfinite(offset[i])) return fail(SPFM_E_INVAL, "grid %d: offset not finite", i);
    }
    for (int i = 0; i < b->n; ++i) {
        const Params& p = b->r[i].p;
        const int h[3] = {hkl[3 * i], hkl[3 * i + 1], hkl[3 * i + 2]};
        hipError_t e = launch_init_planar<float>(b->dense_target(i), p.nx, p.ny, p.nz, p.dx, p.lambda,
                                                 h, offset[i], b->stream);
        if (e == hipSuccess) e = b->to_grid(i);
        if (e != hipSuccess) return fail(SPFM_E_HIP, "init launch: %s", hipGetErrorString(e));
        b->track[i].reset(1, slab_area(p.nx, p.ny, p.nz, p.dx, hkl + 3 * i));
    }
    b->nsteps = 0;
    return SPFM_OK;
}

spfm_status spfm_batch_init_front(spfm_batch* b, const double* n, const double* offset) {
    if (!b || !n || !offset) return fail(SPFM_E_INVAL, "NULL argument");
    for (int i = 0; i < b->n; ++i) {
        const double* ni = n + 3 * i;
        const double nn = std::sqrt(ni[0] * ni[0] + ni[1] * ni[1] + ni[2] * ni[2]);
        if (!(nn > 0.0) || !std::isfinite(nn))
            return fail(SPFM_E_INVAL, "grid %d: n must be finite and nonzero", i);
        if (!std::isfinite(offset[i])) return fail(SPFM_E_INVAL, "grid %d: offset not finite", i);
        for (int d = 0; d < 3; ++d)
            if (ni[d] != 0.0 && !((b->walls >> d) & 1))
                return fail(SPFM_E_INVAL, "grid %d: a front varying along axis %d needs walls on that axis",
                            i, d);
    }
    for (int i = 0; i < b->n; ++i) {
        const Params& p = b->r[i].p;
        hipError_t e = launch_init_front<float>(b->dense_target(i), p.nx, p.ny, p.nz, p.dx, p.lambda,
                                                n + 3 * i, offset[i], b->stream);
        if (e == hipSuccess) e = b->to_grid(i);
        if (e != hipSuccess) return fail(SPFM_E_HIP, "front init: %s", hipGetErrorString(e));
        b->track[i].reset(1, front_area(p, n + 3 * i));
    }
    b->nsteps = 0;
    return SPFM_OK;
}

spfm_status spfm_batch_set_field(spfm_batch* b, int32_t i, const void* src, int src_on_device) {
    if (!b || i < 0 || i >= b->n) return fail(SPFM_E_INVAL, "bad batch index");
    const Params& p = b->r[i].p;
    const size_t bytes = (size_t)p.nx * p.ny * p.nz * sizeof(float);
    spfm_status st = copy_in(b->dense_target(i), src, bytes, src_on_device, b->stream);
    if (st != SPFM_OK) return st;
    HIP_TRY(b->to_grid(i));
    b->track[i].reset(0, 0.0);
    return SPFM_OK;
}

spfm_status spfm_batch_get_field(spfm_batch* b, int32_t i, void* dst, int dst_on_device) {
    if (!b || i < 0 || i >= b->n) return fail(SPFM_E_INVAL, "bad batch index");
    const Params& p = b->r[i].p;
    const size_t bytes = (size_t)p.nx * p.ny * p.nz * sizeof(float);
    const float* src = nullptr;
    HIP_TRY(b->dense_grid(i, &src));
    return copy_out(dst, src, bytes, dst_on_device, b->stream);
}

spfm_status spfm_batch_step(spfm_batch* b, int64_t n) {
    if (!b) return fail(SPFM_E_INVAL, "batch is NULL");
    if (n > 0 && b->tune_res && !b->res_tuned) {
        const spfm_status st = autotune_resident(b);
        if (st != SPFM_OK) return st;
    }
    if (b->segmented()) return run_steps(b, n);
    if (b->resident) return run_resident(b, n);
    if (n > 0 && (b->tune_z || b->tune_tile) && !b->tuned) {
        spfm_status st = autotune(b);
        if (st != SPFM_OK) return st;
    }
    return run_steps(b, n);
}

spfm_status spfm_batch_diagnostics(spfm_batch* b, spfm_diag* out) {
    if (!b || !out) return fail(SPFM_E_INVAL, "NULL argument");
    int bad = 0;
    for (int i = 0; i < b->n; ++i) {
        const Params& p = b->r[i].p;
        const float* field = nullptr;
        HIP_TRY(b->dense_grid(i, &field));
        spfm_status st = b->red.run(field, SPFM_F32, (int64_t)p.nx * p.ny * p.nz, b->stream);
        if (st != SPFM_OK) return st;
        b->track[i].fill(&out[i], *b->red.h_out, p.dx, p.lambda, b->nsteps, p.dt);
        bad += out[i].diverged;
    }
    if (bad) return fail(SPFM_E_DIVERGED, "%d points are non-finite or |phi| > 2", bad);
    return SPFM_OK;
}

int64_t spfm_batch_points(const spfm_batch* b) { return b ? b->points : 0; }

int32_t spfm_batch_zchunk(const spfm_batch* b) { return b ? b->zlen : 0; }

int32_t spfm_batch_kernel(const spfm_batch* b) {
    return b ? (b->resident ? SPFM_KERNEL_RESIDENT : SPFM_KERNEL_TILED) : -1;
}

spfm_status spfm_batch_get_info(const spfm_batch* b, spfm_batch_info* o) {
    if (!b || !o) return fail(SPFM_E_INVAL, "NULL argument");
    o->kernel = b->resident ? SPFM_KERNEL_RESIDENT : SPFM_KERNEL_TILED;
    o->tile_x = b->resident ? 0 : tile_tx(b->tile);
    o->tile_y = b->resident ? 0 : tile_ty(b->tile);
    o->zchunk = b->resident ? 0 : b->zlen;
    o->grids = b->n;
    o->points = b->points;
    o->segment = b->resident ? b->seg_len : 0;
    o->halo = b->resident ? b->seg_halo : 0;
    return SPFM_OK;
}

double spfm_calibrate_cgamma(double lambda_over_dx, int coupling) {
    return calibrate_cgamma(lambda_over_dx, coupling);
}

double spfm_stable_dt(int stencil, int coupling, const double u[3], const double gamma[3],
                      double lambda, double Gamma, double M, double mu, double dx, double C_Gamma) {
    double g[3];
    if (!gamma || (gamma[0] == 0.0 && gamma[1] == 0.0 && gamma[2] == 0.0)) default_gamma(stencil, g);
    else for (int i = 0; i < 3; ++i) g[i] = gamma[i];
    const double zero[3] = {1.0, 0.0, 0.0};
    if (C_Gamma <= 0.0) C_Gamma = calibrate_cgamma(lambda / dx, coupling);
    return stable_dt(stencil, coupling, u ? u : zero, g, lambda, Gamma, M, mu, dx, C_Gamma);
}

const char* spfm_status_string(spfm_status s) {
    switch (s) {
        case SPFM_OK: return "ok";
        case SPFM_E_INVAL: return "invalid argument";
        case SPFM_E_NOMEM: return "out of memory";
        case SPFM_E_HIP: return "HIP runtime error";
        case SPFM_E_UNSTABLE: return "time step above the explicit stability bound";
        case SPFM_E_DIVERGED: return "field diverged";
        case SPFM_E_STATE: return "invalid state";
    }
    return "unknown status";
}

const char* spfm_last_error(void) { return g_err; }

}  // extern "C"
