/*
 * spfm.h -- C ABI of the MI355X (gfx950) implementation of the explicit time
 * step of the Sharp Phase-Field Method (SPFM) of Fleck, Schleifer & Zimbrod,
 * "Frictionless motion of diffuse interfaces by sharp phase-field modeling"
 * (arXiv:1910.05180).
 *
 * The problem (Sec. 2.1): a phase field phi on a uniform simple-cubic grid of
 * spacing dx evolves by the Allen-Cahn law (Eq. 2)
 *     3 lambda Gamma d_t phi = -2 M delta_phi F
 * where F is the discrete free energy of Eq. 1: forward-difference gradient
 * energy over the 3, 9 or 13 directions of the first one, two or three
 * neighbour shells (Tab. 1; 6-, 18- or 26-neighbour stencils), the
 * translationally invariant equilibrium potential g_k of Eq. 6 with grid
 * coupling parameters a_k = tanh(2 r_k.n / lambda) (Eq. 5), and the driving
 * force mu h3(phi), h3 = phi^2 (3 - 2 phi).  The coupling normal n is either a
 * fixed direction (TI_<hkl> model) or the locally measured interface normal
 * (TI_n model, Tab. 2); the continuum-field model (CF, potential
 * 8 phi^2 (1-phi)^2 / 3 per direction) is available as a control.
 * Time integration is forward Euler; the grid is periodic on every axis that
 * has no walls.  Walls (Sec. 2.2) hold a contact angle by Eq. 7: one ghost
 * layer beyond each walled end takes, before every step, the value of its
 * inward neighbour moved along the ideal profile by dx sin(alpha).
 *
 * Conventions.
 *   Field layout: phi[(z*ny + y)*nx + x], x fastest, dtype float or double.
 *   phi = 1 and phi = 0 are the two phases; the normal points from phi = 1
 *   into phi = 0; mu > 0 favours phi = 0; planar interfaces move with
 *   v = -M mu / Gamma along their normal (Sec. 2.1).
 *   Pointers: "device" pointers are HIP device memory on the current device
 *   (for instance torch.cuda tensors); "host" pointers are ordinary memory.
 *   Ownership: the caller owns every pointer it passes; the library owns the
 *   context and any buffer it allocated itself, and frees them in destroy.
 *   Errors: every call returns an spfm_status; nothing is printed.  A failing
 *   call leaves a description in spfm_last_error() (per host thread).
 *   Streams: every call is ordered on the context's stream.  spfm_step and
 *   the field setters are asynchronous; spfm_diagnostics and spfm_get_field
 *   into host memory synchronise the stream.
 *   Threads: a context must not be used by two host threads at once.
 */
#ifndef SPFM_H
#define SPFM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPFM_OK = 0,
    SPFM_E_INVAL = -1,     /* invalid argument */
    SPFM_E_NOMEM = -2,     /* device or host allocation failed */
    SPFM_E_HIP = -3,       /* a HIP runtime call failed */
    SPFM_E_UNSTABLE = -4,  /* dt above the explicit stability bound */
    SPFM_E_DIVERGED = -5,  /* non-finite values or |phi| > 2 found */
    SPFM_E_STATE = -6      /* call not valid in the current state */
} spfm_status;

typedef enum { SPFM_F32 = 0, SPFM_F64 = 1 } spfm_dtype;

/* Tab. 2 models (all with h3): LOCAL = TI_n, GLOBAL = TI_<hkl> with u,
 * CF = continuum-field potential (no translational invariance). */
typedef enum { SPFM_LOCAL = 0, SPFM_GLOBAL = 1, SPFM_CF = 2 } spfm_coupling;

/* Kernel choice: PLAIN = one thread per point reading its 27 neighbours from
 * global memory; TILED = LDS-staged tiles marching along z; RESIDENT = one
 * workgroup per grid holding the whole stored grid in LDS (two copies: at most
 * 20480 FP32 or 10240 FP64 stored points), or for batches per x segment of a
 * grid with halos (spfm_options.segment), taking many steps per launch with
 * workgroup barriers only (not with conserve_volume or tsteps > 1).
 * AUTO = TILED with the tile shape and z-chunk per block chosen by timing
 * candidates on the current field at the first spfm_step (that call
 * synchronises the stream once); for batches whose stored grids all fit the
 * resident kernel, the first spfm_batch_step also times RESIDENT, whole and in
 * segments, and keeps the fastest.  Results do not depend on the kernel choice
 * among TILED and RESIDENT, nor on the tile, z-chunk or segments: they are
 * equal bit for bit. */
typedef enum {
    SPFM_KERNEL_AUTO = 0,
    SPFM_KERNEL_PLAIN = 1,
    SPFM_KERNEL_TILED = 2,
    SPFM_KERNEL_RESIDENT = 3
} spfm_kernel;

typedef struct {
    int32_t nx, ny, nz; /* grid points per axis: >= 3 on periodic axes, >= 1 on walled axes */
    double dx;          /* grid spacing, > 0 */
} spfm_grid;

/* Options.  An all-zero struct selects every default. */
typedef struct {
    int32_t dtype;      /* spfm_dtype; default SPFM_F32 */
    int32_t coupling;   /* spfm_coupling; default SPFM_LOCAL */
    double u[3];        /* GLOBAL: direction of restored invariance (any length > 0) */
    double dt;          /* time step; <= 0 selects 0.1 dx^2 / (M Gamma) */
    double gamma[3];    /* shell weights gamma_1..3 of Eq. 1; all zero selects
                           (1,0,0), (1/3,2/3,0), (14,12,4)/30 for 6/18/26 neighbours */
    double C_Gamma;     /* energy calibration of Eq. 1; <= 0 selects the value for
                           which the ideal planar [100] profile carries energy Gamma
                           per area (TI), or 2/3 (CF) */
    double eps;         /* floor of phi and 1-phi in the normal estimator; <= 0
                           selects 1e-30 (F32) or 1e-300 (F64) */
    double tau;         /* |grad psi| below tau -> normal (1,0,0); <= 0 selects 1e-3 */
    void *stream;       /* hipStream_t to order work on; NULL = the null stream */
    void *d_phi[2];     /* optional caller-owned device ping-pong buffers of the stored
                           field, (nx+2wx)*(ny+2wy)*(nz+2wz) elements of dtype with wd = 1
                           for a walled axis, else 0; both NULL = library allocates */
    int32_t kernel;     /* spfm_kernel */
    int32_t allow_unstable; /* nonzero: skip the dt stability check */
    int32_t zchunk;     /* planes per block of the tiled kernel, 1..4096; 0 = chosen by the
                           library: a size rule (32 planes, 64 for fused steps, shorter, down
                           to 2 (8 fused, 4 with conserve_volume), for grids too small to fill
                           the GPU); for AUTO on a grid that fills it (not with
                           conserve_volume), timed among 8..64 at the first step.
                           Single steps cut each tile column into blocks of at most zchunk
                           planes, except a tail (about 1.4 rounds of the work the GPU keeps
                           resident, at most 35% of the column) in blocks of halving length
                           down to 8 (4 for zchunk < 16), dispatched last so that the GPU
                           drains evenly; fused
                           steps (tsteps > 1) use zchunk planes throughout */
    int32_t tsteps;     /* temporal blocking: steps fused into one pass over the field, 0 or 1 =
                           none, 2..4 = that many (F32 with kernel AUTO or TILED only).  Results
                           equal tsteps single steps of the TILED kernel bit for bit; spfm_step(n)
                           runs n / tsteps fused launches and n % tsteps single tiled steps, so
                           any n equals n tiled steps */
    int32_t walls;      /* bit d (d = 0, 1, 2 for x, y, z): contact-angle walls at both ends of
                           axis d instead of periodic wrap (not with tsteps > 1) */
    double wall_sin[6]; /* faces -x, +x, -y, +y, -z, +z: sin(alpha) of Eq. 7, in [-1, 1]: a ghost
                           is its inward neighbour moved by dx sin(alpha) along the profile
                           coordinate (towards phi = 0 for > 0).  A planar front of normal n
                           (into phi = 0) is held exactly by sin(alpha) = n . e, e the outward
                           normal of the face.  Unused for unwalled axes */
    int32_t interp;     /* interpolation function h of the driving force mu h(phi) (Tab. 2):
                           0 = h3 = phi^2 (3 - 2 phi) (default; the TI models' choice),
                           1 = h5 = phi^3 (10 - 15 phi + 6 phi^2),
                           2 = h_Abel = phi^2 / (phi^2 + (1 - phi)^2); 1 and 2 only with
                           coupling CF (the comparisons of Sec. 3.1), else SPFM_E_INVAL */
    int32_t conserve_volume; /* nonzero: the homogeneous driving force is chosen at every step so
                           that sum phi stays constant (Sec. 3.3; mu at create only sets the
                           stability check); periodic grids, tsteps <= 1, not in batches.  The
                           sums that fix it are exact (terms rounded to 2^-54, added as
                           integers), so the result does not depend on the kernel's schedule;
                           the tiled kernel forms them in the step itself (the untuned tile
                           shape only).  With at most 1024 work items (zchunk) each step also
                           applies the previous step's correction as it reads its input, and
                           spfm_step(n) ends with one correction launch: n + 1 launches, with
                           the library's buffers plus two more fields allocated at the first
                           step; else a correction launch follows every step.  The plain
                           kernel adds a pass for the sums */
    const double *batch_wall_sin; /* batches with walls: 6 values per grid, wall_sin of grid i at
                           6 i (read at spfm_batch_create only); NULL = wall_sin for every grid.
                           Ignored by single contexts */
    int32_t tile[2];    /* tiled kernel: tile column (x, y) of one block, {0, 0} = chosen by the
                           library: 16 x 8 (F32 TI_n) or 64 x 8 untuned, and with kernel AUTO the
                           fastest compiled shape timed at the first step together with the
                           z-chunk.  Compiled shapes: 16x8, 32x8, 64x8, 16x16, 32x16, 64x16 for
                           F32 without walls and h3; 64x8, 32x8, 16x8 for F64 TI_n; 16x8 (F32
                           TI_n) or 64x8 otherwise; with conserve_volume the untuned shape
                           alone.  Another shape is SPFM_E_INVAL.  Results do not depend on the
                           shape */
    int32_t segment[2]; /* batches, resident kernel: {length, halo} cuts every grid along x into
                           pieces of `length` stored columns, one workgroup each, that hold
                           `halo` more columns on each open side and take at most `halo` steps
                           per launch (the halos are stepped redundantly, so no workgroup waits
                           for another); grids not longer than a piece stay whole.  {0, 0} =
                           whole grids, or with kernel AUTO the fastest of the tiled kernel, whole
                           grids and a set of {length, halo} pairs, timed at the first step.
                           length >= 1 and 1 <= halo <= 4096 when given; SPFM_E_INVAL for
                           single contexts and with kernel TILED.  Results do not depend on it */
} spfm_options;

typedef struct {
    int64_t step;              /* steps taken since the last field set or init */
    double time;               /* step * dt */
    double phase_volume;       /* V1 = dx^3 sum phi (FP64, compensated) */
    double interface_area;     /* (4/lambda) dx^3 sum phi(1-phi) (FP64, compensated) */
    double interface_position; /* planar init: (V1 - V1(0)) / A_slab; single sphere:
                                  radius R with (4pi/3)(R^3 + R pi^2 lambda^2/16) = V1;
                                  otherwise NaN */
    double velocity;           /* change of interface_position per unit time since the
                                  previous spfm_diagnostics call; NaN on the first */
    double phi_min, phi_max;
    double sum_phi, sum_x;     /* the raw sums: sum phi, sum phi(1-phi) */
    int32_t diverged;          /* number of points non-finite or |phi| > 2 */
    double mu;                 /* driving force of the last step: the fixed mu, or with
                                  conserve_volume the value chosen (NaN before the first step) */
} spfm_diag;

/* Parameters the library resolved at create time. */
typedef struct {
    double lambda, Gamma, M, mu, dt, dx, C_Gamma, eps, tau;
    double gamma[3];
    double dt_max;             /* explicit stability bound */
    int32_t stencil, coupling, dtype, kernel;
    int32_t zchunk;            /* leading planes per block of the tiled kernel (chosen by
                                  timing at the first spfm_step when kernel is AUTO) */
    int32_t tsteps;            /* steps per fused launch (1 = no temporal blocking) */
    int32_t walls;             /* walled axes (bit mask) */
    int32_t interp;            /* interpolation function (spfm_options.interp) */
    int32_t conserve_volume;
    int32_t tile_x, tile_y;    /* tile column of the tiled kernel (after tuning); 0 for other kernels */
} spfm_info;

/* Shape of a particle from its phi = 1/2 contour (Sec. 3.3, Eq. 8-10 at
 * l = 1/2): contour points on the grid edges, distances from the barycentre
 * sum phi x / sum phi, eps_eff = (R_max - R_min) / (2 R_mean).  Lengths in
 * units of dx * (grid index); one particle not crossing the periodic box
 * faces is assumed. */
typedef struct {
    double centre[3];
    int64_t points;
    double R_mean, R_min, R_max;
    double eps_eff;
} spfm_contour;

typedef struct spfm_ctx spfm_ctx;
typedef struct spfm_batch spfm_batch;

/* Create a context for one grid (Sec. 2.1 statement of the problem).
 * lambda: interface width (Eq. 3), Gamma: interface energy, M: kinetic
 * coefficient, mu: driving force (Eq. 1-2); stencil: 6, 18 or 26.
 * Returns SPFM_E_INVAL for non-positive lambda, Gamma, M or dx, an unknown
 * stencil, coupling or dtype, a grid edge below 3 (below 1 on a walled axis), a grid too large (one
 * stored z-plane of 2^31 bytes or more, ny > 262140 or nz > 65535), a walls mask
 * outside 0..7 or |wall_sin| > 1 on a walled axis, walls with tsteps > 1,
 * a zero GLOBAL direction,
 * F32 with lambda < 0.3 dx, or exactly one of d_phi given;
 * SPFM_E_UNSTABLE when dt exceeds the explicit bound (unless allow_unstable).
 * Argument checks happen before any HIP call.  The field is zero until set. */
spfm_status spfm_create(const spfm_grid *grid, double lambda, double Gamma, double M, double mu,
                        int stencil, const spfm_options *opt, spfm_ctx **out);
/* Free the context and the buffers it allocated.  NULL is a no-op. */
void spfm_destroy(spfm_ctx *ctx);

/* Copy nx*ny*nz values of the context dtype into the current field (the
 * grid points; with walls, the interior of the stored field).  Resets the step
 * counter and the interface reference (position becomes NaN). */
spfm_status spfm_set_field(spfm_ctx *ctx, const void *src, int src_on_device);
/* Copy the nx*ny*nz grid values out (synchronises when dst is host memory). */
spfm_status spfm_get_field(spfm_ctx *ctx, void *dst, int dst_on_device);
/* Device pointer of the current stored field (valid until the next spfm_step):
 * with walls it includes the ghost layers, which hold the values of the last
 * fill (before the last step) and are otherwise undefined. */
spfm_status spfm_field_ptr(spfm_ctx *ctx, void **d_ptr);

/* Eq. 3 initial fields, computed on the device.
 * Planar: periodic slab with integer normal hkl (not all zero): the field
 * depends on s = p.N/|N| - c with period P = gcd_i(n_i |N_i|) dx / |N|; one
 * period is phi = 1 of thickness P/2 between two ideal interfaces, summed over
 * periodic images; c = box centre projected on N plus offset.
 * Spheres: phi = 1 - prod_i (1 - phi_i), phi_i the ideal radial profile of
 * radius radii[i] around centers[3i..3i+2] (host arrays, minimum-image
 * distance).  Both reset the step counter and set the interface reference. */
spfm_status spfm_init_planar(spfm_ctx *ctx, const int32_t hkl[3], double offset);
spfm_status spfm_init_spheres(spfm_ctx *ctx, int32_t n, const double *centers,
                              const double *radii);
/* Allocation-free variant of spfm_init_spheres, for callers that cannot
 * allocate device memory (tight loops that re-initialise a field, harnesses
 * that forbid allocation).  Same arguments and the same field bit for bit; the
 * sphere table is staged in a library-held static device array of at most 4096
 * spheres (128 KiB per GPU, held until the process ends) instead of a
 * per-call allocation.  Calls no hipMalloc or hipFree.  SPFM_E_INVAL for n >
 * 4096 (and as spfm_init_spheres otherwise); SPFM_E_STATE unless the device
 * that was current at spfm_create is current.  The call waits for its own
 * work, so calls from one host thread never overlap; calls that overlap on one
 * GPU (other host threads or processes) share the array and race. */
spfm_status spfm_init_spheres_noalloc(spfm_ctx *ctx, int32_t n, const double *centers,
                                      const double *radii);
/* Eq. 3 single planar front (not periodic): phi = (1 - tanh(2 s / lambda)) / 2,
 * s = p . n/|n| - c, c = the box centre (nx, ny, nz) dx / 2 projected on n/|n|
 * plus offset; phase 1 behind the front, n points into phase 0.  Every axis
 * along which n has a nonzero component must be walled (SPFM_E_INVAL
 * otherwise).  Resets the step counter; interface_position is then the
 * front's displacement along n (phase volume change over the front area,
 * taken as the box cross-section across the axis of the largest |n_d|,
 * divided by |n_d|/|n|). */
spfm_status spfm_init_front(spfm_ctx *ctx, const double n[3], double offset);
/* Box particle with smooth faces: phi = prod_d f(x_d - lo_d) f(hi_d - x_d),
 * f(s) = (1 + tanh(2 s / lambda)) / 2 (Eq. 3), lengths in units of length
 * (x_d = grid index times dx).  lo < hi on every axis. */
spfm_status spfm_init_box(spfm_ctx *ctx, const double lo[3], const double hi[3]);
/* Contour statistics of the current field (FP64 reductions on the device;
 * synchronises).  SPFM_E_STATE for walled grids. */
spfm_status spfm_contour_stats(spfm_ctx *ctx, spfm_contour *out);
/* Free energy of Eq. 1 of the current field (FP64 on the device, compensated
 * sums; synchronises): F = dx^3 sum_p Gamma/(C_Gamma lambda) sum_k gamma_j
 * nu_j [lambda^2/2 ((phi_{p+r_k} - phi_p)/|r_k|)^2 + g_k(phi_p)], one r_k of
 * each opposite pair over the stencil's directions, g_k of Eq. 6 with a_k =
 * tanh(2 r_k.n dx / lambda) (TI_n: n from central differences of psi, as in
 * the step; TI_<hkl>: n = u) or 8 phi^2 (1-phi)^2 / 3 (CF); with with_mu
 * nonzero plus dx^3 sum_p mu h(phi_p) with the context's mu and h.
 * SPFM_E_STATE for walled grids. */
spfm_status spfm_energy(spfm_ctx *ctx, int with_mu, double *out);
/* Radii of a particle's phi = 1/2 surface along n rays from centre, the
 * isotropy of its shape (Sec. 3.3) sampled along seeded directions: psi =
 * ln((1-phi)/phi) of the field with phi clamped to [1e-12, 1 - 1e-12] (the
 * inverse of Eq. 3 up to the factor lambda/4, which does not move its zero),
 * trilinear between grid points of the periodic box, marched in steps of dx/4
 * from the centre to the first sample with psi >= 0 and bisected 44 times.
 * centre: 3 host doubles (x, y, z, units of length = dx * grid index); dirs:
 * 3n host doubles, normalised here; radii: n host doubles, units of length, NaN
 * where the centre is outside the particle or the ray runs half the smallest
 * box edge without crossing.  Synchronises.  SPFM_E_INVAL for n < 1, NULL
 * arrays, a non-finite centre or a zero direction; SPFM_E_STATE for walled
 * grids. */
spfm_status spfm_ray_radii(spfm_ctx *ctx, const double centre[3], int32_t n, const double *dirs,
                           double *radii);

/* Total force on the interfaces of the current field (FP64 compensated sum;
 * synchronises): F = sum_p sum_k gamma_j nu_j (lambda^2 / |r_k|^2 D_k -
 * g_k'(phi_p)), the system sum of the bracket of Eq. 4 (the interface part of
 * the functional derivative of Eq. 1, Sec. 2.1), in units of 1/dx^2 with the
 * context's model and stencil; walled grids take their Eq. 7 ghost values.  It
 * vanishes for an ideal front wherever the model is translationally
 * invariant, and oscillates with the front's position on the grid otherwise
 * (the grid-friction force of Fig. 3).  Evaluated from the field alone: no
 * step is taken and the field is unchanged. */
spfm_status spfm_force(spfm_ctx *ctx, double *out);
/* Change the homogeneous driving force mu of the mu h(phi) term of Eq. 1
 * (Sec. 2.1; it enters the step of Eq. 2 as -2 M mu h'(phi) / (3 lambda Gamma)).
 * Re-checks the explicit stability bound (SPFM_E_UNSTABLE, mu unchanged) and
 * waits for the context stream first: steps already enqueued finish with the
 * old mu, later ones use the new one. */
spfm_status spfm_set_mu(spfm_ctx *ctx, double mu);
/* Enqueue n >= 0 forward-Euler steps of Eq. 2 (the functional derivative of
 * Eq. 1 with the potential of Eq. 6, Sec. 2.1) on the context stream. */
spfm_status spfm_step(spfm_ctx *ctx, int64_t n);
/* FP64 compensated reductions of the current field (synchronises): the phase
 * volume dx^3 sum phi and the interface measures of the spfm_diag fields.
 * The paper defines no area or position for these set-ups; the area is
 * (4/lambda) dx^3 sum phi(1-phi), which the ideal profile of Eq. 3 gives
 * exactly per unit interface area, and the position is the volume change over
 * that area (slabs, fronts) or the radius whose ideal radial profile holds the
 * volume (one sphere), both exact for Eq. 3 profiles (the interface position
 * of Sec. 2.3 as a volume measure; Fig. 1b tracks the same position). */
spfm_status spfm_diagnostics(spfm_ctx *ctx, spfm_diag *out);
spfm_status spfm_get_info(const spfm_ctx *ctx, spfm_info *out);

/* Many independent grids of different sizes stepped together (the problem of
 * Sec. 2.1 for each): one kernel launch per step covers every tile of every
 * grid.  Arrays have n entries.
 * The shared options (dtype must be F32, kernel, stream, C_Gamma <= 0, gamma,
 * eps, tau, allow_unstable, walls, zchunk) apply to every grid.  zchunk 0
 * with kernel TILED: 32 planes, halved down to 2 while the batch gives fewer
 * than 2^19 threads; with kernel AUTO and a batch that fills the GPU (32
 * planes kept) the first spfm_batch_step also times chunks of 4, 8, 16, 32 and
 * 64 planes and keeps the fastest (that call synchronises the stream, so it
 * must not be captured).  Each grid gets its own
 * lambda, Gamma, M, mu and, with walls, its own wall angles from
 * batch_wall_sin (the orientation sweeps of Sec. 3.2 in one launch; the
 * kernel computes the ghost values of Eq. 7 as it reads them); d_phi must be
 * NULL, tsteps <= 1 and conserve_volume 0.  Fields,
 * initial conditions and diagnostics refer to the interior of each grid. */
spfm_status spfm_batch_create(int32_t n, const spfm_grid *grids, const double *lambda,
                              const double *Gamma, const double *M, const double *mu,
                              int stencil, const spfm_options *opt, spfm_batch **out);
void spfm_batch_destroy(spfm_batch *b);
spfm_status spfm_batch_init_planar(spfm_batch *b, const int32_t *hkl /* 3n */,
                                   const double *offset /* n */);
/* A planar front of normal n (3 per grid, into phi = 0) through the centre of
 * grid i shifted by offset[i] along it (Eq. 3), as spfm_init_front; a normal
 * component along an axis needs walls on that axis.  Positions are then
 * tracked along each grid's normal. */
spfm_status spfm_batch_init_front(spfm_batch *b, const double *n /* 3n */,
                                  const double *offset /* n */);
spfm_status spfm_batch_set_field(spfm_batch *b, int32_t i, const void *src, int src_on_device);
spfm_status spfm_batch_get_field(spfm_batch *b, int32_t i, void *dst, int dst_on_device);
/* Enqueue n >= 0 forward-Euler steps of Eq. 2 (Sec. 2.1) of every grid of
 * the batch, each with its own coefficients.  Tiled kernel: one launch per
 * step covering all grids; resident kernel in x segments: one launch per halo's
 * worth of steps; both issued as replays of captured HIP graphs of 16 launches
 * for long runs (on a non-null stream).  Resident kernel on whole grids: up to
 * 4096 steps per launch.  The same sweeps of Sec. 3.1-3.2 (driving forces,
 * orientations) that the paper runs one grid at a time.  With kernel AUTO the
 * first call times the candidates (see spfm_kernel) and synchronises the
 * stream once. */
spfm_status spfm_batch_step(spfm_batch *b, int64_t n);
/* spfm_diagnostics for every grid of the batch (out: n entries; the FP64
 * compensated sums and interface measures of each grid's interior). */
spfm_status spfm_batch_diagnostics(spfm_batch *b, spfm_diag *out /* n entries */);
/* Total points over all grids. */
int64_t spfm_batch_points(const spfm_batch *b);
/* Leading z-chunk of the batch's work items (after tuning, if any); 0 for NULL. */
int32_t spfm_batch_zchunk(const spfm_batch *b);
/* The step kernel the batch uses: SPFM_KERNEL_TILED or SPFM_KERNEL_RESIDENT; -1 for NULL. */
int32_t spfm_batch_kernel(const spfm_batch *b);
/* What the batch runs (after tuning, if any): kernel, tile column and leading
 * z-chunk of the tiled kernel (0 for the resident one), grid and point counts,
 * and the resident kernel's x-segment length and halo ({0, 0}: whole grids). */
typedef struct {
    int32_t kernel, tile_x, tile_y, zchunk, grids;
    int64_t points;
    int32_t segment, halo;
} spfm_batch_info;
spfm_status spfm_batch_get_info(const spfm_batch *b, spfm_batch_info *out);

/* Host-only helpers (no HIP call): the calibration C_Gamma(lambda/dx) used
 * when C_Gamma <= 0, and the explicit stability bound for a parameter set
 * with the h3 driving force (spfm_get_info reports the bound of a context). */
double spfm_calibrate_cgamma(double lambda_over_dx, int coupling);
double spfm_stable_dt(int stencil, int coupling, const double u[3], const double gamma[3],
                      double lambda, double Gamma, double M, double mu, double dx,
                      double C_Gamma);

const char *spfm_status_string(spfm_status s);
const char *spfm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SPFM_H */
