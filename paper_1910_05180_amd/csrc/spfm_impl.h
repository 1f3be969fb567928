// Internal declarations of the SPFM GPU library: step coefficients, the
// per-point update shared by every step kernel, and the kernel launchers.
//
// Per-point update (forward Euler of Eq. 2 with the functional derivative of
// Eq. 1).  With x = phi(1-phi), u = 1-2phi and shell weights
// W_j = gamma_j nu_j / |r_j|^2:
//
//   d_t phi = A lambda^2 sum_k W_k (D_k - P_k) - 6 B x,
//   A = 2M / (3 C_Gamma lambda^2),  B = 2 M mu / (3 lambda Gamma),
//
// D_k = phi(p+r_k) + phi(p-r_k) - 2 phi(p) is the second difference along
// direction k and P_k = (|r_k|^2/lambda^2) g_k'(phi) is the second difference
// the ideal profile of Eq. 3 would have there (Eq. 4-6).  Writing
// a_k = tanh(beta_k/2), beta_k = 4 r_k.n / lambda, the derivative of Eq. 6
// becomes  P_k = u y_k / (1 + y_k),  y_k = m_k x,  m_k = 2 cosh(beta_k) - 2,
// so the TI coupling needs only m_k, which for TI_n is built from
// E_i = exp(4 dx n_i / lambda) by hyperbolic addition formulas.  The sum over
// each shell is accumulated as one fraction (one reciprocal per shell).
// The CF control has P_k = (|r_k|^2 / lambda^2) (16/3) x u instead.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace spfm {

enum Coupling : int { kLocal = 0, kGlobal = 1, kCF = 2 };
// Interpolation function of the driving force (Tab. 2): h3 = phi^2 (3 - 2 phi),
// h5 = phi^3 (10 - 15 phi + 6 phi^2), h_Abel = phi^2 / (phi^2 + (1-phi)^2); with
// x = phi(1-phi) their slopes are 6x, 30x^2 and 2x/(1-2x)^2.  The paper pairs
// h5 and h_Abel with the CF potential only.
enum Interp : int { kH3 = 0, kH5 = 1, kHAbel = 2 };
// Kernel variants: the couplings above with h3, and CF with h5 or h_Abel.
enum KernelCoupling : int { kCF5 = 3, kCFAbel = 4 };
constexpr bool is_cf(int C) { return C >= kCF; }
inline int kernel_coupling(int coupling, int interp) {
    return coupling == kCF && interp == kH5 ? kCF5 : (coupling == kCF && interp == kHAbel ? kCFAbel : coupling);
}

// Slope h'(phi) of the interpolation function, in FP64.
__host__ __device__ __forceinline__ double h_slope(int interp, double phi) {
    const double x = phi * (1.0 - phi);
    if (interp == kH5) return 30.0 * x * x;
    if (interp == kHAbel) {
        const double d = 1.0 - 2.0 * x;
        return 2.0 * x / (d * d);
    }
    return 6.0 * x;
}
// The interpolation of a kernel coupling.
constexpr int kernel_interp(int C) { return C == kCF5 ? kH5 : (C == kCFAbel ? kHAbel : kH3); }

// Exact sums for the constant-volume correction.  Each term v is rounded once
// to a multiple of 2^-54 (|v| clamped to 64: the integer part of v 2^24, then
// the remainder in units of 2^-54), and the rounded terms are added as 128-bit
// integers.  Integer addition is exact and associative, so a total does not
// depend on how the points are split among threads, work items or launches:
// the correction is the same for every tile shape, z-chunk and kernel.
// s[0] sums phi* - phi, s[1] sums h'(phi); a partial is stored as 4 words
// (low and high word of s[0], then of s[1]).
struct CvAcc {
    __int128 s[2];
    __device__ __forceinline__ static __int128 fix(double v) {
        v = fmin(fmax(v, -64.0), 64.0);
        const double a = v * 0x1p24;
        const double h = rint(a);                        // |h| <= 2^30
        const int r = (int)rint((a - h) * 0x1p30);       // a - h is exact, |r| <= 2^29
        return (__int128)(int)h * ((__int128)1 << 30) + r;
    }
    __device__ __forceinline__ void add(double dphi, double hp) {
        s[0] += fix(dphi);
        s[1] += fix(hp);
    }
    __device__ __forceinline__ void add_words(const unsigned long long* w) {
        s[0] += (__int128)(((unsigned __int128)w[1] << 64) | w[0]);
        s[1] += (__int128)(((unsigned __int128)w[3] << 64) | w[2]);
    }
    __device__ __forceinline__ void store(unsigned long long* w) const {
        w[0] = (unsigned long long)s[0];
        w[1] = (unsigned long long)((unsigned __int128)s[0] >> 64);
        w[2] = (unsigned long long)s[1];
        w[3] = (unsigned long long)((unsigned __int128)s[1] >> 64);
    }
    // The value of a sum (one rounding of q 2^-54, q = a 2^30 + b, 0 <= b < 2^30).
    __device__ __forceinline__ static double value(__int128 q) {
        const long long a = (long long)(q >> 30);
        const int b = (int)(q & (((__int128)1 << 30) - 1));
        return (double)a * 0x1p-24 + (double)b * 0x1p-54;
    }
};
__device__ __forceinline__ __int128 shfl_xor_i128(__int128 v, int m) {
    const unsigned __int128 u = (unsigned __int128)v;
    unsigned w[4] = {(unsigned)u, (unsigned)(u >> 32), (unsigned)(u >> 64), (unsigned)(u >> 96)};
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = __shfl_xor(w[i], m);
    return (__int128)(((unsigned __int128)w[3] << 96) | ((unsigned __int128)w[2] << 64) |
                      ((unsigned __int128)w[1] << 32) | w[0]);
}
// Sum of a over the block (NT threads, a multiple of 64), stored to dst by
// thread 0.  Every thread of the block must call it.
template <int NT>
__device__ __forceinline__ void cv_block_store(CvAcc a, unsigned long long* dst) {
    for (int m = 32; m > 0; m >>= 1) {
        a.s[0] += shfl_xor_i128(a.s[0], m);
        a.s[1] += shfl_xor_i128(a.s[1], m);
    }
    __shared__ unsigned long long red[NT / 64][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) a.store(red[wave]);
    __syncthreads();
    if (threadIdx.x == 0) {
        CvAcc t{{0, 0}};
        for (int w = 0; w < NT / 64; ++w) t.add_words(red[w]);
        t.store(dst);
    }
}

template <typename T>
struct StepCoef {
    int nx, ny, nz;
    int pad;
    T K[3];    // dt A lambda^2 W_j per shell
    T A1, A2;  // tail sums: K_1 + 4 K_2 + 4 K_3 and K_2 + 2 K_3 (A3 = K_3)
    T kcf;     // CF: dt A (16/3) sum_k gamma_j nu_j
    T b;       // dt 6 B
    T kap2;    // LOCAL: 4 dx / (lambda ln 2), exponent scale for exp2
    T kap2h;   // LOCAL: kap2 / 2 (FP32 evaluates 2^(+-kap2 n_i / 2))
    T eps;     // floor of the log arguments in psi
    T tau2;    // LOCAL: |grad log2((1-phi)/phi)|^2 (central differences, per 2 dx)
               // below tau2 -> normal (1,0,0)
    T mg[13];  // GLOBAL: m_k per direction, shells 1|2|3 as in point_update
    T msum[3]; // GLOBAL: sum of m_k per shell
    T xtail;   // below this phi(1-phi) every y_k = m_k x is under one ulp of 1,
               // so y_k / (1 + y_k) equals y_k to the working precision
};

// psi' = log2((1-phi)/phi) with both arguments floored at eps; the interface
// normal is the direction of grad psi' (psi = (lambda ln2 / 4) psi' is the
// inverse of Eq. 3, linear in position on an ideal profile).
// FP32 uses the native CDNA transcendental instructions (v_log_f32, v_exp_f32,
// v_rcp_f32, v_rsq_f32; about 1 ulp); FP64 uses the full-precision library.
// max(v, eps) for eps > 0 as a signed-integer max of the bit patterns: positive
// floats order like their patterns, negative ones (and -0) lose to eps, a NaN
// stays NaN; one instruction, and the loaded value needs no quieting.
__device__ __forceinline__ float floor_pos(float v, float eps) {
    return __int_as_float(max(__float_as_int(v), __float_as_int(eps)));
}
__device__ __forceinline__ float psi2(float phi, float eps) {
    return __builtin_amdgcn_logf(floor_pos(1.0f - phi, eps)) - __builtin_amdgcn_logf(floor_pos(phi, eps));
}
__device__ __forceinline__ double psi2(double phi, double eps) {
    return log2(fmax(1.0 - phi, eps)) - log2(fmax(phi, eps));
}
__device__ __forceinline__ float fast_exp2(float v) { return __builtin_amdgcn_exp2f(v); }
__device__ __forceinline__ double fast_exp2(double v) { return exp2(v); }
__device__ __forceinline__ float fast_rsqrt(float v) { return __builtin_amdgcn_rsqf(v); }
__device__ __forceinline__ double fast_rsqrt(double v) { return rsqrt(v); }
__device__ __forceinline__ float fast_rcp(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double fast_rcp(double v) { return 1.0 / v; }

// Raw buffer access to one z-plane: the descriptor (base, size in bytes) lives
// in scalar registers and every lane supplies a 32-bit byte offset, so no
// 64-bit address arithmetic runs on the vector unit.  Dword 3 selects the
// 32-bit data format that gfx9 raw buffer instructions expect.
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, 0x00020000);
}
__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, int off, float*) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, int off, double*) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
// Aux = cache-policy bits of the store: 0 (default) or kStoreThrough = sc0 | sc1
// (system scope, written through the L2).  Writing the new field through
// leaves fewer dirty L2 lines to flush when the step kernel ends: the TI_n step
// measured 1.5% faster with it (FP32), the bandwidth-heavier CF step 1.3% slower.
constexpr int kStoreThrough = 17;
template <int Aux = 0>
__device__ __forceinline__ void buf_store(float v, __amdgpu_buffer_rsrc_t r, int off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, Aux);
}
template <int Aux = 0>
__device__ __forceinline__ void buf_store(double v, __amdgpu_buffer_rsrc_t r, int off) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, off, 0, Aux);
}

// An empty statement with side effects: the compiler may not speculate the
// block containing it, so a wave-uniform branch around that block stays a
// branch instead of being turned into an unconditional computation and a select.
__device__ __forceinline__ void keep_branch() { __asm__ volatile("" ::: "memory"); }

// Running sum of y_k / (1 + y_k) kept as one fraction num/den, started from
// the first term y_0.
template <typename T>
struct Frac {
    T num, den;
    __device__ __forceinline__ explicit Frac(T y) : num(y), den(y + T(1)) {}
    __device__ __forceinline__ void add(T y) {
        num = fma(y, num + den, num);
        den = fma(den, y, den);
    }
    __device__ __forceinline__ T value() const { return num * fast_rcp(den); }
};

// sum_j K_j sum_{k in shell j} y_k / (1 + y_k), one fraction per shell (y2 is
// read for S >= 18, y3 for S = 26).
template <typename T, int S>
__device__ __forceinline__ T shell_sums(const T (&y1)[3], const T (&y2)[6], const T (&y3)[4],
                                        const StepCoef<T>& k) {
    Frac<T> f1(y1[0]);
    f1.add(y1[1]);
    f1.add(y1[2]);
    T q = k.K[0] * f1.value();
    if (S >= 18) {
        Frac<T> f2(y2[0]);
#pragma unroll
        for (int i = 1; i < 6; ++i) f2.add(y2[i]);
        q = fma(k.K[1], f2.value(), q);
    }
    if (S >= 26) {
        Frac<T> f3(y3[0]);
#pragma unroll
        for (int i = 1; i < 4; ++i) f3.add(y3[i]);
        q = fma(k.K[2], f3.value(), q);
    }
    return q;
}

// Shell sums of second differences s_j = sum_{k in shell j} (phi(p+r_k) + phi(p-r_k) - 2 phi(p))
// from a neighbourhood accessor at(dx,dy,dz), dx,dy,dz in {-1,0,1}.  Shell 1 (the
// largest weight) is formed from differences to the centre value, exact for
// nearby values; shells 2 and 3 from sums of opposite neighbours.  Bulk regions
// (all values equal) give exactly 0.
template <typename T, int S, typename At>
__device__ __forceinline__ void shell_laplacian(At at, T p, T& s1, T& s2, T& s3) {
    s1 = ((at(1, 0, 0) - p) + (at(-1, 0, 0) - p)) + ((at(0, 1, 0) - p) + (at(0, -1, 0) - p)) +
         ((at(0, 0, 1) - p) + (at(0, 0, -1) - p));
    s2 = T(0);
    s3 = T(0);
    if (S >= 18) {
        s2 = (((at(1, 1, 0) + at(-1, -1, 0)) + (at(1, -1, 0) + at(-1, 1, 0))) +
              ((at(0, 1, 1) + at(0, -1, -1)) + (at(0, 1, -1) + at(0, -1, 1)))) +
             ((at(1, 0, 1) + at(-1, 0, -1)) + (at(1, 0, -1) + at(-1, 0, 1)));
        s2 = fma(T(-12), p, s2);
    }
    if (S >= 26) {
        s3 = ((at(1, 1, 1) + at(-1, -1, -1)) + (at(1, 1, -1) + at(-1, -1, 1))) +
             ((at(1, -1, 1) + at(-1, 1, -1)) + (at(-1, 1, 1) + at(1, -1, -1)));
        s3 = fma(T(-8), p, s3);
    }
}

// New value of phi at one point from its value p, the shell sums s1..s3 of
// second differences and grad(gx,gy,gz), which sets the central differences of
// psi' across the point (LOCAL only; called only where phi(1-phi) != 0).
template <typename T, int S, int C, typename Grad>
__device__ __forceinline__ T point_incr(T p, T s1, T s2, T s3, Grad grad, const StepCoef<T>& k);
template <typename T, int S, int C, typename Grad>
__device__ __forceinline__ T point_core(T p, T s1, T s2, T s3, Grad grad, const StepCoef<T>& k) {
    return p + point_incr<T, S, C>(p, s1, s2, s3, grad, k);
}
// The increment of one forward-Euler step at the point, dt d_t phi (point_core
// adds it to p).
template <typename T, int S, int C, typename Grad>
__device__ __forceinline__ T point_incr(T p, T s1, T s2, T s3, Grad grad, const StepCoef<T>& k) {
    const T x = p * (T(1) - p);
    const T u = fma(T(-2), p, T(1));
    T upd = k.K[0] * s1;
    if (S >= 18) upd = fma(k.K[1], s2, upd);
    if (S >= 26) upd = fma(k.K[2], s3, upd);
    if (is_cf(C)) {
        upd = fma(-k.kcf, x * u, upd);
    } else if (x != T(0)) {
        T q;
        if (C == kLocal) {
            T gx, gy, gz;
            grad(gx, gy, gz);
            T g2 = fma(gx, gx, fma(gy, gy, gz * gz));
            // Fallback normal (1,0,0) where |grad psi'| is below tau; rare, so
            // waves without such a lane skip the selects.
            const bool flat = !(g2 >= k.tau2);
            if (__ballot(flat) != 0) {
                keep_branch();
                gx = flat ? T(1) : gx;
                gy = flat ? T(0) : gy;
                gz = flat ? T(0) : gz;
                g2 = flat ? T(1) : g2;
            }
            const T rg = fast_rsqrt(g2);
            // c_i = 2cosh(kappa n_i) - 2 and s_i = 2sinh(kappa n_i) (the latter for
            // the full coupling only)
            T sx, sy, sz, cx, cy, cz;
            if constexpr (sizeof(T) == 4) {
                // FP32: c_i = (F - G)^2 with F = 2^(a/2), G = 2^(-a/2); six hardware
                // exponentials are cheaper than a reciprocal chain.
                const T sc = k.kap2h * rg;
                const T hx = sc * gx, hy = sc * gy, hz = sc * gz;
                const T fx = fast_exp2(hx), gx_ = fast_exp2(-hx);
                const T fy = fast_exp2(hy), gy_ = fast_exp2(-hy);
                const T fz = fast_exp2(hz), gz_ = fast_exp2(-hz);
                const T dx = fx - gx_, dy = fy - gy_, dz = fz - gz_;
                cx = dx * dx;
                cy = dy * dy;
                cz = dz * dz;
                sx = fma(fx, fx, -(gx_ * gx_));   // F^2 - G^2
                sy = fma(fy, fy, -(gy_ * gy_));
                sz = fma(fz, fz, -(gz_ * gz_));
            } else {
                // E_i = 2^(kappa n_i) and 1/E_i from one reciprocal; c_i = (E-1)^2/E
                const T sc = k.kap2 * rg;
                const T ex = fast_exp2(sc * gx), ey = fast_exp2(sc * gy), ez = fast_exp2(sc * gz);
                const T r = fast_rcp(ex * ey * ez);
                const T rx = r * ey * ez, ry = r * ex * ez, rz = r * ex * ey;
                cx = (ex - T(1)) * (ex - T(1)) * rx;
                cy = (ey - T(1)) * (ey - T(1)) * ry;
                cz = (ez - T(1)) * (ez - T(1)) * rz;
                sx = ex - rx;
                sy = ey - ry;
                sz = ez - rz;
            }
            // The full coupling only where some lane of the wave needs it, the tail
            // form only where some lane can take it: the votes keep both branches
            // wave-uniform, so tail-only waves skip the full coupling and waves
            // whose every lane needs it skip the tail sums.
            // (q is set below for every lane that reads it: a lane without the
            // full coupling makes its wave take the tail branch.)
            const bool full = !(fabs(x) < k.xtail);
            const unsigned long long vfull = __ballot(full);
            if (vfull != __ballot(true)) {
                keep_branch();
                // Tail: y/(1+y) -> y, with the per-shell sums of m_k in closed form,
                // sum_2 = sum_pairs (C_a C_b - 4), sum_3 = C_x C_y C_z - 8, C = c + 2.
                // K_1 s_1 + K_2 s_2 + K_3 s_3 = A1 c1 + A2 c2 + K_3 cx cy cz with
                // c1 = sum c, c2 = sum of pair products (A1, A2 folded on the host).
                const T cxy = cx + cy, pxy = cx * cy;
                const T c1 = cxy + cz;
                q = k.A1 * c1;
                if (S >= 18) q = fma(k.A2, fma(cz, cxy, pxy), q);
                if (S >= 26) q = fma(k.K[2], pxy * cz, q);
                q *= x;
            }
            if (vfull != 0) {
                keep_branch();
                // y_k = x m_k straight from x-scaled pieces: with
                // 2cosh(a +- b) - 2 = c_a + c_b + (c_a c_b +- s_a s_b)/2,
                // y = x c_a + x c_b + (x/2)(c_a c_b +- s_a s_b).
                const T xh = T(0.5) * x;
                const T y1[3] = {x * cx, x * cy, x * cz};
                T y2[6];   // shell 2: x+y, x-y, y+z, y-z, x+z, x-z
                T y3[4];   // shell 3: x+y+z, x+y-z, x-y+z, x-y-z
                T pxy = T(0), mxy = T(0);   // c_x c_y +- s_x s_y
                if (S >= 18) {
                    {
                        const T ps = sx * sy, b = y1[0] + y1[1];
                        pxy = fma(cx, cy, ps);
                        mxy = fma(cx, cy, -ps);
                        y2[0] = fma(xh, pxy, b);
                        y2[1] = fma(xh, mxy, b);
                    }
                    {
                        const T ps = sy * sz, b = y1[1] + y1[2];
                        y2[2] = fma(xh, fma(cy, cz, ps), b);
                        y2[3] = fma(xh, fma(cy, cz, -ps), b);
                    }
                    {
                        const T ps = sx * sz, b = y1[0] + y1[2];
                        y2[4] = fma(xh, fma(cx, cz, ps), b);
                        y2[5] = fma(xh, fma(cx, cz, -ps), b);
                    }
                }
                if (S >= 26) {
                    // w = x +- y: m_w = c_x + c_y + (c_x c_y +- s_x s_y)/2 and
                    // 2sinh(w) = (s_x (c_y+2) +- (c_x+2) s_y)/2; then
                    // x (2cosh(w +- z) - 2) = x m_w + x c_z + (x/2)(m_w c_z +- s_w s_z),
                    // with x m_w = y2[0] or y2[1].
                    const T cxy = cx + cy;
                    const T mp = fma(T(0.5), pxy, cxy), mm = fma(T(0.5), mxy, cxy);
                    const T csy = (cx + T(2)) * sy;
                    const T hp = T(0.5) * fma(sx, cy + T(2), csy);
                    const T hm = T(0.5) * fma(sx, cy + T(2), -csy);
                    {
                        const T ps = hp * sz, b = y2[0] + y1[2];
                        y3[0] = fma(xh, fma(mp, cz, ps), b);
                        y3[1] = fma(xh, fma(mp, cz, -ps), b);
                    }
                    {
                        const T ps = hm * sz, b = y2[1] + y1[2];
                        y3[2] = fma(xh, fma(mm, cz, ps), b);
                        y3[3] = fma(xh, fma(mm, cz, -ps), b);
                    }
                }
                const T qf = shell_sums<T, S>(y1, y2, y3, k);
                q = full ? qf : q;
            }
        } else {
            q = x * fma(k.K[0], k.msum[0], fma(k.K[1], k.msum[1], k.K[2] * k.msum[2]));
            const bool full = !(fabs(x) < k.xtail);
            if (__ballot(full) != 0) {
                keep_branch();
                const T y1[3] = {k.mg[0] * x, k.mg[1] * x, k.mg[2] * x};
                T y2[6], y3[4];
#pragma unroll
                for (int i = 0; i < 6; ++i) y2[i] = k.mg[3 + i] * x;
#pragma unroll
                for (int i = 0; i < 4; ++i) y3[i] = k.mg[9 + i] * x;
                const T qf = shell_sums<T, S>(y1, y2, y3, k);
                q = full ? qf : q;
            }
        }
        upd = fma(-u, q, upd);
    }
    // Driving force mu h'(phi); b holds dt 6B (h3), dt 30B (h5) or dt 2B (h_Abel).
    if (C == kCF5) {
        upd = fma(-k.b, x * x, upd);
    } else if (C == kCFAbel) {
        const T d = T(1) - T(2) * x;
        upd = fma(-k.b, x / (d * d), upd);
    } else {
        upd = fma(-k.b, x, upd);
    }
    return upd;
}

// Per-column values a thread of a z-marching sweep keeps for one plane: the
// plane's contribution to the shell sums of the column's points, read once
// from the staged plane and used by the three points z-1, z, z+1.
template <typename T>
struct PlaneRegs {
    T c;        // phi at the column
    T fc;       // sum of phi over the 4 in-plane face neighbours
    T dc;       // sum of phi over the 4 in-plane diagonal neighbours
    T gx, gy;   // LOCAL: in-plane central differences of psi' at the column
    T pc;       // LOCAL: psi' at the column
};

// PlaneRegs of one column from a staged plane (phi at P, psi' at Q, row stride
// LX), both pointing at the corner cell of the column's 3 x 3 neighbourhood:
// every offset lies within 2 LX + 2 elements of it, so one base address serves
// all the paired LDS reads.
template <typename T, int S, int C, int LX>
__device__ __forceinline__ void plane_sums(const T* P, const T* Q, PlaneRegs<T>& R) {
    R.c = P[LX + 1];
    R.fc = (P[LX + 2] + P[LX]) + (P[2 * LX + 1] + P[1]);
    if (S >= 18) R.dc = (P[2 * LX + 2] + P[0]) + (P[2 * LX] + P[2]);
    if (C == kLocal) {
        R.gx = Q[LX + 2] - Q[LX];
        R.gy = Q[2 * LX + 1] - Q[1];
        R.pc = Q[LX + 1];
    }
}

// New value of phi at a point from the PlaneRegs of its column on the planes
// below (Rm), at (R0) and above (Rp) it.  The shell sums of second differences
// come from the raw plane sums, each with its own multiple of the centre value
// taken off (exactly 0 where phi is 0 or 1 throughout; elsewhere the rounding
// of the sums stays well below half an ulp of the new value):
//   s1 = F(z) + c(z-1) + c(z+1) - 6p, s2 = D(z) + F(z-1) + F(z+1) - 12p,
//   s3 = D(z-1) + D(z+1) - 8p.
template <typename T, int S, int C>
__device__ __forceinline__ T point_from_planes(const PlaneRegs<T>& Rm, const PlaneRegs<T>& R0,
                                               const PlaneRegs<T>& Rp, const StepCoef<T>& k) {
    const T p = R0.c;
    const T s1 = fma(T(-6), p, R0.fc + (Rm.c + Rp.c));
    T s2 = T(0), s3 = T(0);
    if (S >= 18) s2 = fma(T(-12), p, R0.dc + (Rm.fc + Rp.fc));
    if (S >= 26) s3 = fma(T(-8), p, Rm.dc + Rp.dc);
    auto grad = [&](T& gx, T& gy, T& gz) {
        gx = R0.gx;
        gy = R0.gy;
        gz = Rp.pc - Rm.pc;
    };
    return point_core<T, S, C>(p, s1, s2, s3, grad, k);
}

// New value of phi at one point.  at(dx,dy,dz) returns phi at the offset
// (dx,dy,dz in {-1,0,1}); grad as in point_core.
template <typename T, int S, int C, typename At, typename Grad>
__device__ __forceinline__ T point_update(At at, Grad grad, const StepCoef<T>& k) {
    const T p = at(0, 0, 0);
    T s1, s2, s3;
    shell_laplacian<T, S>(at, p, s1, s2, s3);
    return point_core<T, S, C>(p, s1, s2, s3, grad, k);
}

// dt d_t phi at one point (the increment of point_update).
template <typename T, int S, int C, typename At, typename Grad>
__device__ __forceinline__ T point_rate_dt(At at, Grad grad, const StepCoef<T>& k) {
    const T p = at(0, 0, 0);
    T s1, s2, s3;
    shell_laplacian<T, S>(at, p, s1, s2, s3);
    return point_incr<T, S, C>(p, s1, s2, s3, grad, k);
}

// Contact-angle walls (walls.hip): stored dims, the walled axes (bit d = axis d)
// and the composed Eq. 7 coefficient for every ghost class (cx, cy, cz in
// {-1, 0, 1}: below the low wall, inside, above the high wall), at index
// (cx + 1) + 3 (cy + 1) + 9 (cz + 1).
template <typename T>
struct WallCoef {
    int sx, sy, sz;
    int walls;
    T a[27];
};

// Eq. 7 as a map of the inward neighbour's value v: the ideal profile moved by
// the length d with tanh(2 d / lambda) = a (a = 0 returns v exactly).  The one
// expression both the ghost fill and the walled sweeps evaluate.
template <typename T>
__device__ __forceinline__ T wall_map(T v, T a) {
    return (T(1) - a) * v / (T(1) - a * (T(2) * v - T(1)));
}

// ---- launchers (step_kernels.hip, reduce.hip, init.hip, walls.hip) ----
struct TileItem {   // one block of the batched step: grid index, tile origin, planes
    int inst;
    int x0, y0, z0;
    int zlen;
};

template <typename T>
hipError_t launch_step_plain(const T* in, T* out, const StepCoef<T>& k, int stencil, int coupling,
                             hipStream_t s);
// One block per entry of the device table d_items (nitems entries, in dispatch order).
// d_wall (device memory) non-null: the stored grid has contact-angle walls, and
// ghost cells are computed from their interior neighbours as they are staged
// (Eq. 7), so no fill launch is needed.
// cv_part non-null (periodic grids, the untuned tile shape only): the step also
// writes, for work item i, the exact sums of phi* - phi and h'(phi) over its
// points into cv_part[4i .. 4i+3] (CvAcc; the constant-volume correction).
// fuse non-null (with cv_part): `in` holds the previous step's uncorrected
// phi*, and the step first applies that step's correction as it reads its
// planes (CvFuse below), so that one launch per step does both.
template <typename T>
struct CvFuse {
    const T* old;                     // the field the previous step started from
    T* corr;                          // receives the corrected field (the step's input)
    const unsigned long long* part;   // the previous step's sums, 4 words per work item
    int nparts;                       // at most kCvDirectParts
};
template <typename T>
hipError_t launch_step_tiled(const T* in, T* out, const StepCoef<T>& k, int stencil, int coupling,
                             int tile, const TileItem* d_items, int nitems, const WallCoef<T>* d_wall,
                             unsigned long long* cv_part, const CvFuse<T>* fuse, hipStream_t s);
// The tiled and batched steps of one kernel coupling (sweep.h; instantiated in
// the per-coupling translation units).
template <typename T, int C>
hipError_t launch_tiled_coupling(const T* in, T* out, const StepCoef<T>& k, int stencil, int tile,
                                 const TileItem* items, int nitems, const WallCoef<T>* wall,
                                 unsigned long long* cv_part, const CvFuse<T>* fuse, hipStream_t s);
template <int C>
hipError_t launch_batched_coupling(const float* in, float* out, const StepCoef<float>* coef,
                                   const int64_t* offset, int stencil, int tile, const TileItem* items,
                                   int nitems, const WallCoef<float>* wall, hipStream_t s);
// TB = tsteps (2..4) steps per launch, FP32 (temporal.hip).
hipError_t launch_step_temporal(const float* in, float* out, const StepCoef<float>& k, int stencil,
                                int coupling, int tsteps, int zlen, hipStream_t s);
// Batched step: instance i reads buf_in + offset[i], writes buf_out + offset[i];
// with d_wall (one entry per instance) the grids have walls, as for the tiled step.
hipError_t launch_step_batched(const float* buf_in, float* buf_out, const StepCoef<float>* d_coef,
                               const int64_t* d_offset, const TileItem* d_items, int nitems,
                               const WallCoef<float>* d_wall, int stencil, int coupling, int tile,
                               hipStream_t s);
// Resident step (resident.hip): one block per grid keeps the stored grid in LDS
// (two copies, 2 x cells x sizeof(T) <= kResidentLdsBytes) and takes nsteps steps
// in one launch: reads buf_in + offset[g], writes buf_out + offset[g] (which may
// be the same buffer).  Results equal nsteps tiled steps bit for bit.
// d_items null: block g holds grid g whole.  Otherwise block b holds the part
// of grid items[b].inst given there (x segments with halos, see resident.hip):
// then nsteps must not exceed any halo, buf_in and buf_out must differ, and
// max_cells bounds the cells of any block's region.
struct ResItem {
    int inst;   // grid
    int rx0;    // region: stored x in [rx0, rx0 + rw), mod nx (rx0 < 0 wraps a periodic axis)
    int rw;
    int ox;     // columns written back: stored x in [ox, ox + olen)
    int olen;
};
constexpr int kResidentLdsBytes = 163840;   // gfx950: LDS one workgroup may allocate
int resident_max_cells(int elem_bytes);
template <typename T>
hipError_t launch_step_resident(const T* buf_in, T* buf_out, const StepCoef<T>* d_coef,
                                const int64_t* d_offset, const WallCoef<T>* d_wall,
                                const ResItem* d_items, int nblocks, int max_cells, int nsteps,
                                int stencil, int coupling, hipStream_t s);
// Tile shapes of the single-step tiled kernels: a block marches one tile
// column TX x TY along z, each of its waves computing a 16 x 4 patch.  The
// untuned shapes: FP32 TI_n uses 16 x 8 columns (two waves): its full-coupling
// branch makes the work of a wave uneven from plane to plane, and a block of
// few waves loses little at its barriers while the SIMD runs waves of other
// blocks; the other kernels use 64 x 8 columns (eight waves), whose halo is
// relatively smaller.  The autotuner times the other compiled shapes.
enum TileShape : int {
    kTile16x8 = 0, kTile32x8 = 1, kTile64x8 = 2, kTile16x16 = 3, kTile32x16 = 4, kTile64x16 = 5,
    kNumTileShapes = 6
};
constexpr int tile_tx(int t) {
    return (t == kTile16x8 || t == kTile16x16) ? 16 : ((t == kTile32x8 || t == kTile32x16) ? 32 : 64);
}
constexpr int tile_ty(int t) { return t >= kTile16x16 ? 16 : 8; }
constexpr int default_tile(bool f32, int coupling) { return f32 && coupling == kLocal ? kTile16x8 : kTile64x8; }
// Shapes compiled for a kernel variant (kernel coupling C, walled or not): every
// shape for the FP32 steps with h3 (TI_n, TI_<hkl>, CF); 64 x 8, 32 x 8 and
// 16 x 8 for FP64 TI_n; the untuned shape alone for walled grids (small, launch
// bound) and for CF with h5 or h_Abel.
constexpr bool tile_compiled(bool f32, int C, bool W, int t) {
    return t == default_tile(f32, C) ||
           (!W && (f32 ? C <= kCF : (C == kLocal && (t == kTile32x8 || t == kTile16x8))));
}
constexpr int kWaveX = 16;
// LDS row stride of a staged halo plane: 48 (16- and 32-wide tiles) and 80
// (64-wide) put the four rows of a 16 x 4 wave patch in distinct LDS banks.
// Every smaller stride that holds a 16-wide row and its halo gives two-way bank
// conflicts; 48 caps 16 x 8 blocks at 10 per CU by LDS (5 waves per SIMD
// instead of 7) and still runs the TI_n step 1.8% faster.
constexpr int lds_row(int tx) { return tx == 64 ? 80 : 48; }
constexpr int kTileZ = 32;   // default planes per block (the z-chunk is a launch argument)
constexpr int kNumXcd = 8;   // MI355X: workgroup IDs are dealt to the 8 XCDs round robin

// Dispatch slot b -> logical tile: XCD (b mod 8) receives one contiguous run of
// logical tiles (x fastest, then y, then z), so tiles that share halo rows and
// columns are processed by the same XCD and meet in its L2.
__host__ __device__ __forceinline__ int xcd_remap(int b, int n) {
    const int q = n / kNumXcd, r = n % kNumXcd;
    const int k = b % kNumXcd, i = b / kNumXcd;
    return k < r ? k * (q + 1) + i : r * (q + 1) + (k - r) * q + i;
}

// Number of ghost points of a padded field (the threads of one fill).
int64_t wall_ghosts(int sx, int sy, int sz, int walls);
template <typename T>
hipError_t launch_fill_walls(T* phi, const WallCoef<T>& w, int64_t nghost, hipStream_t s);
template <typename T>
hipError_t launch_box_copy(T* dst, int dnx, int dny, int dx0, int dy0, int dz0, const T* src,
                           int snx, int sny, int sx0, int sy0, int sz0, int bx, int by, int bz,
                           hipStream_t s);
template <typename T>
hipError_t launch_init_front(T* phi, int nx, int ny, int nz, double dx, double lambda,
                             const double n[3], double offset, hipStream_t s);

// Force density of the field (force.hip): dt d_t phi without the driving force
// (coefficients k with mu = 0) at every interior point of the stored grid
// (walled axes wx, wy, wz skip one ghost layer per end), packed densely into
// dens (nx*ny*nz interior values).  Ghost layers must hold their Eq. 7 values.
template <typename T>
hipError_t launch_force_density(const T* phi, T* dens, const StepCoef<T>& k, int walls, int stencil,
                                int coupling, hipStream_t s);

// Constant volume and contour statistics (volume.hip).  launch_cv_correct: the
// partial sums of phi_new - phi_old and h'(phi_old) (at most kReduceBlocks CvAcc
// partials, 4 words each, in d_part), then the correction.  launch_cv_apply: the
// correction from nparts partials already written by the step (cv_part of
// launch_step_tiled); beyond kCvDirectParts they are first reduced into d_total
// (4 words).  Both apply phi_new -= g h'(phi_old) with g = sum(phi_new -
// phi_old) / sum h'(phi_old) and store g, mu = g / dt_beta in d_state (2
// doubles).  launch_contour_stats: d_part holds kReduceBlocks x 8 doubles, d_out
// 7 doubles (barycentre x, y, z, then count, sum R, min R, max R in grid units).
constexpr int kCvDirectParts = 1024;
template <typename T>
hipError_t launch_cv_correct(const T* phi_old, T* phi_new, int64_t n, int interp, double dt_beta,
                             unsigned long long* d_part, double* d_state, hipStream_t s);
// phi_out non-null: the corrected field goes there instead of into phi_new.
template <typename T>
hipError_t launch_cv_apply(const T* phi_old, T* phi_new, int64_t n, int interp, double dt_beta,
                           const unsigned long long* d_part, int nparts, unsigned long long* d_total,
                           double* d_state, hipStream_t s, T* phi_out = nullptr);
template <typename T>
hipError_t launch_contour_stats(const T* phi, int nx, int ny, int nz, double* d_part, double* d_out,
                                hipStream_t s);
// Coefficients of the free energy of Eq. 1 (FP64): per-shell weights
// gamma_j nu_j (0 beyond the stencil), the prefactor Gamma / (C_Gamma lambda),
// and for TI_<hkl> the a_k = tanh(2 r_k.u dx / lambda) of its fixed direction.
struct EnergyCoef {
    double w[3];
    double pref;
    double lambda, dx, mu, eps, tau;
    double ag[13];
    int ndir;       // 3, 9 or 13 directions
    int coupling;   // 0 TI_n, 1 TI_<hkl>, 2 CF (the spfm_coupling values)
    int interp;     // kH3, kH5 or kHAbel (for the mu h(phi) term)
};
// F = dx^3 sum_p f_p of Eq. 1 (with mu h(phi) when with_mu), compensated FP64
// sums: per-block partials in d_part (2 x 1024 doubles), the total in *d_out.
template <typename T>
hipError_t launch_energy(const T* phi, int nx, int ny, int nz, const EnergyCoef& c, int with_mu,
                         double* d_part, double* d_out, hipStream_t s);
// Radii of the phi = 1/2 surface along n rays (d_dirs: 3n device doubles) from
// centre (host, grid units) into d_radii (n device doubles, grid units).
template <typename T>
hipError_t launch_ray_radii(const T* phi, int nx, int ny, int nz, const double* centre,
                           const double* d_dirs, int n, double* d_radii, hipStream_t s);
template <typename T>
hipError_t launch_init_box(T* phi, int nx, int ny, int nz, double dx, double lambda,
                           const double lo[3], const double hi[3], hipStream_t s);

struct ReduceOut {   // device result of the diagnostics reduction
    double sum_phi, sum_x;
    double phi_min, phi_max;
    unsigned long long bad;
};
template <typename T>
hipError_t launch_reduce(const T* phi, int64_t n, double* d_partials, ReduceOut* d_out,
                         hipStream_t s);
constexpr int kReduceBlocks = 1024;
constexpr int kReduceThreads = 256;
constexpr int kPartialStride = 7;   // doubles per block partial: s1 c1 s2 c2 min max bad

template <typename T>
hipError_t launch_init_planar(T* phi, int nx, int ny, int nz, double dx, double lambda,
                              const int hkl[3], double offset, hipStream_t s);
template <typename T>
hipError_t launch_init_spheres(T* phi, int nx, int ny, int nz, double dx, double lambda, int n,
                               const double* d_spheres, hipStream_t s);
// Allocation-free sphere initialisation: the device address, on the current
// device, of a static table of kMaxScratchSpheres spheres (4 doubles each).
constexpr int kMaxScratchSpheres = 4096;
hipError_t sphere_scratch(double** out);

}  // namespace spfm
