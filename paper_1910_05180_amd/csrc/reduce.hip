// Diagnostics reductions: sum phi, sum phi(1-phi), min, max and a count of
// points that are non-finite or have |phi| > 2, over a field of any dtype.
// Every value is promoted to FP64 and accumulated with error-free
// transformations (TwoSum), per thread, then across the 64 lanes of a wave
// with shuffles, across the waves of a block through LDS, and finally over the
// block partials by a single block in a fixed order, so the result does not
// depend on scheduling (bitwise reproducible for a given size).
#include "spfm_impl.h"

namespace spfm {

namespace {

struct Acc {
    double s, c;
    __device__ __forceinline__ void add(double v) {
        const double t = s + v;
        const double bp = t - s;
        c += (s - (t - bp)) + (v - bp);
        s = t;
    }
    __device__ __forceinline__ void merge(double os, double oc) {
        const double t = s + os;
        const double bp = t - s;
        c += oc + ((s - (t - bp)) + (os - bp));
        s = t;
    }
};

struct Part {
    Acc a1, a2;
    double mn, mx, bad;
    __device__ __forceinline__ void merge(const Part& o) {
        a1.merge(o.a1.s, o.a1.c);
        a2.merge(o.a2.s, o.a2.c);
        mn = fmin(mn, o.mn);
        mx = fmax(mx, o.mx);
        bad += o.bad;
    }
    __device__ __forceinline__ Part shfl_xor(int m) const {
        Part o;
        o.a1.s = __shfl_xor(a1.s, m); o.a1.c = __shfl_xor(a1.c, m);
        o.a2.s = __shfl_xor(a2.s, m); o.a2.c = __shfl_xor(a2.c, m);
        o.mn = __shfl_xor(mn, m); o.mx = __shfl_xor(mx, m); o.bad = __shfl_xor(bad, m);
        return o;
    }
};

__device__ __forceinline__ Part block_reduce(Part p) {
    // wave64 butterfly: every lane ends with the same value
    for (int m = 32; m > 0; m >>= 1) p.merge(p.shfl_xor(m));
    __shared__ double sh[kReduceThreads / 64][kPartialStride];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        sh[wave][0] = p.a1.s; sh[wave][1] = p.a1.c; sh[wave][2] = p.a2.s; sh[wave][3] = p.a2.c;
        sh[wave][4] = p.mn; sh[wave][5] = p.mx; sh[wave][6] = p.bad;
    }
    __syncthreads();
    Part r = p;
    if (threadIdx.x == 0) {
        r.a1 = {sh[0][0], sh[0][1]}; r.a2 = {sh[0][2], sh[0][3]};
        r.mn = sh[0][4]; r.mx = sh[0][5]; r.bad = sh[0][6];
        for (int w = 1; w < kReduceThreads / 64; ++w) {
            Part o;
            o.a1 = {sh[w][0], sh[w][1]}; o.a2 = {sh[w][2], sh[w][3]};
            o.mn = sh[w][4]; o.mx = sh[w][5]; o.bad = sh[w][6];
            r.merge(o);
        }
    }
    return r;
}

template <typename T>
__global__ __launch_bounds__(kReduceThreads) void k_reduce_partial(const T* __restrict__ phi,
                                                                   int64_t n,
                                                                   double* __restrict__ partials) {
    Part p;
    p.a1 = {0.0, 0.0}; p.a2 = {0.0, 0.0};
    p.mn = INFINITY; p.mx = -INFINITY; p.bad = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kReduceThreads;
    for (int64_t i = (int64_t)blockIdx.x * kReduceThreads + threadIdx.x; i < n; i += stride) {
        const double v = (double)phi[i];
        p.a1.add(v);
        p.a2.add(v * (1.0 - v));
        p.mn = fmin(p.mn, v);
        p.mx = fmax(p.mx, v);
        if (!(fabs(v) <= 2.0)) p.bad += 1.0;
    }
    const Part r = block_reduce(p);
    if (threadIdx.x == 0) {
        double* o = partials + (size_t)blockIdx.x * kPartialStride;
        o[0] = r.a1.s; o[1] = r.a1.c; o[2] = r.a2.s; o[3] = r.a2.c;
        o[4] = r.mn; o[5] = r.mx; o[6] = r.bad;
    }
}

__global__ __launch_bounds__(kReduceThreads) void k_reduce_final(const double* __restrict__ partials,
                                                                 int nparts,
                                                                 ReduceOut* __restrict__ out) {
    Part p;
    p.a1 = {0.0, 0.0}; p.a2 = {0.0, 0.0};
    p.mn = INFINITY; p.mx = -INFINITY; p.bad = 0.0;
    for (int b = threadIdx.x; b < nparts; b += kReduceThreads) {
        const double* q = partials + (size_t)b * kPartialStride;
        Part o;
        o.a1 = {q[0], q[1]}; o.a2 = {q[2], q[3]};
        o.mn = q[4]; o.mx = q[5]; o.bad = q[6];
        p.merge(o);
    }
    const Part r = block_reduce(p);
    if (threadIdx.x == 0) {
        out->sum_phi = r.a1.s + r.a1.c;
        out->sum_x = r.a2.s + r.a2.c;
        out->phi_min = r.mn;
        out->phi_max = r.mx;
        out->bad = (unsigned long long)r.bad;
    }
}

}  // namespace

template <typename T>
hipError_t launch_reduce(const T* phi, int64_t n, double* d_partials, ReduceOut* d_out,
                         hipStream_t s) {
    hipLaunchKernelGGL((k_reduce_partial<T>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, phi,
                       n, d_partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kReduceThreads), 0, s, d_partials,
                       kReduceBlocks, d_out);
    return hipGetLastError();
}

template hipError_t launch_reduce<float>(const float*, int64_t, double*, ReduceOut*, hipStream_t);
template hipError_t launch_reduce<double>(const double*, int64_t, double*, ReduceOut*, hipStream_t);

}  // namespace spfm
