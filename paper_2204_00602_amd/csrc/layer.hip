// HIP kernels (gfx950) of the SLOS layer recurrence.
//
// One launch computes layer k of the recurrence of arXiv 2204.00602, Section
// 3.2.3 (SLOS), in gather form:
//     A_k[t] = sum_{j : t_j > 0} U[j, i_k] * A_{k-1}[t - e_j],
// every output written by exactly one lane, no atomics.  The last layer fuses
// the normalisation a(S) = A_n[S] sqrt(prod s_j!) / sqrt(prod t_i!) (Eq.
// eqperm), |a|^2 and an FP64 per-wave partial of sum_S P(S).
//
// Work unit: one leaf per wave (see LeafRec).  The wave computes, with scalar
// arithmetic, the base rank in A_{k-1} of every predecessor block reached
// through a high mode; those reads are contiguous (lane x reads base + x).
// Predecessors through the q low modes come from the per-(q, K) inner table.
// U's column i_k is staged in LDS; u[255] = 0 pads short term lists.
#include <hip/hip_runtime.h>

#include "slos_internal.h"

namespace {

template <typename T> struct Cx;
template <> struct Cx<float> { using type = float2; };
template <> struct Cx<double> { using type = double2; };

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// acc += u * v (complex), four fused multiply-adds
template <typename C>
__device__ __forceinline__ void cmac(C &acc, const C u, const C v)
{
    acc.x = fma_(u.x, v.x, acc.x);
    acc.x = fma_(-u.y, v.y, acc.x);
    acc.y = fma_(u.x, v.y, acc.y);
    acc.y = fma_(u.y, v.x, acc.y);
}

// Error-free accumulation of a*b into (s, c): the product's rounding error
// comes from an FMA, the sum's from Knuth's two-sum; both go to c.
__device__ __forceinline__ void acc_exact(float &s, float &c, float a, float b)
{
#pragma clang fp contract(off)
    float p = a * b;
    float pe = __builtin_fmaf(a, b, -p);
    float t = s + p;
    float bb = t - s;
    float e = (s - (t - bb)) + (p - bb);
    s = t;
    c = c + (e + pe);
}

struct CompAcc {
    float2 s, c;
};

__device__ __forceinline__ void cmac_comp(CompAcc &a, const float2 u, const float2 v)
{
    acc_exact(a.s.x, a.c.x, u.x, v.x);
    acc_exact(a.s.x, a.c.x, -u.y, v.y);
    acc_exact(a.s.y, a.c.y, u.x, v.y);
    acc_exact(a.s.y, a.c.y, u.y, v.x);
}

template <typename T, bool COMP> struct Acc;
template <typename T> struct Acc<T, false> {
    using C = typename Cx<T>::type;
    C a;
    __device__ __forceinline__ void zero() { a = C{0, 0}; }
    __device__ __forceinline__ void mac(const C u, const C v) { cmac(a, u, v); }
    __device__ __forceinline__ C value() const { return a; }
    __device__ __forceinline__ double re() const { return (double)a.x; }
    __device__ __forceinline__ double im() const { return (double)a.y; }
};
template <> struct Acc<float, true> {
    CompAcc a;
    __device__ __forceinline__ void zero() { a.s = float2{0.f, 0.f}; a.c = float2{0.f, 0.f}; }
    __device__ __forceinline__ void mac(const float2 u, const float2 v) { cmac_comp(a, u, v); }
    __device__ __forceinline__ float2 value() const { return float2{a.s.x + a.c.x, a.s.y + a.c.y}; }
    __device__ __forceinline__ double re() const { return (double)a.s.x + (double)a.c.x; }
    __device__ __forceinline__ double im() const { return (double)a.s.y + (double)a.c.y; }
};

constexpr int kMaxWaves = 4;  // workgroups of at most 256 threads

template <typename T, int MODE, bool COMP, int RR>
__global__ __launch_bounds__(256) void layer_kernel(LayerParams p)
{
    using C = typename Cx<T>::type;
    __shared__ C u_lds[256];
    __shared__ uint64_t base_lds[kMaxWaves][SLOS_MAX_PHOTONS];
    __shared__ C hu_lds[kMaxWaves][SLOS_MAX_PHOTONS];

    const C *__restrict__ X = (const C *)p.X;
    const C *__restrict__ Um = (const C *)p.U;
    for (int j = threadIdx.x; j < 256; j += blockDim.x) {
        C v{0, 0};
        if (j < p.m) v = Um[(size_t)j * p.m + p.col];
        u_lds[j] = v;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wpb = blockDim.x >> 6;
    const uint64_t gw = (uint64_t)blockIdx.x * wpb + wv;
    const uint64_t nw = (uint64_t)gridDim.x * wpb;
    const uint64_t *__restrict__ binom = p.binom;
    const int bs = p.bstride;
    double psum = 0.0;

    for (uint64_t li = gw; li < p.nleaves; li += nw) {
        const LeafRec *L = p.leaves + li;
        const uint64_t out_base = L->out_base;
        const uint32_t size = L->size;
        const int nhp = L->nhp;
        const InnerType ty = p.types[L->tab];

        // Predecessor blocks through the high modes.  Positions r = k, k-1, ..
        // hold the high photons (descending modes); c_r = d_r + r - 1.  For the
        // top photon of mode d at position r:
        //   rank(t) - rank(t - e_d) = C(c_r, r) + sum_{r' > r} C(c_{r'} - 1, r').
        uint64_t S = 0;
        int nh = 0;
        int grp = 0;
        int prev = -1;
        double hifac = 1.0;
        for (int idx = 0; idx < nhp; ++idx) {
            const int r = p.k - idx;
            const int d = L->hm[idx];
            const int c = d + r - 1;
            if (d != prev) {
                base_lds[wv][nh] = out_base - (binom[c * bs + r] + S);
                hu_lds[wv][nh] = u_lds[d];
                ++nh;
                grp = 1;
                prev = d;
            } else {
                ++grp;
                hifac *= (double)grp;
            }
            S += binom[(c - 1) * bs + r];
        }
        // the block of the same high part with K-1 low photons
        const uint64_t low_base = out_base - S;
        const uint32_t *__restrict__ pred = p.pred + ty.pred_off;
        const int cmax = (int)ty.cmax;
        const double fac_hi = MODE != SLOS_MODE_MID ? sqrt(hifac) * p.norm_t : 1.0;

        for (uint32_t t0 = 0; t0 < size; t0 += 64 * RR) {
            Acc<T, COMP> acc[RR];
#pragma unroll
            for (int q = 0; q < RR; ++q) acc[q].zero();

            for (int h = 0; h < nh; ++h) {
                const uint64_t b = base_lds[wv][h];
                const C u = hu_lds[wv][h];
                const C *__restrict__ Xb = X + b;
#pragma unroll
                for (int q = 0; q < RR; ++q) {
                    const uint32_t x = t0 + q * 64 + lane;
                    if (x < size) acc[q].mac(u, Xb[x]);
                }
            }
            const C *__restrict__ Xl = X + low_base;
            for (int c = 0; c < cmax; ++c) {
#pragma unroll
                for (int q = 0; q < RR; ++q) {
                    const uint32_t x = t0 + q * 64 + lane;
                    if (x < size) {
                        const uint32_t e = pred[(size_t)c * size + x];
                        acc[q].mac(u_lds[e >> 24], Xl[e & SLOS_PRED_MASK]);
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < RR; ++q) {
                const uint32_t x = t0 + q * 64 + lane;
                if (x < size) {
                    if (MODE == SLOS_MODE_MID) {
                        ((C *)p.Y)[out_base + x] = acc[q].value();
                    } else {
                        const double f = fac_hi * p.lowfac[ty.fac_off + x];
                        const double ar = acc[q].re() * f;
                        const double ai = acc[q].im() * f;
                        const double pr = ar * ar + ai * ai;
                        psum += pr;
                        if (MODE == SLOS_MODE_AMPL)
                            ((C *)p.Y)[out_base + x] = C{(T)ar, (T)ai};
                        else
                            ((T *)p.Y)[out_base + x] = (T)pr;
                    }
                }
            }
        }
    }

    if (MODE != SLOS_MODE_MID) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) psum += __shfl_xor(psum, off, 64);
        if (lane == 0) p.partials[gw] = psum;
    }
}

// Deterministic sum of the per-wave partials: fixed strided order per thread,
// then a fixed tree in LDS.
__global__ __launch_bounds__(256) void reduce_kernel(const double *__restrict__ part, int count,
                                                     double *__restrict__ out)
{
    __shared__ double sh[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < count; i += 256) s += part[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

template <typename T>
__global__ void vacuum_kernel(void *out, int mode, double *sum_p)
{
    using C = typename Cx<T>::type;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (mode == SLOS_MODE_PROB)
            ((T *)out)[0] = (T)1;
        else
            ((C *)out)[0] = C{(T)1, (T)0};
        if (sum_p) *sum_p = 1.0;
    }
}

template <typename T, int MODE, bool COMP>
hipError_t launch_rr(const LayerParams &p, const LayerLaunch &l, hipStream_t s)
{
    dim3 g(l.grid), b(l.threads);
    switch (l.rr) {
    case 1: hipLaunchKernelGGL((layer_kernel<T, MODE, COMP, 1>), g, b, 0, s, p); break;
    case 2: hipLaunchKernelGGL((layer_kernel<T, MODE, COMP, 2>), g, b, 0, s, p); break;
    default: hipLaunchKernelGGL((layer_kernel<T, MODE, COMP, 4>), g, b, 0, s, p); break;
    }
    return hipGetLastError();
}

template <typename T, bool COMP>
hipError_t launch_mode(const LayerParams &p, const LayerLaunch &l, hipStream_t s)
{
    switch (l.mode) {
    case SLOS_MODE_AMPL: return launch_rr<T, SLOS_MODE_AMPL, COMP>(p, l, s);
    case SLOS_MODE_PROB: return launch_rr<T, SLOS_MODE_PROB, COMP>(p, l, s);
    default: return launch_rr<T, SLOS_MODE_MID, COMP>(p, l, s);
    }
}

} // namespace

int slos_launch_layer(const LayerParams &p, const LayerLaunch &l, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (l.c64) {
        if (l.compensated) return (int)launch_mode<float, true>(p, l, s);
        return (int)launch_mode<float, false>(p, l, s);
    }
    return (int)launch_mode<double, false>(p, l, s);
}

int slos_launch_reduce(const double *partials, int count, double *out, void *stream)
{
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, partials, count, out);
    return (int)hipGetLastError();
}

int slos_launch_vacuum(void *out, int c64, int mode, double *sum_p, void *stream)
{
    if (c64)
        hipLaunchKernelGGL(vacuum_kernel<float>, dim3(1), dim3(64), 0, (hipStream_t)stream, out, mode, sum_p);
    else
        hipLaunchKernelGGL(vacuum_kernel<double>, dim3(1), dim3(64), 0, (hipStream_t)stream, out, mode, sum_p);
    return (int)hipGetLastError();
}
