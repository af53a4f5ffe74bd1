// HIP kernels (gfx950): amplitudes of selected outputs only.
//
// The layer recurrence of Section 3.2.3 restricted to one target S: only the
// states t <= S (componentwise) can reach S, so for each target the kernel runs
//     A[0] = 1,  A[t] = sum_{j : t_j > 0} U[j, i_|t|] A[t - e_j]
// over that sub-lattice and returns a(S) = A[S] sqrt(prod s_j!) / sqrt(prod t_i!)
// (Eq. eqperm).  The sub-lattice has R = prod_j (s_j + 1) states, 2^n for an
// output without bunching, instead of the C(m+n-1, n) states of the full
// distribution: the way to a few outputs of a space too large to enumerate.
//
// One workgroup per target.  States are numbered in mixed radix over the
// occupied modes of S (digit q = occupation of the q-th occupied mode, radix
// s_q + 1), so t - e_j is the index minus a stride.  Targets with the same
// multiset of occupations share one table (built on the host): the states
// listed layer by layer, each with the mask of its non-zero digits, read from
// global memory (it stays in cache); the workgroup keeps only A in LDS and
// fills it layer by layer, a barrier between layers.  Each state's terms are
// summed in a fixed order (digits ascending), so results are reproducible.
#include <hip/hip_runtime.h>

#include "slos_ext.h"

namespace {

template <typename T> struct Cs;
template <> struct Cs<float> { using type = float2; };
template <> struct Cs<double> { using type = double2; };

template <typename T>
__global__ __launch_bounds__(256) void select_kernel(SelectParams p)
{
    using C = typename Cs<T>::type;
    extern __shared__ __align__(16) unsigned char lds[];
    C *A = (C *)lds;                                               // R_max states
    __shared__ C uk[SLOS_SELECT_MAX_OCC];                          // U[mode_q, i_k]
    const C *Um = (const C *)p.U;
    const int tid = threadIdx.x, nt = blockDim.x;

    for (int64_t ti = blockIdx.x; ti < p.count; ti += gridDim.x) {
        const SelectTarget &tg = p.targets[ti];
        const SelectPattern &pt = p.patterns[tg.pattern];
        const int nocc = (int)tg.nocc;
        const uint16_t *state = p.state + pt.off;
        const uint32_t *mask = p.mask + pt.off;
        if (tid == 0) A[0] = C{(T)1, (T)0};
        for (int k = 1; k <= p.n; ++k) {
            __syncthreads();  // layer k - 1 complete; uk free
            if (tid < nocc) uk[tid] = Um[(size_t)tg.mode[tid] * p.m + p.cols[k - 1]];
            __syncthreads();
            for (uint32_t i = pt.lstart[k] + tid; i < pt.lstart[k + 1]; i += nt) {
                const uint32_t x = state[i];
                T ar = 0, ai = 0;
                for (uint32_t mk = mask[i]; mk; mk &= mk - 1u) {  // non-zero digits, ascending
                    const int q = __builtin_ctz(mk);
                    const C u = uk[q], v = A[x - pt.stride[q]];
                    ar = fma(u.x, v.x, ar);
                    ar = fma(-u.y, v.y, ar);
                    ai = fma(u.x, v.y, ai);
                    ai = fma(u.y, v.x, ai);
                }
                A[x] = C{ar, ai};
            }
        }
        __syncthreads();
        if (tid == 0) {
            const C a = A[pt.R - 1];
            ((C *)p.out)[ti] = C{(T)((double)a.x * tg.fac), (T)((double)a.y * tg.fac)};
        }
        __syncthreads();  // A is reused by the next target
    }
}

} // namespace

int slos_launch_select(const SelectParams &p, int c64, void *stream)
{
    const size_t es = c64 ? sizeof(float2) : sizeof(double2);
    const size_t lds = (size_t)p.r_max * es;
    const int grid = (int)std::min<int64_t>(std::max<int64_t>(p.count, 1), 4096);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (c64) {
        e = hipFuncSetAttribute((const void *)select_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)SLOS_LDS_DYNAMIC_MAX);
        if (e != hipSuccess) return (int)e;
        hipLaunchKernelGGL(select_kernel<float>, dim3(grid), dim3(256), lds, s, p);
    } else {
        e = hipFuncSetAttribute((const void *)select_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)SLOS_LDS_DYNAMIC_MAX);
        if (e != hipSuccess) return (int)e;
        hipLaunchKernelGGL(select_kernel<double>, dim3(grid), dim3(256), lds, s, p);
    }
    return (int)hipGetLastError();
}
