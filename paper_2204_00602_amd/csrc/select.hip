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
// occupied modes of S (digit p = occupation of the p-th occupied mode, radix
// s_p + 1), so t - e_j is the index minus a stride.  The workgroup keeps A, the
// mask of non-zero digits of every state and the state indices sorted by layer
// |t| (a counting sort) in LDS, and fills A layer by layer, each layer touching
// only its own states, a barrier between layers; each state's terms are summed
// in a fixed order (digits ascending), so results are reproducible.
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
    extern __shared__ unsigned char lds[];
    C *A = (C *)lds;                                               // R_max states
    uint32_t *mask = (uint32_t *)(lds + (size_t)p.r_max * sizeof(C));
    uint16_t *order = (uint16_t *)(mask + p.r_max);                // states sorted by layer
    uint8_t *layer = (uint8_t *)(order + p.r_max);
    __shared__ C uk[SLOS_SELECT_MAX_OCC];                          // U[mode_p, i_k]
    __shared__ uint32_t stride[SLOS_SELECT_MAX_OCC];
    __shared__ uint32_t lcount[SLOS_MAX_PHOTONS + 2], lstart[SLOS_MAX_PHOTONS + 2];
    const C *Um = (const C *)p.U;
    const int tid = threadIdx.x, nt = blockDim.x;

    for (int64_t ti = blockIdx.x; ti < p.count; ti += gridDim.x) {
        const SelectTarget tg = p.targets[ti];
        const uint32_t R = tg.R;
        const int nocc = tg.nocc;
        if (tid < nocc) {
            uint32_t st = 1;
            for (int q = 0; q < tid; ++q) st *= (uint32_t)tg.mult[q] + 1u;
            stride[tid] = st;
        }
        if (tid <= p.n + 1) lcount[tid] = 0;
        __syncthreads();
        // layer and mask of non-zero digits of every state; thread tid takes
        // states tid, tid + nt, ... so that the lanes of a wave touch
        // consecutive LDS words
        for (uint32_t x = tid; x < R; x += nt) {
            uint32_t rest = x, mk = 0, k = 0;
            for (int q = 0; q < nocc; ++q) {
                const uint32_t rad = (uint32_t)tg.mult[q] + 1u;
                const uint32_t dq = rest % rad;
                rest /= rad;
                k += dq;
                mk |= (dq ? 1u : 0u) << q;
            }
            mask[x] = mk;
            layer[x] = (uint8_t)k;
            atomicAdd(&lcount[k], 1u);
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t run = 0;
            for (int k = 0; k <= p.n; ++k) {
                lstart[k] = run;
                run += lcount[k];
                lcount[k] = lstart[k];  // becomes the scatter cursor
            }
            lstart[p.n + 1] = run;
        }
        __syncthreads();
        // counting sort by layer (the order within a layer does not matter:
        // each state is computed by one thread, its terms in a fixed order)
        for (uint32_t x = tid; x < R; x += nt) order[atomicAdd(&lcount[layer[x]], 1u)] = (uint16_t)x;
        if (tid == 0) A[0] = C{(T)1, (T)0};
        for (int k = 1; k <= p.n; ++k) {
            __syncthreads();  // layer k - 1 complete (and the sort, for k = 1); uk free
            if (tid < nocc) uk[tid] = Um[(size_t)tg.mode[tid] * p.m + p.cols[k - 1]];
            __syncthreads();
            for (uint32_t i = lstart[k] + tid; i < lstart[k + 1]; i += nt) {
                const uint32_t x = order[i];
                T ar = 0, ai = 0;
                for (uint32_t mk = mask[x]; mk; mk &= mk - 1u) {  // occupied digits, ascending
                    const int q = __builtin_ctz(mk);
                    const C u = uk[q], v = A[x - stride[q]];
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
            const C a = A[R - 1];
            ((C *)p.out)[ti] = C{(T)((double)a.x * tg.fac), (T)((double)a.y * tg.fac)};
        }
        __syncthreads();  // A, mask, order and layer are reused by the next target
    }
}

} // namespace

int slos_launch_select(const SelectParams &p, int c64, void *stream)
{
    const size_t es = c64 ? sizeof(float2) : sizeof(double2);
    const size_t lds = (size_t)p.r_max * (es + 4 + 2 + 1);
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
