// HIP kernels (gfx950): output distribution of an imperfect single-photon
// source (Section 3.2.4: emission probability, pair emission, indistinguish-
// ability; Appendix A.4 prints its effect on the Ralph CNOT).
//
// Every photon of the input comes from a source of its own.  Source s emits
// nothing (p0), one photon (p1) or two (p2); an emitted first photon is in
// the common wavepacket with probability x = sqrt(V), else distinguishable
// from everything, and a second photon is always distinguishable.  Photons of
// different wavepackets do not interfere, so an emission event's law is the
// convolution of its groups' laws.  A distinguishable photon entering mode i
// acts on a probability vector over Fock states as
//     (L_i P)[t] = sum_{j : t_j > 0} |U[j, i]|^2 P[t - e_j],
// the layer recurrence of Section 3.2.3 on probabilities with real weights.
// With A the set of sources whose first photon is common and P_A the law of
// that group (Eq. eqperm, computed by the batch kernel), the mixture is
//     sum_A  prod_{s in A} x (p1 + p2 L_s)  prod_{s not in A} (p0 + (1-x)(p1 L_s + p2 L_s^2))  P_A.
// The L_s commute, so the sum over A folds source by source, a butterfly over
// the subsets: for each subset A' of the sources not yet folded,
//     Q_{A'} = x (p1 + p2 L_s) P_{A' + s} + (p0 + (1-x)(p1 L_s + p2 L_s^2)) P_{A'}
//            = p0 P_{A'} + x p1 P_{A'+s} + L_s Z,
//     Z      = x p2 P_{A'+s} + (1-x) p1 P_{A'} + (1-x) p2 L_s P_{A'},
// two passes of y = gamma L(in) + alpha a + beta b per step, 3 (2^n - 1)
// applications of L in all instead of the 5^n emission events.
//
// Vectors are graded: photon numbers 0..nmax, each in colex order, one after
// the other.  The L pass walks the leaves of photon numbers 1..nmax (the leaf
// descriptors of the layer kernel, ranks shifted to the graded layout): one
// wave per leaf, lane x takes output x, predecessors through the leaf's fixed
// high modes are whole blocks at the same inner position (coalesced), those
// through its low modes come from the inner table.  FP64 throughout.
#include <hip/hip_runtime.h>

#include "slos_ext.h"

namespace {

__global__ __launch_bounds__(256) void src_fill_kernel(SrcFillParams p)
{
    const uint32_t s = blockIdx.y;
    double *y = p.slots + (size_t)s * p.G;
    const int k = __popc(s);
    const int64_t ao = p.amp_off[s];
    const uint64_t lo = (ao >= 0 && k <= p.nmax) ? p.off[k] : p.G;
    const uint64_t hi = (ao >= 0 && k <= p.nmax) ? p.off[k + 1] : p.G;
    const double2 *a = (const double2 *)p.amp + (ao >= 0 ? ao : 0);
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < p.G;
         g += (uint64_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        if (g >= lo && g < hi) {
            const double2 z = a[g - lo];
            v = z.x * z.x + z.y * z.y;
        }
        y[g] = v;
    }
}

__global__ __launch_bounds__(256) void src_pass_kernel(SrcPassParams p)
{
    __shared__ double W[256];
    const double2 *U = (const double2 *)p.U;
    for (int j = threadIdx.x; j < 256; j += blockDim.x) {
        double w = 0.0;
        if (j < p.m) {
            const double2 u = U[(size_t)j * p.m + p.col];
            w = u.x * u.x + u.y * u.y;
        }
        W[j] = w;  // W[SLOS_ZERO_MODE] stays 0 (m <= 255)
    }
    __syncthreads();
    const uint32_t r = blockIdx.y;
    const double *__restrict__ in = p.in + (size_t)r * p.s_in;
    const double *a = p.a + (size_t)r * p.s_a;
    const double *b = p.b + (size_t)r * p.s_b;
    double *y = p.y + (size_t)r * p.s_y;
    const int klo = __popc(r);
    const int khi = min(p.nmax, klo + p.span);
    const uint64_t glo = klo <= p.nmax ? p.off[klo] : p.off[p.nmax + 1];
    const uint64_t ghi = p.off[khi + 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) y[0] = klo == 0 ? p.alpha * a[0] + p.beta * b[0] : 0.0;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (uint64_t li = (uint64_t)blockIdx.x * nw + wv; li < p.nleaves; li += (uint64_t)gridDim.x * nw) {
        const LeafDescNarrow &d = p.desc[li];
        const uint64_t ob = d.h.out_base, lb = d.h.low_base;
        const uint32_t size = d.h.size;
        if (ob < glo || ob >= ghi) {  // photon number outside the support of y
            for (uint32_t x = lane; x < size; x += 64) y[ob + x] = 0.0;
            continue;
        }
        const uint32_t nh = d.h.nh, cmax = d.h.cmax;
        const uint32_t *pr = p.pred + d.h.pred_off;
        for (uint32_t x = lane; x < size; x += 64) {
            double acc = 0.0;
            for (uint32_t g = 0; g < nh; ++g) acc = fma(W[d.mode[g]], in[lb - d.delta[g] + x], acc);
            for (uint32_t c = 0; c < cmax; ++c) {
                const uint32_t e = pr[(size_t)c * size + x];
                acc = fma(W[e >> 24], in[lb + (e & SLOS_PRED_MASK)], acc);
            }
            y[ob + x] = p.gamma * acc + p.alpha * a[ob + x] + p.beta * b[ob + x];
        }
    }
}

// Per photon number k = blockIdx.y: block blockIdx.x sums a fixed chunk of
// [off[k], off[k+1]) in a fixed order into (mass, physical, kept).
__global__ __launch_bounds__(256) void src_stats_kernel(SrcStatsParams p)
{
    __shared__ int8_t grp[256];
    __shared__ uint8_t gc[256][SLOS_PS_MAX_GROUPS];
    __shared__ double red[3][256];
    const int tid = threadIdx.x;
    grp[tid] = p.group[tid];
    __syncthreads();
    const int k = blockIdx.y;
    const uint64_t lo = p.off[k], n = p.off[k + 1] - lo;
    const uint64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const uint64_t c0 = min(n, (uint64_t)blockIdx.x * chunk), c1 = min(n, c0 + chunk);
    double mass = 0.0, phys = 0.0, kept = 0.0;
    for (uint64_t i = c0 + tid; i < c1; i += blockDim.x) {
        const double v = p.P[lo + i];
        mass += v;
        // colex unrank: the top photon's mode first, rank = sum_r C(d_r + r - 1, r)
        for (int g = 0; g < p.ngroups; ++g) gc[tid][g] = 0;
        uint64_t rank = i;
        int c = p.m + k - 2, prev = -1, occ = 0;
        for (int r = k; r >= 1; --r) {
            while (c >= r && p.binom[(size_t)c * p.bstride + r] > rank) --c;
            if (c < r - 1) c = r - 1;
            if (c >= r) rank -= p.binom[(size_t)c * p.bstride + r];
            const int d = c - r + 1;
            occ += d != prev;
            prev = d;
            const int g = grp[d];
            if (g >= 0) gc[tid][g] += 1;
            --c;  // the next photon's c_{r-1} = d_{r-1} + r - 2 <= c_r - 1
        }
        if (occ >= p.min_modes) {
            phys += v;
            bool ok = true;
            for (int g = 0; g < p.ngroups; ++g) ok = ok && gc[tid][g] >= p.cmin[g] && gc[tid][g] <= p.cmax[g];
            if (ok) kept += v;
        }
    }
    red[0][tid] = mass;
    red[1][tid] = phys;
    red[2][tid] = kept;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h)
            for (int q = 0; q < 3; ++q) red[q][tid] += red[q][tid + h];
        __syncthreads();
    }
    if (tid < 3) p.partials[((size_t)k * gridDim.x + blockIdx.x) * 3 + tid] = red[tid][0];
}

__global__ __launch_bounds__(256) void src_stats_final(const double *__restrict__ part, int nb,
                                                       double *__restrict__ result)
{
    __shared__ double red[3][256];
    const int k = blockIdx.x, tid = threadIdx.x;
    for (int q = 0; q < 3; ++q) {
        double s = 0.0;
        for (int i = tid; i < nb; i += blockDim.x) s += part[((size_t)k * nb + i) * 3 + q];
        red[q][tid] = s;
    }
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h)
            for (int q = 0; q < 3; ++q) red[q][tid] += red[q][tid + h];
        __syncthreads();
    }
    if (tid < 3) result[k * 3 + tid] = red[tid][0];
}

} // namespace

int slos_launch_src_fill(const SrcFillParams &p, int nslots, void *stream)
{
    const uint64_t blocks = std::min<uint64_t>((p.G + 255) / 256, 1024);
    hipLaunchKernelGGL(src_fill_kernel, dim3((unsigned)std::max<uint64_t>(blocks, 1), nslots), dim3(256), 0,
                       (hipStream_t)stream, p);
    return (int)hipGetLastError();
}

int slos_launch_src_pass(const SrcPassParams &p, int npairs, void *stream)
{
    const uint64_t blocks = std::min<uint64_t>((p.nleaves + 3) / 4, 2048);
    hipLaunchKernelGGL(src_pass_kernel, dim3((unsigned)std::max<uint64_t>(blocks, 1), npairs), dim3(256), 0,
                       (hipStream_t)stream, p);
    return (int)hipGetLastError();
}

int slos_launch_src_stats(const SrcStatsParams &p, void *stream)
{
    hipLaunchKernelGGL(src_stats_kernel, dim3(SLOS_SRC_STATS_BLOCKS, p.nmax + 1), dim3(256), 0, (hipStream_t)stream,
                       p);
    hipLaunchKernelGGL(src_stats_final, dim3(p.nmax + 1), dim3(256), 0, (hipStream_t)stream, p.partials,
                       SLOS_SRC_STATS_BLOCKS, p.result);
    return (int)hipGetLastError();
}
