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
// that group (Eq. eqperm), the mixture is
//     sum_A  prod_{s in A} x (p1 + p2 L_s)  prod_{s not in A} (p0 + (1-x)(p1 L_s + p2 L_s^2))  P_A.
// The L_s commute, so the sum over A folds source by source, a butterfly over
// the subsets: for each subset A' of the sources not yet folded,
//     Q_{A'} = x (p1 + p2 L_s) P_{A' + s} + (p0 + (1-x)(p1 L_s + p2 L_s^2)) P_{A'}
//            = p0 P_{A'} + x p1 P_{A'+s} + L_s Z,
//     Z      = x p2 P_{A'+s} + (1-x) p1 P_{A'} + (1-x) p2 L_s P_{A'},
// two passes of y = gamma L(in) + alpha a + beta b per step, 3 (2^n - 1)
// applications of L in all instead of the 5^n emission events.
//
// The common groups of all 2^n subsets come from a ladder: the recurrence
// vector of A is that of A minus its highest source advanced by one layer (one
// launch per subset size), then squared and normalised into the slots.
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

__global__ __launch_bounds__(256) void src_group_kernel(SrcGroupParams p)
{
    __shared__ double2 uc[256];
    const uint32_t A = p.subsets[blockIdx.y];
    const int top = 31 - __clz(A);
    const uint32_t parent = A & ~(1u << top);
    const int col = p.modes[top];
    const double2 *U = (const double2 *)p.U;
    for (int j = threadIdx.x; j < 256; j += blockDim.x) uc[j] = j < p.m ? U[(size_t)j * p.m + col] : double2{0.0, 0.0};
    __syncthreads();
    const double2 *__restrict__ X = p.amp + p.amp_off[parent];
    double2 *__restrict__ Y = p.amp + p.amp_off[A];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (uint64_t li = p.leaf_lo + (uint64_t)blockIdx.x * nw + wv; li < p.leaf_hi; li += (uint64_t)gridDim.x * nw) {
        const LeafDescNarrow &d = p.desc[li];
        const uint64_t ob = d.h.out_base - p.off_out, lb = d.h.low_base - p.off_in;
        const uint32_t size = d.h.size, nh = d.h.nh, cmax = d.h.cmax;
        const uint32_t *pr = p.pred + d.h.pred_off;
        const double2 *hb[SLOS_NARROW_GROUPS];
        double2 ug[SLOS_NARROW_GROUPS];
#pragma unroll
        for (int g = 0; g < SLOS_NARROW_GROUPS; ++g) {
            const bool on = (uint32_t)g < nh;
            hb[g] = X + (on ? lb - d.delta[g] : lb);
            ug[g] = on ? uc[d.mode[g]] : double2{0.0, 0.0};
        }
        const double2 *lowb = X + lb;
        for (uint32_t x = lane; x < size; x += 64) {
            double re = 0.0, im = 0.0;
#pragma unroll
            for (int g = 0; g < SLOS_NARROW_GROUPS; ++g)
                if ((uint32_t)g < nh) {
                    const double2 v = hb[g][x];
                    re = fma(ug[g].x, v.x, fma(-ug[g].y, v.y, re));
                    im = fma(ug[g].x, v.y, fma(ug[g].y, v.x, im));
                }
            for (uint32_t e = 0; e < cmax; ++e) {
                const uint32_t t = pr[(size_t)e * size + x];
                const double2 u = uc[t >> 24], v = lowb[t & SLOS_PRED_MASK];
                re = fma(u.x, v.x, fma(-u.y, v.y, re));
                im = fma(u.x, v.y, fma(u.y, v.x, im));
            }
            Y[ob + x] = double2{re, im};
        }
    }
}

__global__ __launch_bounds__(256) void src_fill_kernel(SrcFillParams p)
{
    const uint32_t s = blockIdx.y;
    const int k = __popc(s);
    const int64_t ao = p.amp_off[s];
    if (ao < 0 || k > p.nmax) return;
    double *y = p.slots + (size_t)s * p.G;
    if (k == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) y[0] = 1.0;
        return;
    }
    const double2 *a = p.amp + ao;
    const double inv = p.inv_tfac[s];
    const uint64_t base = p.off[k];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (uint64_t li = p.leaves_upto[k - 1] + (uint64_t)blockIdx.x * nw + wv; li < p.leaves_upto[k];
         li += (uint64_t)gridDim.x * nw) {
        const LeafDescNarrow &d = p.desc[li];
        const uint64_t ob = d.h.out_base;  // graded rank
        const double fh = d.h.fac_hi * d.h.fac_hi * inv;
        const double *lf = p.lowfac + d.h.fac_off;
        const uint32_t size = d.h.size;
        for (uint32_t x = lane; x < size; x += 64) {
            const double2 z = a[ob - base + x];
            const double f = lf[x];
            y[ob + x] = (z.x * z.x + z.y * z.y) * (fh * f * f);
        }
    }
}

__device__ __forceinline__ bool in_support(int k, int c, int lo, int len, int nmax)
{
    return k >= c + lo && k <= min(nmax, c + lo + len);
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
    const int c = __popc(r);
    if (blockIdx.x == 0 && threadIdx.x == 0 && c == 0) {
        double v = 0.0;
        if (in_support(0, c, p.a_lo, p.a_len, p.nmax)) v += p.alpha * a[0];
        if (in_support(0, c, p.b_lo, p.b_len, p.nmax)) v += p.beta * b[0];
        y[0] = v;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (uint64_t li = (uint64_t)blockIdx.x * nw + wv; li < p.nleaves; li += (uint64_t)gridDim.x * nw) {
        const LeafDescNarrow &d = p.desc[li];
        const int k = (int)d.h.pad;
        if (!in_support(k, c, 0, p.y_len, p.nmax)) continue;
        const bool useL = in_support(k - 1, c, p.in_lo, p.in_len, p.nmax);
        const double ca = in_support(k, c, p.a_lo, p.a_len, p.nmax) ? p.alpha : 0.0;
        const double cb = in_support(k, c, p.b_lo, p.b_len, p.nmax) ? p.beta : 0.0;
        const uint64_t ob = d.h.out_base, lb = d.h.low_base;
        const uint32_t size = d.h.size;
        const uint32_t nh = useL ? d.h.nh : 0u, cmax = useL ? d.h.cmax : 0u;
        const uint32_t *pr = p.pred + d.h.pred_off;
        // the leaf's groups in registers: the stores to y below may alias the
        // descriptor as far as the compiler knows, which would reload it per output
        const double *hb[SLOS_NARROW_GROUPS];
        double wg[SLOS_NARROW_GROUPS];
#pragma unroll
        for (int g = 0; g < SLOS_NARROW_GROUPS; ++g) {
            const bool on = (uint32_t)g < nh;
            hb[g] = in + (on ? lb - d.delta[g] : lb);
            wg[g] = on ? W[d.mode[g]] : 0.0;
        }
        const double *lowb = in + lb;
        // two outputs per lane and step (x and x + 64): twice the loads in flight
        for (uint32_t x0 = lane; x0 < size; x0 += 128) {
            const uint32_t x1 = x0 + 64;
            const bool two = x1 < size;
            const uint32_t x1c = two ? x1 : x0;
            double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
            for (int g = 0; g < SLOS_NARROW_GROUPS; ++g)
                if ((uint32_t)g < nh) {
                    acc0 = fma(wg[g], hb[g][x0], acc0);
                    acc1 = fma(wg[g], hb[g][x1c], acc1);
                }
            for (uint32_t e = 0; e < cmax; ++e) {
                const uint32_t t0 = pr[(size_t)e * size + x0], t1 = pr[(size_t)e * size + x1c];
                acc0 = fma(W[t0 >> 24], lowb[t0 & SLOS_PRED_MASK], acc0);
                acc1 = fma(W[t1 >> 24], lowb[t1 & SLOS_PRED_MASK], acc1);
            }
            double v0 = p.gamma * acc0, v1 = p.gamma * acc1;
            if (ca != 0.0) {
                v0 += ca * a[ob + x0];
                v1 += ca * a[ob + x1c];
            }
            if (cb != 0.0) {
                v0 += cb * b[ob + x0];
                v1 += cb * b[ob + x1c];
            }
            y[ob + x0] = v0;
            if (two) y[ob + x1] = v1;
        }
    }
}

// Block i sums the states [i * chunk, (i + 1) * chunk) of its photon number k
// (blocks blk_off[k] .. blk_off[k+1] - 1 cover photon number k) in a fixed order
// into (mass, physical, kept); src_stats_final adds each number's blocks in order.
__global__ __launch_bounds__(256) void src_stats_kernel(SrcStatsParams p)
{
    __shared__ int8_t grp[256];
    __shared__ double red[3][256];
    extern __shared__ uint64_t bin[];  // C(a, r) for a < m + nmax - 1, r <= nmax (dynamic)
    const int tid = threadIdx.x;
    grp[tid] = p.group[tid];
    const int bs = p.bstride, na = (p.m + p.nmax - 1) * bs;
    for (int i = tid; i < na; i += blockDim.x) bin[i] = p.binom[i];
    __syncthreads();
    int k = 0;
    while (blockIdx.x >= p.blk_off[k + 1]) ++k;
    const uint64_t lo = p.off[k], n = p.off[k + 1] - lo;
    const uint64_t c0 = min(n, (uint64_t)(blockIdx.x - p.blk_off[k]) * p.chunk), c1 = min(n, c0 + p.chunk);
    double mass = 0.0, phys = 0.0, kept = 0.0;
    for (uint64_t i = c0 + tid; i < c1; i += blockDim.x) {
        const double v = p.P[lo + i];
        mass += v;
        // colex unrank, top photon first: rank = sum_r C(d_r + r - 1, r); group
        // counts in 8-bit fields (groups 0-7 in g0, 8-15 in g1)
        uint64_t rank = i, g0 = 0, g1 = 0;
        int c = p.m + k - 2, prev = -1, occ = 0;
        for (int r = k; r >= 1; --r) {
            while (c >= r && bin[c * bs + r] > rank) --c;
            if (c < r - 1) c = r - 1;
            if (c >= r) rank -= bin[c * bs + r];
            const int d = c - r + 1;
            occ += d != prev;
            prev = d;
            const int g = grp[d];
            if (g >= 0) {
                if (g < 8) g0 += uint64_t(1) << (8 * g);
                else g1 += uint64_t(1) << (8 * (g - 8));
            }
            --c;  // the next photon's c_{r-1} = d_{r-1} + r - 2 <= c_r - 1
        }
        if (occ >= p.min_modes) {
            phys += v;
            bool ok = true;
            for (int g = 0; g < p.ngroups; ++g) {
                const uint32_t cnt = (uint32_t)(((g < 8 ? g0 : g1) >> (8 * (g & 7))) & 0xFFu);
                ok = ok && cnt >= p.cmin[g] && cnt <= p.cmax[g];
            }
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
    if (tid < 3) p.partials[(size_t)blockIdx.x * 3 + tid] = red[tid][0];
}

__global__ __launch_bounds__(256) void src_stats_final(SrcStatsParams p)
{
    __shared__ double red[3][256];
    const int k = blockIdx.x, tid = threadIdx.x;
    for (int q = 0; q < 3; ++q) {
        double s = 0.0;
        for (uint32_t i = p.blk_off[k] + tid; i < p.blk_off[k + 1]; i += blockDim.x) s += p.partials[(size_t)i * 3 + q];
        red[q][tid] = s;
    }
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h)
            for (int q = 0; q < 3; ++q) red[q][tid] += red[q][tid + h];
        __syncthreads();
    }
    if (tid < 3) p.result[k * 3 + tid] = red[tid][0];
}

} // namespace

int slos_launch_src_group(const SrcGroupParams &p, int nsub, void *stream)
{
    const uint64_t blocks = std::min<uint64_t>((p.leaf_hi - p.leaf_lo + 3) / 4, 1024);
    hipLaunchKernelGGL(src_group_kernel, dim3((unsigned)std::max<uint64_t>(blocks, 1), nsub), dim3(256), 0,
                       (hipStream_t)stream, p);
    return (int)hipGetLastError();
}

int slos_launch_src_fill(const SrcFillParams &p, int nslots, void *stream)
{
    uint64_t most = 1;
    for (int k = 1; k <= p.nmax; ++k) most = std::max<uint64_t>(most, p.leaves_upto[k] - p.leaves_upto[k - 1]);
    const uint64_t blocks = std::min<uint64_t>((most + 3) / 4, 1024);
    hipLaunchKernelGGL(src_fill_kernel, dim3((unsigned)blocks, nslots), dim3(256), 0, (hipStream_t)stream, p);
    return (int)hipGetLastError();
}

int slos_launch_src_pass(const SrcPassParams &p, int npairs, void *stream)
{
    const uint64_t blocks = std::min<uint64_t>((p.nleaves + 3) / 4, 4096);
    hipLaunchKernelGGL(src_pass_kernel, dim3((unsigned)std::max<uint64_t>(blocks, 1), npairs), dim3(256), 0,
                       (hipStream_t)stream, p);
    return (int)hipGetLastError();
}

int slos_launch_src_stats(const SrcStatsParams &p, void *stream)
{
    const size_t lds = (size_t)(p.m + p.nmax - 1) * p.bstride * sizeof(uint64_t);
    hipLaunchKernelGGL(src_stats_kernel, dim3(p.blk_off[p.nmax + 1]), dim3(256), lds, (hipStream_t)stream, p);
    hipLaunchKernelGGL(src_stats_final, dim3(p.nmax + 1), dim3(256), 0, (hipStream_t)stream, p);
    return (int)hipGetLastError();
}
