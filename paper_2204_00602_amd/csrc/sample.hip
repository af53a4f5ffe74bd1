// HIP kernels (gfx950): weak simulation from the strong one.
//
// The sampler the paper builds on its strong back-ends (Section 3.2) draws
// outputs S with probability P(S).  From the full distribution in colex order
// this is an inverse-CDF lookup: for a uniform r in [0, 1) the sample is the
// first S whose cumulative probability exceeds r * sum P.  The same prefix sums
// give the partial certificate of Eq. eqpk: P(K), the probability that modes
// K..m-1 are empty, is the sum over the first C(K+n-1, n) states (those states
// form a colex prefix).
//
// Layout: P is cut into blocks of SLOS_CDF_BLOCK states.  cdf_block_kernel sums
// each block in FP64 (one wave per block, fixed order); runs of SLOS_CDF_BLOCK
// block sums are summed again, those few run sums are scanned in one
// workgroup, and cdf_fix_kernel turns the block sums into the exclusive prefix
// bp[0..nb] (bp[nb] = sum P), every step in a fixed order, so the table is
// reproducible; the run prefixes stay after the table (sp = bp + nb + 1), and
// the block kernel also keeps the sums of each block's 16 chunks of 64 states
// (cs = sp + nsup + 1), and a last pass copies every 16^l-th prefix into a
// 16-ary search tree (after cs).  A sample takes 16 lanes, so a wave serves
// four at once: it descends the tree, each level one 16-way step over 16
// consecutive prefixes (one cache line), to its block, finds its chunk from the
// block's 16 chunk sums (one line), and then its state with a 16-lane scan of
// that chunk's 64 probabilities (four per lane): about 1 KB per sample.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "slos_ext.h"

namespace {

constexpr int kChunks = SLOS_CDF_BLOCK / 64;

typedef float cdf_f4 __attribute__((ext_vector_type(4)));
typedef double cdf_d2 __attribute__((ext_vector_type(2)));

// Block b is read in SLOS_CDF_BLOCK / 256 steps of 256 consecutive states: in
// step i lane l holds states 256 i + 4 l .. 256 i + 4 l + 3 (one 16-byte load
// for fp32, two for fp64), so each load of the wave covers one contiguous KiB
// (fp32).  part[i] = the lane's sum of its four states of step i.
constexpr int kSteps = SLOS_CDF_BLOCK / 256;

template <typename T>
__device__ __forceinline__ void lane_parts(const T *__restrict__ P, int64_t M, int64_t b, int lane, bool full,
                                           double *part)
{
    const int64_t base = b * SLOS_CDF_BLOCK + 4 * (int64_t)lane;
    if (full) {
        if constexpr (sizeof(T) == 4) {
            cdf_f4 v[kSteps];
#pragma unroll
            for (int i = 0; i < kSteps; ++i) v[i] = __builtin_nontemporal_load((const cdf_f4 *)(P + base + 256 * i));
#pragma unroll
            for (int i = 0; i < kSteps; ++i)
                part[i] = ((double)v[i].x + (double)v[i].y) + ((double)v[i].z + (double)v[i].w);
        } else {
            cdf_d2 v[2 * kSteps];
#pragma unroll
            for (int i = 0; i < kSteps; ++i) {
                v[2 * i] = __builtin_nontemporal_load((const cdf_d2 *)(P + base + 256 * i));
                v[2 * i + 1] = __builtin_nontemporal_load((const cdf_d2 *)(P + base + 256 * i) + 1);
            }
#pragma unroll
            for (int i = 0; i < kSteps; ++i)
                part[i] = (v[2 * i].x + v[2 * i].y) + (v[2 * i + 1].x + v[2 * i + 1].y);
        }
    } else {
        for (int i = 0; i < kSteps; ++i) {
            double s = 0.0;
            for (int e = 0; e < 4; ++e) {
                const int64_t x = base + 256 * i + e;
                if (x < M) s += (double)P[x];
            }
            part[i] = s;
        }
    }
}

// block sum bp[b] and the block's 16 chunk sums from the lanes' parts: chunk
// 4 i + g (64 states) is step i of lanes 16 g .. 16 g + 15
__device__ __forceinline__ void block_finish(const double *part, int64_t b, int lane, double *__restrict__ bp,
                                             double *__restrict__ cs)
{
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kSteps; ++i) {
        double c = part[i];
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) c += __shfl_xor(c, o, 64);
        if ((lane & 15) == 0) cs[b * kChunks + 4 * i + (lane >> 4)] = c;
        s += part[i];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) bp[b] = s;
}

// One wave per pair of blocks (b, b + nw) per step: both blocks' loads are in
// flight together.
template <typename T>
__global__ __launch_bounds__(256) void cdf_block_kernel(const T *__restrict__ P, int64_t M, int64_t nb,
                                                        double *__restrict__ bp, double *__restrict__ cs)
{
    static_assert(SLOS_CDF_BLOCK == 1024, "16 chunks of 64 states in 4 steps of 256");
    const int lane = threadIdx.x & 63;
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t nfull = M / SLOS_CDF_BLOCK;  // blocks without a tail
    for (int64_t b0 = gw; b0 < nb; b0 += 2 * nw) {
        const int64_t b1 = b0 + nw;
        double p0[kSteps], p1[kSteps];
        lane_parts(P, M, b0, lane, b0 < nfull, p0);
        if (b1 < nb) lane_parts(P, M, b1, lane, b1 < nfull, p1);
        block_finish(p0, b0, lane, bp, cs);
        if (b1 < nb) block_finish(p1, b1, lane, bp, cs);
    }
}

// Sum of each run of SLOS_CDF_BLOCK consecutive entries of v[0..nv): one wave per run.
__global__ __launch_bounds__(256) void cdf_super_kernel(const double *__restrict__ v, int64_t nv, int64_t nsup,
                                                        double *__restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t b = gw; b < nsup; b += nw) {
        double s = 0.0;
        for (int i = 0; i < kChunks; ++i) {
            const int64_t x = b * SLOS_CDF_BLOCK + i * 64 + lane;
            if (x < nv) s += v[x];
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) out[b] = s;
    }
}

// In place, one workgroup: v[0..nv) -> exclusive prefix, v[nv] = total.
__global__ __launch_bounds__(1024) void cdf_scan_kernel(double *__restrict__ v, int64_t nv)
{
    __shared__ double part[1024];
    const int t = threadIdx.x;
    const int64_t per = (nv + 1023) / 1024;
    const int64_t lo = min((int64_t)t * per, nv), hi = min(lo + per, nv);
    double s = 0.0;
    for (int64_t i = lo; i < hi; ++i) s += v[i];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        double run = 0.0;
        for (int i = 0; i < 1024; ++i) {
            const double x = part[i];
            part[i] = run;
            run += x;
        }
        v[nv] = run;
    }
    __syncthreads();
    double run = part[t];
    for (int64_t i = lo; i < hi; ++i) {
        const double x = v[i];
        v[i] = run;
        run += x;
    }
}

// Block sums -> exclusive prefix: each wave takes one run of SLOS_CDF_BLOCK
// block sums, starts from that run's prefix sp[run] and scans it in chunks of
// 64 (wave scans in a fixed order).  bp[nb] = total.
__global__ __launch_bounds__(256) void cdf_fix_kernel(double *__restrict__ bp, int64_t nb,
                                                      const double *__restrict__ sp, int64_t nsup)
{
    const int lane = threadIdx.x & 63;
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t b = gw; b < nsup; b += nw) {
        double run = sp[b];
        for (int i = 0; i < kChunks; ++i) {
            const int64_t x = b * SLOS_CDF_BLOCK + i * 64 + lane;
            const double v = x < nb ? bp[x] : 0.0;
            double c = v;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const double u = __shfl_up(c, o, 64);
                if (lane >= o) c += u;
            }
            if (x < nb) bp[x] = run + (c - v);
            run += __shfl(c, 63, 64);
        }
    }
    if (gw == 0 && lane == 0) bp[nb] = sp[nsup];
}

// Levels 1.. of the search tree: level l entry i = bp[i * 16^l].
__global__ __launch_bounds__(256) void cdf_tree_kernel(const double *__restrict__ bp, double *__restrict__ tree,
                                                       CdfTree t)
{
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ni = (int64_t)gridDim.x * blockDim.x;
    for (int l = 1; l < t.nlev; ++l) {
        int64_t stride = 1;
        for (int q = 0; q < l; ++q) stride *= 16;
        for (int64_t i = i0; i < t.n[l]; i += ni) tree[t.off[l] + i] = bp[i * stride];
    }
}

// pk[K-1] = sum of P over the first ends[K-1] states, K = 1..m; one wave per K.
template <typename T>
__global__ __launch_bounds__(256) void marginal_kernel(const T *__restrict__ P, const double *__restrict__ bp,
                                                       const int64_t *__restrict__ ends, int m,
                                                       double *__restrict__ pk)
{
    const int lane = threadIdx.x & 63;
    const int K = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (K >= m) return;
    const int64_t e = ends[K];
    const int64_t b = e / SLOS_CDF_BLOCK;
    double s = 0.0;
    for (int64_t x = b * SLOS_CDF_BLOCK + lane; x < e; x += 64) s += (double)P[x];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) pk[K] = bp[b] + s;
}

// Four samples per wave, 16 lanes each: ranks[s] = first state whose
// cumulative P exceeds r[s] * total.  A group's lanes hold the same search state;
// each step is one load instruction for all four groups.
template <typename T>
__global__ __launch_bounds__(256) void sample_kernel(const T *__restrict__ P, int64_t M, const double *__restrict__ bp,
                                                     int64_t nb, const double *__restrict__ r, int64_t count,
                                                     int64_t *__restrict__ ranks, CdfTree tr)
{
    const int64_t nsup = (nb + SLOS_CDF_BLOCK - 1) / SLOS_CDF_BLOCK;
    const double *__restrict__ sp = bp + nb + 1;  // run prefixes, nsup + 1 entries
    const double *__restrict__ cs = sp + nsup + 1;  // chunk sums, kChunks per block
    const double *__restrict__ tree = cs + kChunks * nb;
    const int lane = threadIdx.x & 63, g = lane >> 4, l16 = lane & 15;
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    const double total = bp[nb];
    // the group's 16 bits of a wave ballot
    auto gbits = [&](bool pred) -> uint32_t { return (uint32_t)((__ballot(pred) >> (16 * g)) & 0xFFFFu); };
    for (int64_t s0 = gw * 4; s0 < count; s0 += nw * 4) {
        const int64_t sidx = s0 + g;
        const bool live = sidx < count;
        const double t = r[live ? sidx : s0] * total;
        // down the tree: at each level the largest entry <= t among the 16
        // children of the choice above (the tables are non-decreasing and
        // start at 0 <= t, so the predicate holds on a prefix)
        int64_t lo = 0;
        for (int l = tr.nlev - 1; l >= 0; --l) {
            const double *tab = l == 0 ? bp : tree + tr.off[l];
            const int64_t first = lo * 16;  // < n[l]: entry lo above is bp[lo * 16^(l+1)]
            const int64_t end = min(first + 16, tr.n[l]);
            const uint32_t bal = gbits(first + l16 < end && tab[first + l16] <= t);
            lo = first + (bal ? 31 - __builtin_clz(bal) : 0);  // lane 0 of the group holds: tab[first] <= t
        }
        // the block's chunk sums (one line): the first chunk whose running sum
        // exceeds t, else the last chunk of non-zero probability
        const int64_t base = lo * SLOS_CDF_BLOCK;
        const double c_own = cs[lo * kChunks + l16];
        double c_inc = c_own;
#pragma unroll
        for (int o = 1; o < kChunks; o <<= 1) {
            const double u = __shfl_up(c_inc, o, 16);
            if (l16 >= o) c_inc += u;
        }
        const double b0 = bp[lo];
        const uint32_t c_cross = gbits(b0 + c_inc > t && c_own > 0.0);
        const uint32_t c_pos = gbits(c_own > 0.0);
        const int i0 = c_cross ? __builtin_ctz(c_cross) : (c_pos ? 31 - __builtin_clz(c_pos) : 0);
        double run = b0 + __shfl(c_inc - c_own, i0, 16);
        // then the states of the chunks from i0 on, four per lane (rounding
        // between the chunk sums and this scan can move the crossing on to a
        // later chunk)
        int64_t found = -1, last_pos = -1;
        int ci = i0;
        for (int it = 0; it < kChunks; ++it) {
            const bool open = found < 0 && ci < kChunks;
            if (!__ballot(open)) break;
            double v[4];
            const int64_t x0 = base + (int64_t)ci * 64 + 4 * l16;
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = (open && x0 + e < M) ? (double)P[x0 + e] : 0.0;
            double in[4];
            in[0] = v[0];
#pragma unroll
            for (int e = 1; e < 4; ++e) in[e] = in[e - 1] + v[e];
            double lsum = in[3];  // exclusive prefix of the lanes' sums over the group
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) {
                const double u = __shfl_up(lsum, o, 16);
                if (l16 >= o) lsum += u;
            }
            const double excl = lsum - in[3];
            int first_e = -1, last_e = -1;
#pragma unroll
            for (int e = 3; e >= 0; --e) {
                if (v[e] > 0.0 && run + excl + in[e] > t) first_e = e;
                if (last_e < 0 && v[e] > 0.0) last_e = e;
            }
            const uint32_t cross = gbits(open && first_e >= 0);
            const uint32_t pos = gbits(open && last_e >= 0);
            if (open) {
                if (cross) {
                    const int src = __builtin_ctz(cross);
                    found = base + (int64_t)ci * 64 + 4 * src + __shfl(first_e, src, 16);
                }
                if (pos) {
                    const int src = 31 - __builtin_clz(pos);
                    last_pos = base + (int64_t)ci * 64 + 4 * src + __shfl(last_e, src, 16);
                }
                run += __shfl(lsum, 15, 16);  // shuffles stay within the group, all of whose lanes are here
                ++ci;
            }
        }
        // rounding can leave the crossing past the block's recomputed sum:
        // take the block's last state of non-zero probability
        if (found < 0) found = last_pos >= 0 ? last_pos : min(base, M - 1);
        if (l16 == 0 && live) ranks[sidx] = found;
    }
}

} // namespace

int slos_launch_cdf(const void *P, int c64, int64_t M, double *bp, void *stream)
{
    const int64_t nb = (M + SLOS_CDF_BLOCK - 1) / SLOS_CDF_BLOCK;
    const int64_t nsup = (nb + SLOS_CDF_BLOCK - 1) / SLOS_CDF_BLOCK;
    double *sp = bp + nb + 1;    // nsup + 1 run prefixes after the table
    double *cs = sp + nsup + 1;  // then 16 chunk sums per block
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((nb + 3) / 4, 8192));
    const int gsup = (int)std::max<int64_t>(1, std::min<int64_t>((nsup + 3) / 4, 8192));
    hipStream_t s = (hipStream_t)stream;
    if (c64)
        hipLaunchKernelGGL(cdf_block_kernel<float>, dim3(grid), dim3(256), 0, s, (const float *)P, M, nb, bp, cs);
    else
        hipLaunchKernelGGL(cdf_block_kernel<double>, dim3(grid), dim3(256), 0, s, (const double *)P, M, nb, bp, cs);
    hipLaunchKernelGGL(cdf_super_kernel, dim3(gsup), dim3(256), 0, s, (const double *)bp, nb, nsup, sp);
    hipLaunchKernelGGL(cdf_scan_kernel, dim3(1), dim3(1024), 0, s, sp, nsup);
    hipLaunchKernelGGL(cdf_fix_kernel, dim3(gsup), dim3(256), 0, s, bp, nb, (const double *)sp, nsup);
    const CdfTree tr = cdf_tree_layout(nb);
    if (tr.nlev > 1) {
        const int gt = (int)std::max<int64_t>(1, std::min<int64_t>((tr.n[1] + 255) / 256, 1024));
        hipLaunchKernelGGL(cdf_tree_kernel, dim3(gt), dim3(256), 0, s, (const double *)bp, cs + kChunks * nb, tr);
    }
    return (int)hipGetLastError();
}

int slos_launch_marginals(const void *P, int c64, const double *bp, const int64_t *ends, int m, double *pk,
                          void *stream)
{
    const int grid = (m + 3) / 4;
    hipStream_t s = (hipStream_t)stream;
    if (c64)
        hipLaunchKernelGGL(marginal_kernel<float>, dim3(grid), dim3(256), 0, s, (const float *)P, bp, ends, m, pk);
    else
        hipLaunchKernelGGL(marginal_kernel<double>, dim3(grid), dim3(256), 0, s, (const double *)P, bp, ends, m, pk);
    return (int)hipGetLastError();
}

int slos_launch_sample(const void *P, int c64, int64_t M, const double *bp, const double *r, int64_t count,
                       int64_t *ranks, void *stream)
{
    const int64_t nb = (M + SLOS_CDF_BLOCK - 1) / SLOS_CDF_BLOCK;
    const int64_t waves = (count + 3) / 4;  // four samples per wave
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((waves + 3) / 4, 8192));
    hipStream_t s = (hipStream_t)stream;
    if (c64)
        hipLaunchKernelGGL(sample_kernel<float>, dim3(grid), dim3(256), 0, s, (const float *)P, M, bp, nb, r, count,
                           ranks, cdf_tree_layout(nb));
    else
        hipLaunchKernelGGL(sample_kernel<double>, dim3(grid), dim3(256), 0, s, (const double *)P, M, bp, nb, r,
                           count, ranks, cdf_tree_layout(nb));
    return (int)hipGetLastError();
}
