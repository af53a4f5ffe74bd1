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
// (cs = sp + nsup + 1).  A sample finds its run with a 64-way search over sp,
// its block with a 64-way search over that run's part of bp, its chunk from the
// block's 16 chunk sums (one cache line), and then its state with a wave scan
// of that chunk: about 400 bytes per sample instead of half a 4 KB block.
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

// One wave per sample: ranks[s] = first state whose cumulative P exceeds r[s] * total.
template <typename T>
__global__ __launch_bounds__(256) void sample_kernel(const T *__restrict__ P, int64_t M, const double *__restrict__ bp,
                                                     int64_t nb, const double *__restrict__ r, int64_t count,
                                                     int64_t *__restrict__ ranks)
{
    const int64_t nsup = (nb + SLOS_CDF_BLOCK - 1) / SLOS_CDF_BLOCK;
    const double *__restrict__ sp = bp + nb + 1;  // run prefixes, nsup + 1 entries
    const double *__restrict__ cs = sp + nsup + 1;  // chunk sums, kChunks per block
    const int lane = threadIdx.x & 63;
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    const double total = bp[nb];
    for (int64_t sidx = gw; sidx < count; sidx += nw) {
        const double t = r[sidx] * total;
        // the run of SLOS_CDF_BLOCK blocks first: largest s with sp[s] <= t over
        // the small run-prefix table (cache resident), then the largest block b
        // of that run with bp[b] <= t; both 64-way searches (the tables are
        // non-decreasing and start at 0 <= t, so the predicate holds on a prefix)
        int64_t lo = 0, hi = nsup;
        while (hi - lo > 1) {
            const int64_t step = (hi - lo + 63) / 64;
            const int64_t pos = lo + (int64_t)lane * step;
            const bool ok = pos < hi && sp[pos] <= t;
            const uint64_t bal = __ballot(ok);
            const int last = bal ? 63 - __builtin_clzll(bal) : 0;
            lo = lo + (int64_t)last * step;
            hi = min(lo + step, hi);
        }
        lo = lo * SLOS_CDF_BLOCK;
        hi = min(lo + SLOS_CDF_BLOCK, nb);
        while (hi - lo > 1) {
            const int64_t step = (hi - lo + 63) / 64;
            const int64_t pos = lo + (int64_t)lane * step;
            const bool ok = pos < hi && bp[pos] <= t;
            const uint64_t bal = __ballot(ok);
            const int last = bal ? 63 - __builtin_clzll(bal) : 0;  // lane 0 holds for r >= 0
            lo = lo + (int64_t)last * step;
            hi = min(lo + step, hi);
        }
        // the block's chunk sums (one line): the first chunk whose running sum
        // exceeds t, else the last chunk of non-zero probability
        const int64_t base = lo * SLOS_CDF_BLOCK;
        const double c_own = lane < kChunks ? cs[lo * kChunks + lane] : 0.0;
        double c_inc = c_own;
#pragma unroll
        for (int o = 1; o < kChunks; o <<= 1) {
            const double u = __shfl_up(c_inc, o, 64);
            if (lane >= o) c_inc += u;
        }
        const uint64_t c_cross = __ballot(lane < kChunks && bp[lo] + c_inc > t && c_own > 0.0);
        const uint64_t c_pos = __ballot(lane < kChunks && c_own > 0.0);
        const int i0 = c_cross ? __builtin_ctzll(c_cross) : (c_pos ? 63 - __builtin_clzll(c_pos) : 0);
        // then the states of the chunks from i0 on (rounding between the chunk
        // sums and this scan can move the crossing on to a later chunk)
        double run = bp[lo] + __shfl(c_inc - c_own, i0, 64);
        int64_t found = -1, last_pos = -1;
        for (int i = i0; i < kChunks && found < 0; ++i) {
            const int64_t x = base + i * 64 + lane;
            const double v = x < M ? (double)P[x] : 0.0;
            double c = v;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const double u = __shfl_up(c, o, 64);
                if (lane >= o) c += u;
            }
            const uint64_t cross = __ballot(run + c > t && v > 0.0);
            const uint64_t pos = __ballot(v > 0.0);
            if (cross) found = base + i * 64 + __builtin_ctzll(cross);
            if (pos) last_pos = base + i * 64 + 63 - __builtin_clzll(pos);
            run += __shfl(c, 63, 64);
        }
        // rounding can leave the crossing past the block's recomputed sum:
        // take the block's last state of non-zero probability
        if (found < 0) found = last_pos >= 0 ? last_pos : min(base, M - 1);
        if (lane == 0) ranks[sidx] = found;
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
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((count + 3) / 4, 8192));
    hipStream_t s = (hipStream_t)stream;
    if (c64)
        hipLaunchKernelGGL(sample_kernel<float>, dim3(grid), dim3(256), 0, s, (const float *)P, M, bp, nb, r, count,
                           ranks);
    else
        hipLaunchKernelGGL(sample_kernel<double>, dim3(grid), dim3(256), 0, s, (const double *)P, M, bp, nb, r,
                           count, ranks);
    return (int)hipGetLastError();
}
