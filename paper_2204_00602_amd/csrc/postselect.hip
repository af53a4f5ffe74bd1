// HIP kernels (gfx950): post-selection over mode groups.
//
// A Processor keeps only the outputs that pass its heralds and post-selection
// function (Section 3.2.7, the CNOT analysis, and the Processor appendix).  Here
// the predicate is a conjunction over groups of modes: output S is kept iff
// for every group g, count_min[g] <= sum_{j in g} s_j <= count_max[g].  The
// kernels sum P over the kept outputs (the gate's performance), optionally
// write P masked to the kept outputs, and turn a list of output ranks into the
// post-selected conditional probabilities P(S) / sum_kept P.
//
// Each thread walks a contiguous run of colex ranks: it unranks the first
// state with the binomial table and then steps to the colex successor, which
// moves one photon from the lowest occupied mode a to a + 1 and the other
// photons of mode a to mode 0 (so the next lowest occupied mode is known
// without a search).  The occupation vector and the group counts live in the
// thread's LDS row; a count of out-of-range groups decides each state.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "slos_ext.h"

namespace {

constexpr int kPsHead = 256 + 2 * SLOS_PS_MAX_GROUPS;  // LDS bytes of the group table and count bounds

__device__ __forceinline__ uint64_t binom_at(const PostselectParams &p, int a, int b)
{
    return p.binom[(size_t)a * p.bstride + b];
}

// Occupations of colex rank `rank` of F(m, n) into t[0..m); rank = sum_r C(d_r + r - 1, r)
// over the sorted photon modes d_1 <= .. <= d_n.
__device__ void unrank(const PostselectParams &p, uint64_t rank, uint8_t *t)
{
    for (int j = 0; j < p.m; ++j) t[j] = 0;
    int c = p.m + p.n - 2;
    for (int r = p.n; r >= 1; --r) {
        while (c >= r && binom_at(p, c, r) > rank) --c;
        if (c < r - 1) c = r - 1;
        rank -= (c >= r) ? binom_at(p, c, r) : 0;
        t[c - (r - 1)] += 1;
        --c;
    }
}

__device__ __forceinline__ bool kept(const PostselectParams &p, const uint8_t *cnt)
{
    bool ok = true;
    for (int g = 0; g < p.ngroups; ++g) ok = ok && cnt[g] >= p.cmin[g] && cnt[g] <= p.cmax[g];
    return ok;
}

__device__ __forceinline__ void count_groups(const PostselectParams &p, const uint8_t *t, uint8_t *cnt)
{
    for (int g = 0; g < p.ngroups; ++g) cnt[g] = 0;
    for (int j = 0; j < p.m; ++j)
        if (p.group[j] >= 0) cnt[p.group[j]] += t[j];
}

template <typename T>
__global__ __launch_bounds__(256) void postselect_kernel(PostselectParams p)
{
    extern __shared__ __align__(16) unsigned char lds[];
    // the group table in LDS (per-lane lookups), then one row per thread:
    // occupations t[0..m) and group counts cnt[0..SLOS_PS_MAX_GROUPS)
    int8_t *grp = (int8_t *)lds;
    uint8_t *lo = lds + 256, *hi = lo + SLOS_PS_MAX_GROUPS;
    for (int j = threadIdx.x; j < 256; j += blockDim.x) grp[j] = p.group[j];
    if (threadIdx.x < SLOS_PS_MAX_GROUPS) {
        lo[threadIdx.x] = p.cmin[threadIdx.x];
        hi[threadIdx.x] = p.cmax[threadIdx.x];
    }
    __syncthreads();
    uint8_t *t = lds + kPsHead + (size_t)threadIdx.x * (p.m + SLOS_PS_MAX_GROUPS);
    uint8_t *cnt = t + p.m;
    const int lane = threadIdx.x & 63;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t s0 = tid * p.run;
    const uint64_t s1 = min(s0 + p.run, (uint64_t)p.M);
    const T *P = (const T *)p.P;
    T *out = (T *)p.masked;
    double acc = 0.0;
    if (s0 < s1) {
        unrank(p, s0, t);
        count_groups(p, t, cnt);
        // number of groups whose count is out of range; the state is kept iff 0
        int viol = 0;
        for (int g = 0; g < p.ngroups; ++g) viol += (cnt[g] < lo[g] || cnt[g] > hi[g]) ? 1 : 0;
        auto move = [&](int j, int d) {
            const int g = grp[j];
            if (g >= 0) {
                const int c0 = cnt[g], c1 = c0 + d;
                viol += ((c1 < lo[g] || c1 > hi[g]) ? 1 : 0) - ((c0 < lo[g] || c0 > hi[g]) ? 1 : 0);
                cnt[g] = (uint8_t)c1;
            }
        };
        int a = 0;  // lowest occupied mode
        while (a < p.m - 1 && t[a] == 0) ++a;
        for (uint64_t s = s0; s < s1; ++s) {
            const T v = P[s];
            const bool ok = viol == 0;
            if (ok) acc += (double)v;
            if (out) out[s] = ok ? v : (T)0;
            if (s + 1 < s1) {
                // a < m - 1 since s is not the last state; modes below a are
                // empty, so afterwards the lowest occupied mode is 0 if photons
                // went back to mode 0, else a + 1
                const int c = t[a];
                t[a] = 0;
                t[a + 1] += 1;
                t[0] += (uint8_t)(c - 1);
                move(a, -c);
                move(a + 1, 1);
                move(0, c - 1);
                a = c > 1 ? 0 : a + 1;
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) p.partials[tid / 64] = acc;
}

// ---- leaf path --------------------------------------------------------------
// The last layer's leaves fix the occupations of their high modes and run
// their K low photons over the q low modes in the colex order of F(q, K).
// The group counts of an output are those of its leaf's high part (from the
// leaf record) plus those of its low part, which depend only on the leaf's
// inner type and the state's rank in it: ps_low_kernel tabulates them once per
// call for the inner types the last layer uses, and ps_leaf_kernel reads P and
// the table with the leaf's outputs (contiguous, so all accesses coalesce).

// Occupations of colex rank `rank` of F(q, K) (the same decoding as unrank).
__device__ void unrank_q(const PostselectParams &p, int q, int K, uint64_t rank, uint8_t *t)
{
    for (int j = 0; j < q; ++j) t[j] = 0;
    int c = q + K - 2;
    for (int r = K; r >= 1; --r) {
        while (c >= r && binom_at(p, c, r) > rank) --c;
        if (c < r - 1) c = r - 1;
        rank -= (c >= r) ? binom_at(p, c, r) : 0;
        t[c - (r - 1)] += 1;
        --c;
    }
}

__global__ __launch_bounds__(256) void ps_low_kernel(PostselectParams p)
{
    extern __shared__ __align__(16) unsigned char lds[];
    uint8_t *t = lds + (size_t)threadIdx.x * 256;  // occupations of up to 255 low modes
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= p.entries) return;
    // inner type of entry e: last type with off <= e
    uint32_t lo = 0, hi = p.ntypes;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (p.types[mid].off <= e) lo = mid;
        else hi = mid;
    }
    const PsType ty = p.types[lo];
    unrank_q(p, ty.q, ty.K, e - ty.off, t);
    uint8_t c[SLOS_PS_MAX_GROUPS] = {};
    for (int j = 0; j < ty.q; ++j)
        if (p.group[j] >= 0) c[p.group[j]] += t[j];
    uint4 w;
    w.x = c[0] | c[1] << 8 | c[2] << 16 | (uint32_t)c[3] << 24;
    w.y = c[4] | c[5] << 8 | c[6] << 16 | (uint32_t)c[7] << 24;
    w.z = c[8] | c[9] << 8 | c[10] << 16 | (uint32_t)c[11] << 24;
    w.w = c[12] | c[13] << 8 | c[14] << 16 | (uint32_t)c[15] << 24;
    if (p.ngroups <= 4) ((uint32_t *)p.low)[e] = w.x;  // narrow table: 4 bytes per state
    else ((uint4 *)p.low)[e] = w;
}

__device__ __forceinline__ uint32_t byte_of(const uint4 &w, int g)
{
    const uint32_t d = g < 4 ? w.x : g < 8 ? w.y : g < 12 ? w.z : w.w;
    return (d >> (8 * (g & 3))) & 0xFFu;
}

// table entry of a low state: 16 group counts, or 4 in one word (NARROW)
template <bool NARROW> struct LowEntry;
template <> struct LowEntry<false> { using type = uint4; };
template <> struct LowEntry<true> { using type = uint32_t; };
__device__ __forceinline__ uint32_t count_of(const uint4 &w, int g) { return byte_of(w, g); }
__device__ __forceinline__ uint32_t count_of(uint32_t w, int g) { return (w >> (8 * (g & 3))) & 0xFFu; }

// one wave per leaf of the last layer; one FP64 partial per wave.  NARROW:
// at most 4 groups, table entries of 4 bytes
template <typename T, bool NARROW>
__global__ __launch_bounds__(256) void ps_leaf_kernel(PostselectParams p)
{
    using E = typename LowEntry<NARROW>::type;
    constexpr int NG = NARROW ? 4 : SLOS_PS_MAX_GROUPS;
    __shared__ int8_t grp[256];
    for (int j = threadIdx.x; j < 256; j += blockDim.x) grp[j] = p.group[j];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const uint64_t gw = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint64_t nw = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const T *P = (const T *)p.P;
    T *out = (T *)p.masked;
    double acc = 0.0;
    // the 64-byte leaf record: lane i < 16 holds dword i (one coalesced load),
    // fields are read back with readlane; the next record is fetched early
    auto fetch = [&](uint64_t li) -> uint32_t {
        return (li < p.nleaves && lane < 16) ? ((const uint32_t *)(p.leaves + li))[lane] : 0u;
    };
    auto rl = [](uint32_t v, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)v, l); };
    uint32_t rec = fetch(gw);
    for (uint64_t li = gw; li < p.nleaves; li += nw) {
        const uint32_t cur = rec;
        rec = fetch(li + nw);
        const uint64_t base = (uint64_t)rl(cur, 0) | ((uint64_t)rl(cur, 1) << 32);
        const uint32_t size = rl(cur, 2), tab = rl(cur, 3);
        const uint32_t nhp = (rl(cur, 4) >> 16) & 0xFFu;
        // group counts of the high part (wave-uniform)
        uint32_t hc[SLOS_PS_MAX_GROUPS];
#pragma unroll
        for (int g = 0; g < SLOS_PS_MAX_GROUPS; ++g) hc[g] = 0;
        for (uint32_t i = 0; i < nhp; ++i) {
            const uint32_t mode = (rl(cur, 8 + (int)(i >> 2)) >> (8 * (i & 3))) & 0xFFu;
            const int g = grp[mode];
#pragma unroll
            for (int h = 0; h < SLOS_PS_MAX_GROUPS; ++h) hc[h] += (g == h) ? 1u : 0u;
        }
        const E *low = (const E *)p.low + p.type_off[tab];
        // NARROW: the four group counts of an output are the bytes of
        // (table entry + hp) (each at most n <= 32, so bytes never carry), and
        // "lo_g <= c_g <= hi_g for every g" is one test on guard bits: with
        // G = 0x80 in each byte, ((c | G) - lo) and ((hi | G) - c) keep bit 7 of
        // byte g iff c_g >= lo_g and hi_g >= c_g (bounds clamped to 127, unused
        // groups [0, 127]; no byte borrows).
        uint32_t hp = 0, lo4 = 0, hi4 = 0;
        if (NARROW) {
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const bool used = g < p.ngroups;
                const uint32_t a = p.cmin[g], b = p.cmax[g];
                hp |= (used ? hc[g] : 0u) << (8 * g);
                lo4 |= (used ? (a < 127u ? a : 127u) : 0u) << (8 * g);
                hi4 |= (used ? (b < 127u ? b : 127u) : 127u) << (8 * g);
            }
        }
        // kSteps outputs per lane and step (x0 + 64u), loads first: P is read
        // once (non-temporal, so the shared low-state table stays in L2).
        // Measured at m=24, n=12: 4 per step 1.33 ms, 8 1.24 ms, 16 1.52 ms.
        constexpr int kSteps = 8;
        for (uint32_t x0 = lane; x0 < size; x0 += 64u * kSteps) {
            E w[kSteps];
            T v[kSteps];
#pragma unroll
            for (int u = 0; u < kSteps; ++u) {
                const uint32_t x = x0 + 64u * u;
                const uint32_t xc = x < size ? x : x0;
                w[u] = low[xc];
                v[u] = __builtin_nontemporal_load(P + base + xc);
            }
#pragma unroll
            for (int u = 0; u < kSteps; ++u) {
                const uint32_t x = x0 + 64u * u;
                if (x >= size) break;
                bool ok = true;
                if constexpr (NARROW) {
                    constexpr uint32_t G = 0x80808080u;
                    const uint32_t c = (uint32_t)w[u] + hp;
                    ok = ((((c | G) - lo4) & ((hi4 | G) - c)) & G) == G;
                } else {
#pragma unroll
                    for (int g = 0; g < NG; ++g) {
                        if (g < p.ngroups) {
                            const uint32_t c = count_of(w[u], g) + hc[g];
                            ok = ok && c >= p.cmin[g] && c <= p.cmax[g];
                        }
                    }
                }
                if (ok) acc += (double)v[u];
                if (out) out[base + x] = ok ? v[u] : (T)0;
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) p.partials[gw] = acc;
}

// table[i] = P[ranks[i]] / sum_kept if output ranks[i] is kept, else 0.
template <typename T>
__global__ __launch_bounds__(64) void postselect_table_kernel(PostselectParams p, const int64_t *ranks,
                                                              int64_t nranks, const double *sum, double *table)
{
    extern __shared__ __align__(16) unsigned char lds[];
    uint8_t *t = lds + (size_t)threadIdx.x * (p.m + SLOS_PS_MAX_GROUPS);
    uint8_t *cnt = t + p.m;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nranks) return;
    const int64_t r = ranks[i];
    if (r < 0 || r >= p.M) {
        table[i] = 0.0;
        return;
    }
    unrank(p, (uint64_t)r, t);
    count_groups(p, t, cnt);
    const double v = (double)((const T *)p.P)[r];
    table[i] = kept(p, cnt) ? v / *sum : 0.0;
}

template <typename K>
hipError_t allow_lds(K kernel, size_t bytes)
{
    static bool done = false;  // per instantiation
    if (done || bytes <= 65536) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) done = true;
    return e;
}

} // namespace

int slos_launch_postselect(const PostselectParams &p, int c64, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (p.nleaves > 0) {
        // leaf path: tabulate the low parts, then one wave per leaf
        const int gl = (int)((p.entries + 255) / 256);
        hipError_t e = allow_lds(ps_low_kernel, 256 * 256);
        if (e != hipSuccess) return (int)e;
        hipLaunchKernelGGL(ps_low_kernel, dim3(gl > 0 ? gl : 1), dim3(256), 256 * 256, s, p);
        if ((e = hipGetLastError()) != hipSuccess) return (int)e;
        const int grid = SLOS_PS_MAX_WAVES / 4;
        const bool narrow = p.ngroups <= 4;
        if (c64 && narrow)
            hipLaunchKernelGGL((ps_leaf_kernel<float, true>), dim3(grid), dim3(256), 0, s, p);
        else if (c64)
            hipLaunchKernelGGL((ps_leaf_kernel<float, false>), dim3(grid), dim3(256), 0, s, p);
        else if (narrow)
            hipLaunchKernelGGL((ps_leaf_kernel<double, true>), dim3(grid), dim3(256), 0, s, p);
        else
            hipLaunchKernelGGL((ps_leaf_kernel<double, false>), dim3(grid), dim3(256), 0, s, p);
        return (int)hipGetLastError();
    }
    // no photons: one output, walked by one thread
    const uint64_t threads = (p.M + p.run - 1) / p.run;
    const int grid = (int)((threads + 255) / 256);
    const size_t lds = kPsHead + 256 * (size_t)(p.m + SLOS_PS_MAX_GROUPS);
    hipError_t e = c64 ? allow_lds(postselect_kernel<float>, lds) : allow_lds(postselect_kernel<double>, lds);
    if (e != hipSuccess) return (int)e;
    if (c64)
        hipLaunchKernelGGL(postselect_kernel<float>, dim3(grid), dim3(256), lds, s, p);
    else
        hipLaunchKernelGGL(postselect_kernel<double>, dim3(grid), dim3(256), lds, s, p);
    return (int)hipGetLastError();
}

int slos_launch_postselect_table(const PostselectParams &p, int c64, const int64_t *ranks, int64_t nranks,
                                 const double *sum, double *table, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    const int grid = (int)((nranks + 63) / 64);
    const size_t lds = 64 * (size_t)(p.m + SLOS_PS_MAX_GROUPS);
    if (c64)
        hipLaunchKernelGGL(postselect_table_kernel<float>, dim3(grid), dim3(64), lds, s, p, ranks, nranks, sum,
                           table);
    else
        hipLaunchKernelGGL(postselect_table_kernel<double>, dim3(grid), dim3(64), lds, s, p, ranks, nranks, sum,
                           table);
    return (int)hipGetLastError();
}
