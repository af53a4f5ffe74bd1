// HIP kernels (gfx950) of the SLOS layer recurrence.
//
// One launch computes layer k of the recurrence of arXiv 2204.00602, Section
// 3.2.3 (SLOS), in gather form:
//     A_k[t] = sum_{j : t_j > 0} U[j, i_k] * A_{k-1}[t - e_j],
// every output written by exactly one lane, with no atomics on data (the work
// tickets and the recorded maximum of a compensated layer are atomic counters
// that schedule and bound, never outputs).  The last layer fuses
// the normalisation a(S) = A_n[S] sqrt(prod s_j!) / sqrt(prod t_i!) (Eq.
// eqperm), |a|^2 and an FP64 per-wave partial of sum_S P(S).
//
// Work unit: one leaf per workgroup at a time (see LeafRec and the host-built
// leaf descriptors).  The workgroup stages the leaf's low block in LDS and
// deals the leaf's tiles to its waves.  Every predecessor block reached
// through a high mode is contiguous (lane x reads base + x), its base taken
// from the descriptor; predecessors through the q low modes come from the
// per-(q, K) inner table and the staged block.  U's column i_k is staged in
// LDS; u[255] = 0 pads short term lists.  The batch kernel further down runs
// whole small instances per workgroup, one leaf per wave.
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

// ---- compensated complex64 accumulation ---------------------------------
// SLOS_COMP_TWOSUM: every real product a*b is split exactly into p + pe with an
// FMA (two-product) and added to the running sum s with Knuth's two-sum; both
// rounding errors go to a second float c.  Ten operations per product.
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

// Default compensated mode: biased FMA accumulation.  The sum starts at a
// power of two sigma >= 4 * sum_i |a_i b_i| (a bound known before the sum).  Every partial sum then stays within [3/4, 5/4] sigma, so
// for t = fma(a, b, s) the difference s - t is exact (Sterbenz) and
// fma(a, b, s - t) is the FMA's rounding error, correct to one rounding of a
// number below ulp(sigma).  Those errors go to a second float c, and the
// result is (s - sigma) + c, where s - sigma is exact again.  The error-free
// transformation is the two-sum of s and a*b computed with the FMA; the bias
// makes its short form exact.  Four operations per real product; the error is
// within one rounding of the result plus O(terms * 2^-46 * sigma).
__device__ __forceinline__ void acc_biased(float &s, float &c, float a, float b)
{
#pragma clang fp contract(off)
    const float t = __builtin_fmaf(a, b, s);
    const float d = s - t;
    c = c + __builtin_fmaf(a, b, d);
    s = t;
}

// 8 * 2^floor(log2 b) (> 4b), at least 2^-117
__device__ __forceinline__ float bias_for(float b)
{
    const float f = __uint_as_float(__float_as_uint(b) & 0x7F800000u);
    return 8.0f * fmaxf(f, 0x1p-120f);
}

template <typename T, int COMP> struct Acc;
template <typename T> struct Acc<T, SLOS_COMP_NONE> {
    using C = typename Cx<T>::type;
    C a;
    __device__ __forceinline__ void zero() { a = C{0, 0}; }
    __device__ __forceinline__ void start(float) {}
    __device__ __forceinline__ void mac(const C u, const C v) { cmac(a, u, v); }
    __device__ __forceinline__ C value() const { return a; }
    __device__ __forceinline__ double re() const { return (double)a.x; }
    __device__ __forceinline__ double im() const { return (double)a.y; }
};
template <> struct Acc<float, SLOS_COMP_TWOSUM> {
    CompAcc a;
    __device__ __forceinline__ void zero() { a.s = float2{0.f, 0.f}; a.c = float2{-0.f, -0.f}; }
    __device__ __forceinline__ void start(float) {}
    __device__ __forceinline__ void mac(const float2 u, const float2 v) { cmac_comp(a, u, v); }
    __device__ __forceinline__ float2 value() const { return float2{a.s.x + a.c.x, a.s.y + a.c.y}; }
    __device__ __forceinline__ double re() const { return (double)a.s.x + (double)a.c.x; }
    __device__ __forceinline__ double im() const { return (double)a.s.y + (double)a.c.y; }
};
template <> struct Acc<float, SLOS_COMP_BIASED> {
    float sr, si, cr, ci, sigma;
    // the error sums start at -0, the identity of IEEE addition, so the first
    // term's addition folds away
    __device__ __forceinline__ void zero()
    {
        sr = si = sigma = 0.f;
        cr = ci = -0.f;
    }
    __device__ __forceinline__ void start(float bias)
    {
        sigma = bias;
        sr = bias;
        si = bias;
    }
    __device__ __forceinline__ void mac(const float2 u, const float2 v)
    {
        acc_biased(sr, cr, u.x, v.x);
        acc_biased(sr, cr, -u.y, v.y);
        acc_biased(si, ci, u.x, v.y);
        acc_biased(si, ci, u.y, v.x);
    }
    __device__ __forceinline__ float2 value() const { return float2{(sr - sigma) + cr, (si - sigma) + ci}; }
    __device__ __forceinline__ double re() const { return (double)(sr - sigma) + (double)cr; }
    __device__ __forceinline__ double im() const { return (double)(si - sigma) + (double)ci; }
};

// FP64 mode: each term's complex64 factors are widened to FP64, where their
// products are exact (24-bit significands), and the products are summed with
// FP64 FMAs: one FP64 rounding per real product, four FMAs and up to four
// conversions per complex term (the FP64 FMA issues at the FP32 rate here).
template <> struct Acc<float, SLOS_COMP_F64> {
    double r, i;
    __device__ __forceinline__ void zero() { r = i = 0.0; }
    __device__ __forceinline__ void start(float) {}
    __device__ __forceinline__ void mac(const float2 uf, const float2 v)
    {
        const double2 u{(double)uf.x, (double)uf.y};
        const double vr = (double)v.x, vi = (double)v.y;
        r = __builtin_fma(u.x, vr, r);
        r = __builtin_fma(-u.y, vi, r);
        i = __builtin_fma(u.x, vi, i);
        i = __builtin_fma(u.y, vr, i);
    }
    __device__ __forceinline__ float2 value() const { return float2{(float)r, (float)i}; }
    __device__ __forceinline__ double re() const { return r; }
    __device__ __forceinline__ double im() const { return i; }
};

// cache-policy operand of the global-to-LDS copy: 0 = default, bit 1 =
// non-temporal
#define SLOS_CPOL_DEFAULT 0
#define SLOS_CPOL_NT 2

// ---- cross-lane helpers (wave64) -------------------------------------------
__device__ __forceinline__ uint32_t rl32(uint32_t v, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)v, l); }
__device__ __forceinline__ uint64_t rl64(uint64_t v, int l)
{
    return (uint64_t)rl32((uint32_t)v, l) | ((uint64_t)rl32((uint32_t)(v >> 32), l) << 32);
}
__device__ __forceinline__ float rlv(float v, int l) { return __uint_as_float(rl32(__float_as_uint(v), l)); }
__device__ __forceinline__ double rlv(double v, int l)
{
    return __longlong_as_double((long long)rl64((uint64_t)__double_as_longlong(v), l));
}
// dst lane receives `v` from the lane that names it (ds_permute); later writers win
__device__ __forceinline__ uint32_t push32(uint32_t v, int dst)
{
    return (uint32_t)__builtin_amdgcn_ds_permute(dst << 2, (int)v);
}
__device__ __forceinline__ uint64_t push64(uint64_t v, int dst)
{
    return (uint64_t)push32((uint32_t)v, dst) | ((uint64_t)push32((uint32_t)(v >> 32), dst) << 32);
}
__device__ __forceinline__ float pushv(float v, int dst) { return __uint_as_float(push32(__float_as_uint(v), dst)); }
__device__ __forceinline__ double pushv(double v, int dst)
{
    return __longlong_as_double((long long)push64((uint64_t)__double_as_longlong(v), dst));
}

// ---- leaf descriptors --------------------------------------------------------
// A descriptor is fetched with one coalesced load (lane l holds dword l) and
// read back with readlane, so every field is wave-uniform.
template <bool WIDE> struct DescT;
template <> struct DescT<false> {
    using type = LeafDescNarrow;
    static constexpr int kDwords = (int)(sizeof(LeafDescNarrow) / 4);
};
template <> struct DescT<true> {
    using type = LeafDescWide;
    static constexpr int kDwords = (int)(sizeof(LeafDescWide) / 4);
};

// Lanes 0..63 hold dwords 0..63 of the descriptor (the wide form uses a
// second register for dwords 64..83).
template <bool WIDE>
struct DescRegs {
    uint32_t a;
    uint32_t b;
};

// A pass reads each descriptor once, non-temporally; the batch kernel
// (CACHED) reads one (m, k) descriptor set for every instance of that m, so
// it keeps them in the L2.
template <bool WIDE, bool CACHED = false>
__device__ __forceinline__ DescRegs<WIDE> load_desc(const void *descs, uint64_t li, int lane)
{
    const uint32_t *w = (const uint32_t *)((const char *)descs + li * sizeof(typename DescT<WIDE>::type));
    DescRegs<WIDE> r;
    constexpr int nd = DescT<WIDE>::kDwords;
    if (CACHED) {
        r.a = lane < nd ? w[lane] : 0u;
        r.b = (WIDE && lane + 64 < nd) ? w[64 + lane] : 0u;
    } else {
        r.a = lane < nd ? __builtin_nontemporal_load(&w[lane]) : 0u;
        r.b = (WIDE && lane + 64 < nd) ? __builtin_nontemporal_load(&w[64 + lane]) : 0u;
    }
    return r;
}

template <bool WIDE>
__device__ __forceinline__ uint32_t desc_dword(const DescRegs<WIDE> &r, int i)
{
    return i < 64 ? rl32(r.a, i) : rl32(r.b, i - 64);
}

struct Leaf {
    uint64_t out_base;
    uint64_t low_base;
    double fac_hi;
    uint32_t size;
    uint32_t low_size;
    uint32_t pred_off;
    uint32_t fac_off;
    int cmax;
    int nh;
};

template <bool WIDE>
__device__ __forceinline__ Leaf decode_head(const DescRegs<WIDE> &r)
{
    Leaf L;
    L.out_base = (uint64_t)rl32(r.a, 0) | ((uint64_t)rl32(r.a, 1) << 32);
    L.low_base = (uint64_t)rl32(r.a, 2) | ((uint64_t)rl32(r.a, 3) << 32);
    L.fac_hi = __longlong_as_double((long long)((uint64_t)rl32(r.a, 4) | ((uint64_t)rl32(r.a, 5) << 32)));
    L.size = rl32(r.a, 6);
    L.low_size = rl32(r.a, 7);
    L.pred_off = rl32(r.a, 8);
    L.fac_off = rl32(r.a, 9);
    const uint32_t ck = rl32(r.a, 10);
    L.cmax = (int)(ck & 0xFFu);
    L.nh = (int)((ck >> 8) & 0xFFu);
    return L;
}

// rank in A_{k-1} of group g's block and the mode of group g
template <bool WIDE>
__device__ __forceinline__ uint64_t group_base(const DescRegs<WIDE> &r, const Leaf &L, int g)
{
    if (WIDE) {
        const int d = 12 + 2 * g;
        const uint64_t dl = (uint64_t)desc_dword<WIDE>(r, d) | ((uint64_t)desc_dword<WIDE>(r, d + 1) << 32);
        return L.low_base - dl;
    }
    return L.low_base - (uint64_t)rl32(r.a, 12 + g);
}

template <bool WIDE>
__device__ __forceinline__ int group_mode(const DescRegs<WIDE> &r, int g)
{
    constexpr int first = WIDE ? 12 + 2 * SLOS_WIDE_GROUPS : 12 + SLOS_NARROW_GROUPS;
    return (int)((desc_dword<WIDE>(r, first + (g >> 2)) >> (8 * (g & 3))) & 0xFFu);
}

// Loads through a wave-uniform base pointer and a 32-bit per-lane byte
// offset (the scalar-base + vector-offset addressing form).
template <typename V>
__device__ __forceinline__ V ld_off(const void *base, uint32_t off)
{
    return *(const V *)((const char *)base + off);
}

// complex64 load through a buffer resource made from a wave-uniform base (no
// range limit: word 2 = 0xFFFFFFFF; word 3 = the 32-bit data format that raw
// loads need on this chip family) and a 32-bit per-lane byte offset.  The
// resource is built with scalar instructions, so a block base costs no vector
// instruction per lane.
#define SLOS_RSRC_WORD3 0x00020000
__device__ __forceinline__ float2 ld_buf_c64(const void *base, uint32_t off)
{
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, -1, SLOS_RSRC_WORD3);
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
// 32-bit table load: per-lane offset `off` plus a wave-uniform offset `soff`
__device__ __forceinline__ uint32_t ld_buf_u32(const void *base, uint32_t off, uint32_t soff)
{
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, -1, SLOS_RSRC_WORD3);
    return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0);
}

// Stage A_{k-1}[low_base, low_base + low_size) into this wave's LDS slice with
// direct global-to-LDS copies of 16-byte chunks (64 lanes x 16 B per
// instruction).  The copy starts at the 16-byte boundary at or below the
// block, so the block begins `skew` bytes into the slice; up to 1 KiB past
// the block is read as well (the layer buffers carry that slack).
//
// Cache policy CPOL: each input element is staged once per layer, but a low
// block is also read whole as a high-mode block by the leaves one photon up
// (high part h + e_j, one low photon fewer), so intermediate layers and the
// batch kernel stage with the default policy, which keeps it in L2 for them;
// the last layer of a large pass stages non-temporally (measured slightly
// faster there, where the high-mode blocks fill the L2).
template <typename C, int CPOL = SLOS_CPOL_DEFAULT>
__device__ __forceinline__ const C *stage_low(const C *__restrict__ X, const Leaf &L, unsigned char *slice,
                                              int lane)
{
    const uintptr_t sa = (uintptr_t)(X + L.low_base);
    const uintptr_t a0 = sa & ~(uintptr_t)15;
    const uint32_t skew = (uint32_t)(sa - a0);
    const uint32_t nbytes = skew + L.low_size * (uint32_t)sizeof(C);
    for (uint32_t done = 0; done < nbytes; done += 1024u) {
        if (done + 16u * (uint32_t)lane < nbytes) {
            const void *src = (const void *)(a0 + done + 16u * (uint32_t)lane);
            __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)(slice + done), 16, 0,
                                             CPOL);
        }
    }
    return (const C *)(slice + skew);
}

// One tile: RT outputs per lane, x = t0 + i*64 + lane clamped to the leaf so
// every load is in bounds.  tile_load issues all block loads (up to HS high
// groups) and table loads (up to CS low terms) of the tile; tile_compute uses
// them, and loads the groups and terms past those from memory as it goes.
// complex64 two-output tiles hold six of each (80 VGPRs: six waves per SIMD),
// the other tiles eight.
template <typename T, int RT> constexpr int tile_slots() { return (sizeof(T) == 4 && RT == 2) ? 6 : 8; }

template <typename T, int RT>
struct TileIn {
    static constexpr int kHS = tile_slots<T, RT>();
    static constexpr int kCS = tile_slots<T, RT>();
    typename Cx<T>::type v[kHS][RT];
    uint32_t e[kCS][RT];
    double lf[RT];
    uint32_t xc[RT];
    uint32_t off[RT];
};

// BUF_HI / BUF_PRED: complex64 block and table loads through buffer
// resources (no vector address arithmetic) instead of scalar-base global
// loads.  Both forms read the same bytes; which one schedules better depends
// on the kernel around the tile (measured per kernel).
template <typename T, int MODE, int RT, bool WIDE, bool BUF_HI, bool BUF_PRED>
__device__ __forceinline__ void tile_load(TileIn<T, RT> &in, const LayerParams &p, const DescRegs<WIDE> &dr,
                                          const Leaf &L, const typename Cx<T>::type *__restrict__ X, uint32_t t0,
                                          int lane)
{
    using C = typename Cx<T>::type;
    constexpr int kHS = TileIn<T, RT>::kHS, kCS = TileIn<T, RT>::kCS;
#pragma unroll
    for (int i = 0; i < RT; ++i) {
        const uint32_t x = t0 + (uint32_t)(i * 64 + lane);
        in.xc[i] = x < L.size ? x : L.size - 1u;
        in.off[i] = in.xc[i] * (uint32_t)sizeof(C);
    }
    const uint32_t *__restrict__ pred = p.pred + L.pred_off;
    if constexpr (sizeof(T) == 8) {
        // complex128: a fixed number of loads, whatever the leaf.  Slots past
        // the leaf's groups or terms read element 0 (one line for the whole
        // wave) and are not used; straight-line loads let the compiler wait
        // for each one just before its first use.  (Measured faster for
        // complex128, slower for complex64.)
#pragma unroll
        for (int g = 0; g < kHS; ++g) {
            const bool live = g < L.nh;
            const C *Xb = live ? X + group_base<WIDE>(dr, L, g) : X;
#pragma unroll
            for (int i = 0; i < RT; ++i) in.v[g][i] = ld_off<C>(Xb, live ? in.off[i] : 0u);
        }
#pragma unroll
        for (int c = 0; c < kCS; ++c) {
            const bool live = c < L.cmax;
#pragma unroll
            for (int i = 0; i < RT; ++i)
                in.e[c][i] = ld_off<uint32_t>(pred, live ? ((uint32_t)c * L.size + in.xc[i]) * 4u : 0u);
        }
    } else {
        // block and table bases are wave-uniform; each lane adds its own
        // 32-bit offset
#pragma unroll
        for (int g = 0; g < kHS; ++g) {
            if (g < L.nh) {
                const C *Xb = X + group_base<WIDE>(dr, L, g);
#pragma unroll
                for (int i = 0; i < RT; ++i) in.v[g][i] = BUF_HI ? ld_buf_c64(Xb, in.off[i]) : ld_off<C>(Xb, in.off[i]);
            }
        }
        uint32_t xo[RT];
#pragma unroll
        for (int i = 0; i < RT; ++i) xo[i] = in.xc[i] * 4u;
#pragma unroll
        for (int c = 0; c < kCS; ++c) {
            if (c < L.cmax) {
#pragma unroll
                for (int i = 0; i < RT; ++i)
                    in.e[c][i] = BUF_PRED ? ld_buf_u32(pred, xo[i], (uint32_t)c * L.size * 4u)
                                          : ld_off<uint32_t>(pred + (size_t)c * L.size, xo[i]);
            }
        }
    }
    if (MODE != SLOS_MODE_MID) {
#pragma unroll
        for (int i = 0; i < RT; ++i) in.lf[i] = ld_off<double>(p.lowfac + L.fac_off, in.xc[i] * 8u);
    }
}

// sigma: the bias of the compensated mode (see Acc<float, SLOS_COMP_BIASED>).
// omax collects max |Re a| + |Im a| over the complex64 outputs of a mid layer,
// the input bound of a compensated next layer.  CACHED_MID: a mid layer's
// outputs are stored with the default cache policy instead of non-temporally
// (the batch kernel, whose small layers are read back from the L2 by the next
// layer; a large pass's layers outgrow the L2 and stream).
template <typename T, int MODE, int COMP, int RT, bool WIDE, bool CACHED_MID = false>
__device__ __forceinline__ void tile_compute(const TileIn<T, RT> &in, const LayerParams &p, const DescRegs<WIDE> &dr,
                                             const Leaf &L, const typename Cx<T>::type *__restrict__ X,
                                             const typename Cx<T>::type *u_lds, const typename Cx<T>::type *lowbuf,
                                             float sigma, uint32_t t0, int lane, double &psum, float &omax)
{
    using C = typename Cx<T>::type;
    constexpr int kHS = TileIn<T, RT>::kHS, kCS = TileIn<T, RT>::kCS;
    const uint32_t *__restrict__ pred = p.pred + L.pred_off;

    // Low-block element of a table entry: its 24-bit index times the element
    // size with one 24-bit multiply-add, which ignores the mode byte on top
    // (the size is hidden from the optimiser, which would otherwise turn the
    // multiply into a shift and a mask).
    uint32_t esz = (uint32_t)sizeof(C);
    asm volatile("" : "+v"(esz));
    auto low_at = [&](uint32_t e) -> C { return *(const C *)((const char *)lowbuf + __umul24(e, esz)); };

    // Visit every term (output i, mode j, predecessor value) of the tile:
    // high groups from registers (or, past kHS groups, straight from memory),
    // low terms from the staged block.  f takes the mode (coefficient from
    // the U column in LDS), fu a coefficient already loaded.
    auto terms = [&](auto &&f, auto &&fu) {
#pragma unroll
        for (int g = 0; g < kHS; ++g) {
            if (g < L.nh) {
                const int j = group_mode<WIDE>(dr, g);
                if constexpr ((COMP == SLOS_COMP_BIASED || COMP == SLOS_COMP_TWOSUM) && !CACHED_MID) {
                    // a group's coefficient U[j, i_k] is the same for the whole
                    // wave: read it through the scalar cache (constant address
                    // space; U is not written while the kernel runs) straight
                    // into an SGPR operand of the multiply-adds (the two-sum
                    // layers, which are issue-bound; the others keep the LDS
                    // column)
                    typedef __attribute__((address_space(4))) const T ConstT;
                    const ConstT *q = (const ConstT *)p.U + 2 * ((size_t)j * p.m + p.col);
                    const C uj{q[0], q[1]};
#pragma unroll
                    for (int i = 0; i < RT; ++i) fu(i, uj, in.v[g][i]);
                } else {
#pragma unroll
                    for (int i = 0; i < RT; ++i) f(i, j, in.v[g][i]);
                }
            }
        }
        for (int g = kHS; g < L.nh; ++g) {  // leaves with more than kHS high groups
            const C *Xb = X + group_base<WIDE>(dr, L, g);
            const int j = group_mode<WIDE>(dr, g);
#pragma unroll
            for (int i = 0; i < RT; ++i) f(i, j, ld_off<C>(Xb, in.off[i]));
        }
#pragma unroll
        for (int c = 0; c < kCS; ++c) {
            if (c < L.cmax) {
#pragma unroll
                for (int i = 0; i < RT; ++i) f(i, (int)(in.e[c][i] >> 24), low_at(in.e[c][i]));
            }
        }
        for (int c = kCS; c < L.cmax; ++c) {  // inner states with more than kCS low terms
#pragma unroll
            for (int i = 0; i < RT; ++i) {
                const uint32_t ec = ld_off<uint32_t>(pred, ((uint32_t)c * L.size + in.xc[i]) * 4u);
                f(i, (int)(ec >> 24), low_at(ec));
            }
        }
    };

    // ---- multiply-add
    Acc<T, COMP> acc[RT];
#pragma unroll
    for (int i = 0; i < RT; ++i) acc[i].zero();
#pragma unroll
    for (int i = 0; i < RT; ++i) acc[i].start(sigma);
    terms([&](int i, int j, const C x) { acc[i].mac(u_lds[j], x); },
          [&](int i, const C uj, const C x) { acc[i].mac(uj, x); });

    // ---- store (through the leaf's wave-uniform output base)
    T *Yb = (T *)p.Y + (MODE == SLOS_MODE_PROB ? 1u : 2u) * L.out_base;
#pragma unroll
    for (int i = 0; i < RT; ++i) {
        if (t0 + (uint32_t)(i * 64 + lane) >= L.size) continue;
        if (MODE == SLOS_MODE_MID) {
            const C a = acc[i].value();
            if (sizeof(T) == 4) omax = fmaxf(omax, (float)(fabs(a.x) + fabs(a.y)));
            T *y = (T *)((char *)Yb + in.off[i]);
            if (CACHED_MID) {
                *(C *)y = a;
            } else {
                __builtin_nontemporal_store(a.x, y);
                __builtin_nontemporal_store(a.y, y + 1);
            }
        } else {
            const double f = L.fac_hi * in.lf[i];
            const double ar = acc[i].re() * f;
            const double ai = acc[i].im() * f;
            const double pr = ar * ar + ai * ai;
            psum += pr;
            if (MODE == SLOS_MODE_AMPL) {
                T *y = (T *)((char *)Yb + in.off[i]);
                __builtin_nontemporal_store((T)ar, y);
                __builtin_nontemporal_store((T)ai, y + 1);
            } else {
                __builtin_nontemporal_store((T)pr, (T *)((char *)Yb + in.off[i] / 2u));
            }
        }
    }
}

// The compensated layers take both loads through buffer resources; the plain
// ones take the blocks through scalar-base global loads and the tables through
// buffer resources only inside the batch kernel (BATCH).
template <typename T, int MODE, int COMP, int RT, bool WIDE, bool BATCH = false>
__device__ __forceinline__ void tile(const LayerParams &p, const DescRegs<WIDE> &dr, const Leaf &L,
                                     const typename Cx<T>::type *__restrict__ X,
                                     const typename Cx<T>::type *u_lds, const typename Cx<T>::type *lowbuf,
                                     float sigma, uint32_t t0, int lane, double &psum, float &omax)
{
    TileIn<T, RT> in;
    constexpr bool comp = COMP != SLOS_COMP_NONE;
    tile_load<T, MODE, RT, WIDE, comp, comp || BATCH>(in, p, dr, L, X, t0, lane);
    tile_compute<T, MODE, COMP, RT, WIDE, BATCH>(in, p, dr, L, X, u_lds, lowbuf, sigma, t0, lane, psum, omax);
}

// Outputs per 64-byte sector: complex values, or probabilities in MODE_PROB.
template <typename T, int MODE> constexpr uint32_t kStoreAlign()
{
    return 64u / (uint32_t)(MODE == SLOS_MODE_PROB ? sizeof(T) : 2 * sizeof(T));
}

// Stage the low block with all waves of the workgroup: 1 KiB chunk c of the
// copy is issued by wave c % W (cache policy as for stage_low).
template <typename C, int CPOL>
__device__ __forceinline__ const C *stage_low_team(const C *__restrict__ X, const Leaf &L, unsigned char *slice,
                                                   int lane, int wv, int W)
{
    const uintptr_t sa = (uintptr_t)(X + L.low_base);
    const uintptr_t a0 = sa & ~(uintptr_t)15;
    const uint32_t skew = (uint32_t)(sa - a0);
    const uint32_t nbytes = skew + L.low_size * (uint32_t)sizeof(C);
    for (uint32_t done = 1024u * (uint32_t)wv; done < nbytes; done += 1024u * (uint32_t)W) {
        if (done + 16u * (uint32_t)lane < nbytes) {
            const void *src = (const void *)(a0 + done + 16u * (uint32_t)lane);
            __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)(slice + done), 16, 0,
                                             CPOL);
        }
    }
    return (const C *)(slice + skew);
}

// One workgroup (W waves) computes one leaf at a time: it stages the leaf's
// low block once in LDS and deals the leaf's tiles out to its waves.  Leaves
// come from per-XCD ticket counters in batches of p.ticket_leaves, so the
// workgroups resident on an XCD work on neighbouring leaves of the colex order
// and share that XCD's L2.
// Register budgets: complex64 two-output tiles to six waves per SIMD (80
// VGPRs; six workgroups' low blocks of up to 24 KiB fit a CU's LDS), other
// complex64 tiles to three (168 VGPRs), complex128 tiles of up to two outputs
// per lane to four (128 VGPRs)
template <typename T, int MODE, int COMP, int RR, bool WIDE>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? (RR == 2 ? 6 : 3) : (RR <= 2 ? 4 : 1)) void layer_kernel(LayerParams p)
{
    using C = typename Cx<T>::type;
    if (blockIdx.y) {
        // instance blockIdx.y of a batch of unitaries through one plan
        const uint64_t b = blockIdx.y;
        p.X = (const char *)p.X + b * p.x_stride;
        p.Y = (char *)p.Y + b * p.y_stride;
        p.U = (const char *)p.U + b * p.u_stride;
        p.partials += b * p.partials_stride;
        p.tickets += b * p.ticket_stride;
        if (p.vmax_in) p.vmax_in += b * p.ticket_stride;
        if (p.vmax_out) p.vmax_out += b * p.ticket_stride;
    }
    // Column p.col of U; entries m..255 stay zero (padded predecessor
    // entries name mode SLOS_ZERO_MODE = 255).
    __shared__ C u_lds[256];
    __shared__ uint32_t ticket_slot[2];
    // the low-block slice; 16-byte aligned for the 16-byte LDS reads of
    // complex128 elements
    extern __shared__ __align__(16) unsigned char dyn_lds[];
    unsigned char *slice = dyn_lds;
    const C *__restrict__ X = (const C *)p.X;
    const C *__restrict__ Um = (const C *)p.U;
    for (int j = threadIdx.x; j < 256; j += blockDim.x) {
        C v{0, 0};
        if (j < p.m) v = Um[(size_t)j * p.m + p.col];
        u_lds[j] = v;
    }

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int W = blockDim.x >> 6;

    // This (virtual) XCD owns chunks xcd, xcd + SLOS_XCDS, ... of xcd_chunk
    // leaves.  Workgroups are dealt to the XCDs round-robin, so
    // blockIdx.x % SLOS_XCDS names the XCD; correctness does not depend on it.
    const uint32_t xcd = blockIdx.x % SLOS_XCDS;
    const uint64_t G = p.xcd_chunk;
    const uint64_t nchunk = (p.nleaves + G - 1) / G;
    const uint64_t owned_chunks = nchunk > xcd ? (nchunk - xcd + SLOS_XCDS - 1) / SLOS_XCDS : 0;
    const uint64_t owned = owned_chunks * G;
    auto to_leaf = [&](uint64_t local) -> uint64_t {
        if (local >= owned) return p.nleaves;
        const uint64_t g = ((local / G) * SLOS_XCDS + xcd) * G + local % G;
        return g < p.nleaves ? g : p.nleaves;  // slots past the end only in the last chunk
    };
    uint32_t *ticket = p.tickets + (size_t)xcd * SLOS_TICKET_STRIDE;
    const uint32_t TB = p.ticket_leaves;

    // first batch
    if (threadIdx.x == 0) ticket_slot[0] = atomicAdd(ticket, TB);
    __syncthreads();
    uint64_t bat_next = ticket_slot[0], bat_end = bat_next + TB;
    uint64_t li = to_leaf(bat_next++);
    DescRegs<WIDE> cur{0u, 0u};
    if (li < p.nleaves) cur = load_desc<WIDE>(p.desc, li, lane);
    uint32_t it = 0;

    // Compensated bias of this layer: every output sums at most one term per
    // mode, so sum |Re,Im products| <= (sum_j |Re u_j| + |Im u_j|) * vmax with
    // vmax = max over A_{k-1} of |Re x| + |Im x| (recorded by the previous
    // layer; 1 for the vacuum).
    float sigma = 0.f, omax = 0.f;
    if constexpr (COMP == SLOS_COMP_BIASED) {
        float l1 = 0.f;
        for (int j = lane; j < p.m; j += 64) l1 += (float)(fabs(u_lds[j].x) + fabs(u_lds[j].y));
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) l1 += __shfl_xor(l1, o, 64);
        const float vin = p.vmax_in ? __uint_as_float(*p.vmax_in) : 1.0f;
        sigma = bias_for(l1 * vin * 1.001f);
    }

    while (li < p.nleaves) {
        const Leaf L = decode_head<WIDE>(cur);
        const C *lowbuf =
            stage_low_team<C, MODE == SLOS_MODE_MID ? SLOS_CPOL_DEFAULT : SLOS_CPOL_NT>(X, L, slice, lane, wv, W);
        const bool refill = bat_next >= bat_end;
        // Refills alternate between the two slots starting with slot 1: the
        // slot written in iteration it is read after this iteration's barrier
        // and written again only in iteration it + 2, after every wave has
        // passed the barrier that ends iteration it + 1 (slot 0 holds the
        // first ticket until the barrier that ends iteration 0).
        if (refill && threadIdx.x == 0) ticket_slot[(it + 1) & 1] = atomicAdd(ticket, TB);
        // the staged block has landed in LDS for every wave
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (refill) {
            bat_next = ticket_slot[(it + 1) & 1];
            bat_end = bat_next + TB;
        }
        const uint64_t nli = to_leaf(bat_next++);
        DescRegs<WIDE> nxt{0u, 0u};
        if (nli < p.nleaves) nxt = load_desc<WIDE>(p.desc, nli, lane);

        double psum = 0.0;
        // Tiles start `shift` states before the leaf, so that every row of 64
        // outputs is stored on whole 64-byte sectors (a row that straddles
        // sectors writes each partial sector separately: +11% write traffic for
        // complex64).  Lanes before the leaf wrap to x >= L.size and are masked
        // like those past its end.
        const uint32_t shift = (uint32_t)L.out_base & (kStoreAlign<T, MODE>() - 1u);
        const uint32_t span = L.size + shift;
        const uint32_t full = span / (64u * RR);              // full tiles
        for (uint32_t t = (uint32_t)wv; t < full; t += (uint32_t)W)
            tile<T, MODE, COMP, RR, WIDE>(p, cur, L, X, u_lds, lowbuf, sigma, t * 64u * RR - shift, lane, psum, omax);
        const uint32_t rows = (span - full * 64u * RR + 63u) / 64u;  // leftover rows of 64
        for (uint32_t r = (uint32_t)wv; r < rows; r += (uint32_t)W)
            tile<T, MODE, COMP, 1, WIDE>(p, cur, L, X, u_lds, lowbuf, sigma, full * 64u * RR + r * 64u - shift, lane,
                                         psum, omax);
        if (MODE != SLOS_MODE_MID) {
            // one FP64 partial per (leaf, wave), summed later in a fixed order
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) psum += __shfl_xor(psum, off, 64);
            if (lane == 0) p.partials[li * (uint64_t)W + (uint64_t)wv] = psum;
        }
        // every wave is done with this low block before the next copy lands
        // (the barrier's workgroup-scope fence waits for the waves' LDS reads;
        // their global stores may still be in flight, nothing here reads them)
        __syncthreads();
        cur = nxt;
        li = nli;
        ++it;
    }
    if (sizeof(T) == 4 && MODE == SLOS_MODE_MID && p.vmax_out) {
        // one atomic per workgroup, and only if it raises the recorded value
        // (all workgroups of a layer share the slot); non-negative floats
        // order like their bit patterns
        __shared__ float wmax[4];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) omax = fmaxf(omax, __shfl_xor(omax, o, 64));
        if (lane == 0) wmax[wv] = omax;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < W; ++w) omax = fmaxf(omax, wmax[w]);
            const uint32_t bits = __float_as_uint(omax);
            if (bits > __hip_atomic_load(p.vmax_out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                atomicMax(p.vmax_out, bits);
        }
    }
}

// ---- batches ----------------------------------------------------------------------
// Phase 1: the workgroup runs its cooperative instances whole, layer after
// layer; its waves take the layer's leaves in turn (each wave stages its leaf's
// low block in its own LDS slice) and a barrier separates layers.  Phase 2:
// each wave runs its own small instances alone, layer after layer, with its
// own U column and scratch pair, ordering its layers with a fence instead of a
// barrier.  Last layers go straight to the packed output.  The host assigns the
// instances (largest first, to the least loaded workgroup or wave), so no
// workgroup waits on another and the schedule is fixed.
template <typename T, int RR>
__device__ __forceinline__ void batch_layer_leaves(const BatchParams &bp, const BatchInst &I, int k, const void *Xv,
                                                   void *Yv, const typename Cx<T>::type *u, unsigned char *slice,
                                                   uint32_t first, uint32_t step, int lane, double &psum)
{
    using C = typename Cx<T>::type;
    const C *X = (const C *)Xv;
    const int n = (int)I.n;
    float bmax = 0.f;  // unused: batches are not compensated
    LayerParams lp{};
    lp.Y = Yv;
    lp.pred = bp.pred;
    lp.lowfac = bp.lowfac;
    const uint32_t nl = I.nleaves[k - 1];
    for (uint32_t li = first; li < nl; li += step) {
        const DescRegs<false> d = load_desc<false, true>(bp.desc, (uint64_t)I.desc_off[k - 1] + li, lane);
        const Leaf L = decode_head<false>(d);
        const C *lowbuf = stage_low<C>(X, L, slice, lane);
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
        const uint32_t full = L.size / (64u * RR);
        if (k == n) {
            for (uint32_t t = 0; t < full; ++t)
                tile<T, SLOS_MODE_AMPL, SLOS_COMP_NONE, RR, false, true>(lp, d, L, X, u, lowbuf, 0.f, t * 64u * RR, lane,
                                                                  psum, bmax);
            for (uint32_t t0 = full * 64u * RR; t0 < L.size; t0 += 64u)
                tile<T, SLOS_MODE_AMPL, SLOS_COMP_NONE, 1, false, true>(lp, d, L, X, u, lowbuf, 0.f, t0, lane, psum, bmax);
        } else {
            for (uint32_t t = 0; t < full; ++t)
                tile<T, SLOS_MODE_MID, SLOS_COMP_NONE, RR, false, true>(lp, d, L, X, u, lowbuf, 0.f, t * 64u * RR, lane,
                                                                 psum, bmax);
            for (uint32_t t0 = full * 64u * RR; t0 < L.size; t0 += 64u)
                tile<T, SLOS_MODE_MID, SLOS_COMP_NONE, 1, false, true>(lp, d, L, X, u, lowbuf, 0.f, t0, lane, psum, bmax);
        }
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
    }
}

template <typename T, int RR, int MAXT>
__global__ __launch_bounds__(MAXT) void batch_kernel(BatchParams bp)
{
    using C = typename Cx<T>::type;
    __shared__ C u_lds[256];
    __shared__ double wsum[MAXT / 64];
    extern __shared__ __align__(16) unsigned char dyn_lds[];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int W = blockDim.x >> 6;
    unsigned char *slice = dyn_lds + (size_t)wv * bp.lds_wave_bytes;
    C *u_own = (C *)(dyn_lds + (size_t)W * bp.lds_wave_bytes) + (size_t)wv * 256;
    const C *Ub = (const C *)bp.U;

    // phase 1: cooperative instances
    {
        C *scr[2];
        scr[0] = (C *)bp.scratch + bp.wg_scr[blockIdx.x];
        scr[1] = scr[0] + bp.scratch_stride;
        for (uint32_t e = bp.wg_start[blockIdx.x]; e < bp.wg_start[blockIdx.x + 1]; ++e) {
            const uint32_t ii = bp.wg_list[e];
            const BatchInst &I = bp.inst[ii];
            const int m = (int)I.m, n = (int)I.n;
            double psum = 0.0;
            for (int k = 1; k <= n; ++k) {
                __syncthreads();  // layer k-1 is complete and every LDS slice is free
                const int col = I.col[k - 1];
                for (int j = threadIdx.x; j < 256; j += blockDim.x) {
                    C v{0, 0};
                    if (j < m) v = Ub[I.U_off + (size_t)j * m + col];
                    u_lds[j] = v;
                }
                __syncthreads();
                const void *X = k == 1 ? bp.vac : (const void *)scr[(k - 1) & 1];
                void *Y = k == n ? (void *)((C *)bp.out + I.out_off) : (void *)scr[k & 1];
                batch_layer_leaves<T, RR>(bp, I, k, X, Y, u_lds, slice, (uint32_t)wv, (uint32_t)W, lane, psum);
            }
            // sum P of the instance: per wave, then over waves in order
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) psum += __shfl_xor(psum, off, 64);
            __syncthreads();
            if (lane == 0) wsum[wv] = psum;
            __syncthreads();
            if (threadIdx.x == 0 && bp.sum_p) {
                double s = 0.0;
                for (int w = 0; w < W; ++w) s += wsum[w];
                bp.sum_p[ii] = s;
            }
        }
    }

    // phase 2: this wave's own instances
    const uint32_t slot = blockIdx.x * (uint32_t)W + (uint32_t)wv;
    C *my[2];
    my[0] = (C *)bp.scratch + bp.small_base + (uint64_t)slot * 2 * bp.small_stride;
    my[1] = my[0] + bp.small_stride;
    for (uint32_t e = bp.wv_start[slot]; e < bp.wv_start[slot + 1]; ++e) {
        const uint32_t ii = bp.wv_list[e];
        const BatchInst &I = bp.inst[ii];
        const int m = (int)I.m, n = (int)I.n;
        double psum = 0.0;
        if (n == 0 && lane == 0) {
            // no photons: the single output is the vacuum, amplitude 1
            ((C *)bp.out)[I.out_off] = C{(T)1, (T)0};
            psum = 1.0;
        }
        for (int k = 1; k <= n; ++k) {
            const int col = I.col[k - 1];
            for (int j = lane; j < 256; j += 64) {
                C v{0, 0};
                if (j < m) v = Ub[I.U_off + (size_t)j * m + col];
                u_own[j] = v;
            }
            __builtin_amdgcn_s_waitcnt(0);
            __builtin_amdgcn_wave_barrier();
            const void *X = k == 1 ? bp.vac : (const void *)my[(k - 1) & 1];
            void *Y = k == n ? (void *)((C *)bp.out + I.out_off) : (void *)my[k & 1];
            batch_layer_leaves<T, RR>(bp, I, k, X, Y, u_own, slice, 0u, 1u, lane, psum);
            // layer k's stores (all lanes) are seen by every lane's loads of layer k + 1
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) psum += __shfl_xor(psum, off, 64);
        if (lane == 0 && bp.sum_p) bp.sum_p[ii] = psum;
    }
}

// Deterministic two-stage sum of the per-leaf partials: workgroup b sums its
// fixed contiguous segment (strided per thread, then a fixed LDS tree) into
// stage[b]; a single workgroup then sums stage[] the same way.
constexpr int kReduceBlocks = 256;

__device__ __forceinline__ double block_sum(double s)
{
    __shared__ double sh[256];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    return sh[0];
}

__global__ __launch_bounds__(256) void reduce_stage1(const double *__restrict__ part, int64_t count,
                                                     double *__restrict__ stage, int64_t stride)
{
    // batch entry blockIdx.y: partials at part + y * stride, stage row y
    part += (int64_t)blockIdx.y * stride;
    stage += (int64_t)blockIdx.y * kReduceBlocks;
    const int64_t seg = (count + kReduceBlocks - 1) / kReduceBlocks;
    const int64_t lo = (int64_t)blockIdx.x * seg;
    const int64_t hi = lo + seg < count ? lo + seg : count;
    double s = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) s += part[i];
    s = block_sum(s);
    if (threadIdx.x == 0) stage[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void reduce_stage2(const double *__restrict__ stage, double *__restrict__ out)
{
    stage += (int64_t)blockIdx.x * kReduceBlocks;
    out += blockIdx.x;
    const double s = block_sum(threadIdx.x < kReduceBlocks ? stage[threadIdx.x] : 0.0);
    if (threadIdx.x == 0) *out = s;
}

__global__ void zero_u32_kernel(uint32_t *buf, int count)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) buf[i] = 0u;
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

template <typename T, int MODE, int COMP, int RR, bool WIDE>
hipError_t launch_one(const LayerParams &p, const LayerLaunch &l, hipStream_t s)
{
    static bool attr_set = false;  // per instantiation; first call per process
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)layer_kernel<T, MODE, COMP, RR, WIDE>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)SLOS_LDS_DYNAMIC_MAX);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const size_t lds = (size_t)p.lds_wave_bytes;  // one low block per workgroup
    hipLaunchKernelGGL((layer_kernel<T, MODE, COMP, RR, WIDE>), dim3(l.grid, l.batch > 1 ? l.batch : 1),
                       dim3(l.threads), lds, s, p);
    return hipGetLastError();
}


template <typename T, int MODE, int COMP, bool WIDE>
hipError_t launch_rr(const LayerParams &p, const LayerLaunch &l, hipStream_t s)
{
    switch (l.rr) {
    case 1: return launch_one<T, MODE, COMP, 1, WIDE>(p, l, s);
    case 2: return launch_one<T, MODE, COMP, 2, WIDE>(p, l, s);
    default: return launch_one<T, MODE, COMP, 4, WIDE>(p, l, s);
    }
}

template <typename T, int MODE, int COMP>
hipError_t launch_wide(const LayerParams &p, const LayerLaunch &l, hipStream_t s)
{
    return l.wide ? launch_rr<T, MODE, COMP, true>(p, l, s) : launch_rr<T, MODE, COMP, false>(p, l, s);
}

template <typename T, int COMP>
hipError_t launch_mode(const LayerParams &p, const LayerLaunch &l, hipStream_t s)
{
    switch (l.mode) {
    case SLOS_MODE_AMPL: return launch_wide<T, SLOS_MODE_AMPL, COMP>(p, l, s);
    case SLOS_MODE_PROB: return launch_wide<T, SLOS_MODE_PROB, COMP>(p, l, s);
    default: return launch_wide<T, SLOS_MODE_MID, COMP>(p, l, s);
    }
}

} // namespace

int slos_launch_layer(const LayerParams &p, const LayerLaunch &l, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (l.c64) {
        if (l.compensated == SLOS_COMP_BIASED) return (int)launch_mode<float, SLOS_COMP_BIASED>(p, l, s);
        if (l.compensated == SLOS_COMP_TWOSUM) return (int)launch_mode<float, SLOS_COMP_TWOSUM>(p, l, s);
        if (l.compensated == SLOS_COMP_F64) return (int)launch_mode<float, SLOS_COMP_F64>(p, l, s);
        return (int)launch_mode<float, SLOS_COMP_NONE>(p, l, s);
    }
    return (int)launch_mode<double, SLOS_COMP_NONE>(p, l, s);
}

int slos_launch_reduce(const double *partials, int64_t count, double *stage, double *out, void *stream, int batch,
                       int64_t stride)
{
    hipLaunchKernelGGL(reduce_stage1, dim3(kReduceBlocks, batch), dim3(256), 0, (hipStream_t)stream, partials, count,
                       stage, stride);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    hipLaunchKernelGGL(reduce_stage2, dim3(batch), dim3(256), 0, (hipStream_t)stream, stage, out);
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

int slos_launch_zero_u32(uint32_t *buf, int count, void *stream)
{
    const int grid = std::max(1, std::min((count + 255) / 256, 1024));
    hipLaunchKernelGGL(zero_u32_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, buf, count);
    return (int)hipGetLastError();
}

template <typename T, int RR, int MAXT>
static hipError_t batch_attr()
{
    return hipFuncSetAttribute((const void *)batch_kernel<T, RR, MAXT>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)SLOS_LDS_DYNAMIC_MAX);
}

template <int MAXT>
static hipError_t batch_attrs()
{
    hipError_t e;
    if ((e = batch_attr<float, 1, MAXT>()) || (e = batch_attr<float, 2, MAXT>()) ||
        (e = batch_attr<float, 4, MAXT>()) || (e = batch_attr<double, 1, MAXT>()) ||
        (e = batch_attr<double, 2, MAXT>()) || (e = batch_attr<double, 4, MAXT>()))
        return e;
    return hipSuccess;
}

int slos_prepare_batch_kernels(void)
{
    hipError_t e;
    if ((e = batch_attrs<256>()) || (e = batch_attrs<1024>())) return (int)e;
    return 0;
}

template <int MAXT>
static void launch_batch(const BatchParams &p, int c64, int rr, dim3 g, dim3 b, size_t lds, hipStream_t s)
{
    if (c64) {
        if (rr == 1) hipLaunchKernelGGL((batch_kernel<float, 1, MAXT>), g, b, lds, s, p);
        else if (rr == 2) hipLaunchKernelGGL((batch_kernel<float, 2, MAXT>), g, b, lds, s, p);
        else hipLaunchKernelGGL((batch_kernel<float, 4, MAXT>), g, b, lds, s, p);
    } else {
        if (rr == 1) hipLaunchKernelGGL((batch_kernel<double, 1, MAXT>), g, b, lds, s, p);
        else if (rr == 2) hipLaunchKernelGGL((batch_kernel<double, 2, MAXT>), g, b, lds, s, p);
        else hipLaunchKernelGGL((batch_kernel<double, 4, MAXT>), g, b, lds, s, p);
    }
}

// Workgroups of up to 256 threads keep the 256-thread register budget; 512 and
// 1024 (more waves on the cooperative instances) take the 1024-thread one.
int slos_launch_batch(const BatchParams &p, int c64, int rr, int threads, int grid, void *stream)
{
    const size_t lds = ((size_t)p.lds_wave_bytes + 256 * (c64 ? 8 : 16)) * (size_t)(threads / 64);
    const hipStream_t s = (hipStream_t)stream;
    if (threads <= 256) launch_batch<256>(p, c64, rr, dim3(grid), dim3(threads), lds, s);
    else launch_batch<1024>(p, c64, rr, dim3(grid), dim3(threads), lds, s);
    return (int)hipGetLastError();
}

