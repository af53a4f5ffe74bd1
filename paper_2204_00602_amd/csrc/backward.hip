// HIP kernels (gfx950) for differentiation: the adjoint of the SLOS layer
// recurrence and the rectangular MZI mesh (phases -> U and its reverse sweep).
//
// Forward layer (arXiv 2204.00602, Section 3.2.3 recurrence):
//     A_k[t] = sum_j U[j, i_k] A_{k-1}[t - e_j].
// With g = dL/d conj(.) (the PyTorch convention for a real loss L), the
// reverse of one layer is
//     g_{k-1}[t'] = sum_j conj(U[j, i_k]) g_k[t' + e_j]          (every mode j)
//     G_U[j, i_k] += sum_{t'} g_k[t' + e_j] conj(A_{k-1}[t'])
// and the last-layer normalisation a = c_S A_n[S] (c_S real) seeds
//     g_n[S] = c_S g_a[S].
// Work unit: the low block of one forward leaf of layer k (these blocks
// partition A_{k-1}); one wave per unit, every output written by one lane, no
// atomics.  Gradient partials are kept per (unit, mode) and summed in a fixed
// order.
#include <hip/hip_runtime.h>

#include "slos_internal.h"

namespace {

template <typename T> struct Cb;
template <> struct Cb<float> { using type = float2; };
template <> struct Cb<double> { using type = double2; };

// ---- seed: g_n = c_S * g_a over the last layer's leaves --------------------
// One wave per leaf.  (Eight waves per leaf, one row of 64 states each, measured
// slower at m=12 n=6 with 64 instances: 10.5 against 8.9 us.)
template <typename T>
__global__ __launch_bounds__(256) void seed_kernel(const LeafDescHead *__restrict__ heads, uint64_t nleaves,
                                                   uint32_t stride_bytes, const double *__restrict__ lowfac,
                                                   const typename Cb<T>::type *__restrict__ ga,
                                                   typename Cb<T>::type *__restrict__ gn, uint64_t ga_stride,
                                                   uint64_t gn_stride)
{
    using C = typename Cb<T>::type;
    // instance blockIdx.y: element offsets
    ga += blockIdx.y * ga_stride;
    gn += blockIdx.y * gn_stride;
    const int lane = threadIdx.x & 63;
    const uint64_t gw = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint64_t nw = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t li = gw; li < nleaves; li += nw) {
        const LeafDescHead h = *(const LeafDescHead *)((const char *)heads + li * stride_bytes);
        for (uint32_t x = lane; x < h.size; x += 64) {
            const double f = h.fac_hi * lowfac[h.fac_off + x];
            const C v = ga[h.out_base + x];
            gn[h.out_base + x] = C{(T)(f * (double)v.x), (T)(f * (double)v.y)};
        }
    }
}

// ---- one reverse layer --------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(64) void bwd_layer_kernel(BwdParams p)
{
    using C = typename Cb<T>::type;
    __shared__ C uc[256];                  // conj(U[j, i_k])
    extern __shared__ double2 part[];      // [jn][64] gradient partials of this wave
    if (blockIdx.y) {
        // instance blockIdx.y of a batch of unitaries through one plan
        const uint64_t b = blockIdx.y;
        p.gk = (const char *)p.gk + b * p.gk_stride;
        p.gkm1 = (char *)p.gkm1 + b * p.gkm1_stride;
        p.Akm1 = (const char *)p.Akm1 + b * p.a_stride;
        p.U = (const char *)p.U + b * p.u_stride;
        p.partials = (char *)p.partials + b * p.partials_stride;
    }
    const C *__restrict__ gk = (const C *)p.gk;
    C *__restrict__ gkm1 = (C *)p.gkm1;
    const C *__restrict__ A = (const C *)p.Akm1;
    const C *__restrict__ Um = (const C *)p.U;
    const int lane = threadIdx.x;
    for (int j = lane; j < 256; j += 64) {
        C v{0, 0};
        if (j < p.m) {
            v = Um[(size_t)j * p.m + p.col];
            v.y = -v.y;
        }
        uc[j] = v;
    }
    __syncthreads();

    for (uint64_t u = blockIdx.x; u < p.nunits; u += gridDim.x) {
        const BwdUnit U = p.units[u];
        for (int j = 0; j < p.jn; ++j) part[j * 64 + lane] = double2{0.0, 0.0};
        const uint32_t *__restrict__ succ = p.succ + U.succ_off;
        const uint64_t *__restrict__ hb = p.hbase + U.hbase_off;
        const uint32_t yend = U.low_size - U.y0 < p.chunk ? U.low_size : U.y0 + p.chunk;
        for (uint32_t y0 = U.y0; y0 < yend; y0 += 64) {
            const uint32_t y = y0 + lane;
            const bool ok = y < yend;
            const uint32_t yc = ok ? y : yend - 1u;
            const C a = A[U.low_base + yc];
            const double ar = (double)a.x, ai = (double)a.y;
            double accr = 0.0, acci = 0.0;
            // the pass that forms g_{k-1} visits every mode, the others only
            // their block of partials
            const int jlo = p.write_g ? 0 : p.jb;
            const int jhi = p.write_g ? p.m : p.jb + p.jn;
            // four successor modes per step, their loads issued first (modes in
            // ascending order within and across steps, so the sums keep one order)
            for (int j0 = jlo; j0 < jhi; j0 += 4) {
                C sv[4];
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const int j = j0 + d < jhi ? j0 + d : j0;
                    // successor t' + e_j: inside the forward leaf for a low mode,
                    // the aligned block of the high part + e_j otherwise
                    const uint64_t pos = j < (int)U.q ? U.out_base + succ[(size_t)j * U.low_size + yc]
                                                      : hb[j - (int)U.q] + yc;
                    sv[d] = gk[pos];
                }
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const int j = j0 + d;
                    if (j >= jhi) break;
                    const double sr = (double)sv[d].x, si = (double)sv[d].y;
                    const double ur = (double)uc[j].x, ui = (double)uc[j].y;
                    accr += ur * sr - ui * si;
                    acci += ur * si + ui * sr;
                    const int jj = j - p.jb;
                    if (ok && jj >= 0 && jj < p.jn) {
                        // s * conj(a)
                        double2 &pj = part[jj * 64 + lane];
                        pj.x += sr * ar + si * ai;
                        pj.y += si * ar - sr * ai;
                    }
                }
            }
            if (ok && p.write_g) gkm1[U.low_base + y] = C{(T)accr, (T)acci};
        }
        // reduce this unit's partials over lanes in a fixed tree
        __syncthreads();
        for (int j = 0; j < p.jn; ++j) {
            double2 v = part[j * 64 + lane];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                v.x += __shfl_xor(v.x, off, 64);
                v.y += __shfl_xor(v.y, off, 64);
            }
            if (lane == 0) ((double2 *)p.partials)[u * (uint64_t)p.m + p.jb + j] = v;
        }
        __syncthreads();
    }
}

// One launch after all reverse layers: for every layer k, colsum_k[j] = sum over
// the layer's units u of partials_k[u][j], formed by one wave in a fixed order
// (per lane over u = lane, lane + 64, ..., then a butterfly over the 64 lanes;
// wave w takes layers w, w + 4, ...), then G_U[j, i] = sum over layers k with
// i_k = i of colsum_k[j], in order of k.
template <typename T>
__global__ __launch_bounds__(256) void colsum_gradu_kernel(const double2 *__restrict__ partials, ColsumLayers L,
                                                            const int32_t *__restrict__ photons, int n, int m,
                                                            typename Cb<T>::type *__restrict__ GU,
                                                            uint64_t partials_stride, uint64_t gu_stride)
{
    using C = typename Cb<T>::type;
    __shared__ double2 cs[SLOS_MAX_PHOTONS];
    partials += blockIdx.y * partials_stride;  // instance blockIdx.y (element strides)
    GU += blockIdx.y * gu_stride;
    const int j = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int W = blockDim.x >> 6;
    for (int k = threadIdx.x >> 6; k < n; k += W) {
        const double2 *pk = partials + L.off[k];
        double2 s{0.0, 0.0};
        for (uint64_t u = (uint64_t)lane; u < L.nunits[k]; u += 64) {
            const double2 v = pk[u * (uint64_t)m + j];
            s.x += v.x;
            s.y += v.y;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            s.x += __shfl_xor(s.x, off, 64);
            s.y += __shfl_xor(s.y, off, 64);
        }
        if (lane == 0) cs[k] = s;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        double gr = 0.0, gi = 0.0;
        for (int k = 0; k < n; ++k)
            if (photons[k] == i) {
                gr += cs[k].x;
                gi += cs[k].y;
            }
        GU[(size_t)j * m + i] = C{(T)gr, (T)gi};
    }
}

// The squared-error loss on target outputs of a batch and its gradient with
// respect to the amplitudes.  One workgroup per instance b:
//   L_b = sum_t (|a_b(r_t)|^2 - P_t[b, t])^2 in FP64 (fixed-order sum), and
//   grad_a[b] = 4 (|a_b(r_t)|^2 - P_t[b, t]) a_b(r_t) at r_t, 0 elsewhere
// (the PyTorch-convention gradient d L / d Re a + i d L / d Im a).  The zeros are
// stored and complete before any target value is written to the same row.
template <typename T>
__global__ __launch_bounds__(256) void sq_loss_kernel(const typename Cb<T>::type *__restrict__ a, uint64_t M,
                                                       const int64_t *__restrict__ ranks, int64_t count,
                                                       const double *__restrict__ p_target,
                                                       typename Cb<T>::type *__restrict__ grad_a,
                                                       double *__restrict__ loss)
{
    using C = typename Cb<T>::type;
    __shared__ double sh[256];
    const uint64_t b = blockIdx.x;
    a += b * M;
    grad_a += b * M;
    p_target += b * (uint64_t)count;
    for (uint64_t r = threadIdx.x; r < M; r += 256) grad_a[r] = C{(T)0, (T)0};
    __builtin_amdgcn_s_waitcnt(0);  // this wave's zeros have reached memory
    __syncthreads();
    double s = 0.0;
    for (int64_t t = threadIdx.x; t < count; t += 256) {
        const int64_t r = ranks[t];
        if (r < 0 || (uint64_t)r >= M) continue;  // outside the output set: ignored
        const C v = a[r];
        const double P = (double)v.x * (double)v.x + (double)v.y * (double)v.y;
        const double d = P - p_target[t];
        s += d * d;
        const T f = (T)(4.0 * d);
        grad_a[r] = C{f * v.x, f * v.y};
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) loss[b] = sh[0];
}

// The same loss with the seed of the adjoint fused in: g_n[b] = c_S grad_a[b]
// at the targets (c_S = scale[t], the normalisation a(S) = c_S A_n[S]) and 0
// elsewhere, written straight into the last layer's gradient buffer (row b at
// b * gn_stride).  Workgroup (x, b) owns states [x * SLOS_SEED_SLICE, ...) of
// row b: it zeroes them, then writes the targets among them; workgroup 0 of
// the row also forms the loss over all targets.  The values are formed
// exactly as the loss kernel and the seed kernel form them one after the
// other, and the loss in the same order, so the results are the same.
#define SLOS_SEED_SLICE 2048u
template <typename T>
__global__ __launch_bounds__(256) void sq_loss_seed_kernel(const typename Cb<T>::type *__restrict__ a, uint64_t M,
                                                            const int64_t *__restrict__ ranks,
                                                            const double *__restrict__ scale, int64_t count,
                                                            const double *__restrict__ p_target,
                                                            typename Cb<T>::type *__restrict__ gn,
                                                            uint64_t gn_stride, double *__restrict__ loss)
{
    using C = typename Cb<T>::type;
    __shared__ double sh[256];
    const uint64_t b = blockIdx.y;
    a += b * M;
    gn += b * gn_stride;
    p_target += b * (uint64_t)count;
    const uint64_t lo = (uint64_t)blockIdx.x * SLOS_SEED_SLICE;
    const uint64_t hi = lo + SLOS_SEED_SLICE < M ? lo + SLOS_SEED_SLICE : M;
    for (uint64_t r = lo + threadIdx.x; r < hi; r += 256) gn[r] = C{(T)0, (T)0};
    __builtin_amdgcn_s_waitcnt(0);  // this wave's zeros have reached memory
    __syncthreads();
    double s = 0.0;
    for (int64_t t = threadIdx.x; t < count; t += 256) {
        const int64_t r = ranks[t];
        if (r < 0 || (uint64_t)r >= M) continue;  // outside the output set: ignored
        const bool mine = (uint64_t)r >= lo && (uint64_t)r < hi;
        if (!mine && blockIdx.x != 0) continue;
        const C v = a[r];
        const double P = (double)v.x * (double)v.x + (double)v.y * (double)v.y;
        const double d = P - p_target[t];
        s += d * d;
        if (mine) {
            const T f = (T)(4.0 * d);
            const C ga{f * v.x, f * v.y};
            const double c = scale[t];
            gn[r] = C{(T)(c * (double)ga.x), (T)(c * (double)ga.y)};
        }
    }
    if (blockIdx.x != 0) return;
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) loss[b] = sh[0];
}

// ---- rectangular MZI mesh --------------------------------------------------------
// MZI(a, b) = PS_1(b) BS PS_0(a) BS with BS = [[c, i s], [i s, c]] at theta = pi/2
// (Eq. eq:bs): the composition BS, PS(phi_a) on mode 0, BS, PS(phi_b) on mode 1.
// Column c holds MZIs on (p, p+1), p = c mod 2, c mod 2 + 2, ..., p + 1 < m, in
// this order; U = T_last ... T_first.
struct Cd {
    double x, y;
};
__device__ __forceinline__ Cd cmul(Cd a, Cd b) { return Cd{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ Cd cadd(Cd a, Cd b) { return Cd{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ Cd cconj(Cd a) { return Cd{a.x, -a.y}; }

// 2x2 MZI block B and its derivatives dB/da, dB/db, from e^{ia} and e^{ib}
__device__ void mzi_block_e(Cd ea, Cd eb, Cd B[4], Cd dA[4], Cd dBb[4])
{
    const double r = 0.70710678118654752440;  // cos(pi/4) = sin(pi/4)
    // BS * BS-like products written out: BS = r [[1, i], [i, 1]]
    // M = BS PS0(a) BS = r^2 [[e^{ia} - 1, i(e^{ia} + 1)], [i(e^{ia} + 1), -e^{ia} + 1]]
    const double h = r * r;
    const Cd m00{h * (ea.x - 1.0), h * ea.y};
    const Cd m01{-h * ea.y, h * (ea.x + 1.0)};   // i h (e^{ia} + 1)
    const Cd m10 = m01;
    const Cd m11{h * (1.0 - ea.x), -h * ea.y};
    // B = diag(1, e^{ib}) M
    B[0] = m00;
    B[1] = m01;
    B[2] = cmul(eb, m10);
    B[3] = cmul(eb, m11);
    // dM/da: d e^{ia} = i e^{ia}
    const Cd iea{-ea.y, ea.x};
    const Cd d00{h * iea.x, h * iea.y};
    const Cd d01{-h * iea.y, h * iea.x};          // i h (i e^{ia})
    const Cd d11{-h * iea.x, -h * iea.y};
    dA[0] = d00;
    dA[1] = d01;
    dA[2] = cmul(eb, d01);
    dA[3] = cmul(eb, d11);
    const Cd ieb{-eb.y, eb.x};
    dBb[0] = Cd{0.0, 0.0};
    dBb[1] = Cd{0.0, 0.0};
    dBb[2] = cmul(ieb, m10);
    dBb[3] = cmul(ieb, m11);
}

__device__ __forceinline__ Cd cexp_i(double a)
{
    double s, c;
    sincos(a, &s, &c);
    return Cd{c, s};
}

// The phase factors e^{i phi} of one phase set: staged in LDS by all lanes at
// once when E is given (the sweeps then need no sincos on their critical path),
// else computed where they are used.
struct PhaseFactors {
    const double *ph;
    Cd *E;  // 2 * nmzi entries, or nullptr
    __device__ void stage(int nmzi, int lane, int nlanes)
    {
        if (!E) return;
        for (int i = lane; i < 2 * nmzi; i += nlanes) E[i] = cexp_i(ph[i]);
        __syncthreads();
    }
    __device__ void block(int k, Cd B[4], Cd dA[4], Cd dB[4]) const
    {
        if (E) mzi_block_e(E[2 * k], E[2 * k + 1], B, dA, dB);
        else mzi_block_e(cexp_i(ph[2 * k]), cexp_i(ph[2 * k + 1]), B, dA, dB);
    }
};

// One wave per phase set (m <= 64).  The MZIs of one mesh column act on
// disjoint row pairs, so a whole column is applied (and differentiated) in one
// step: lane l serves the column's MZI i = l / gc on matrix columns
// l % gc, l % gc + gc, .., with gc = 64 / (most MZIs in a column) rounded down
// to a power of two (8 at m = 12), and a barrier separates the m column steps.
__device__ __forceinline__ int mesh_lanes_per_mzi(int m)
{
    const int most = m / 2 > 0 ? m / 2 : 1;
    int gc = 1;
    while (gc * 2 * most <= 64) gc *= 2;
    return gc;
}

template <typename T>
__global__ __launch_bounds__(64) void mesh_forward_kernel(int m, int nmzi, const double *__restrict__ phases,
                                                          typename Cb<T>::type *__restrict__ Uout, int stage)
{
    using C = typename Cb<T>::type;
    extern __shared__ Cd Ush[];  // m x m, then 2 nmzi phase factors when staged
    const int b = blockIdx.x;
    PhaseFactors pf{phases + (size_t)b * 2 * nmzi, stage ? Ush + m * m : nullptr};
    pf.stage(nmzi, threadIdx.x, blockDim.x);
    const int lane = threadIdx.x, gc = mesh_lanes_per_mzi(m), i = lane / gc, g = lane % gc;
    for (int e = lane; e < m * m; e += 64) Ush[e] = Cd{e / m == e % m ? 1.0 : 0.0, 0.0};
    __syncthreads();
    int k0 = 0;
    for (int col = 0; col < m; ++col) {
        const int cnt = (m - col % 2) / 2;
        if (i < cnt) {
            const int p0 = col % 2 + 2 * i;
            Cd B[4], dA[4], dB[4];
            pf.block(k0 + i, B, dA, dB);
            for (int c = g; c < m; c += gc) {
                const Cd x0 = Ush[p0 * m + c], x1 = Ush[(p0 + 1) * m + c];
                Ush[p0 * m + c] = cadd(cmul(B[0], x0), cmul(B[1], x1));
                Ush[(p0 + 1) * m + c] = cadd(cmul(B[2], x0), cmul(B[3], x1));
            }
        }
        k0 += cnt;
        __syncthreads();
    }
    for (int e = lane; e < m * m; e += 64) {
        const Cd v = Ush[e];
        Uout[(size_t)b * m * m + e] = C{(T)v.x, (T)v.y};
    }
}

// Reverse sweep: with U = L_k T_k R_k, P = L_k^H G_U and Q = L_k^H U = T_k R_k,
//   dL/dphi = Re sum conj(P) o (dT_k T_k^H Q),
// then P <- T_k^H P and Q <- T_k^H Q move to the previous column (the MZIs of a
// column commute, so they share P and Q).  Each MZI's sum over matrix columns
// is per lane, then a reduction over its gc lanes in a fixed order.
template <typename T>
__global__ __launch_bounds__(64) void mesh_backward_kernel(int m, int nmzi, const double *__restrict__ phases,
                                                           const typename Cb<T>::type *__restrict__ GU,
                                                           double *__restrict__ gphases, int stage)
{
    extern __shared__ Cd sh[];  // P (m x m), Q (m x m), then 2 nmzi phase factors when staged
    Cd *P = sh;
    Cd *Q = sh + m * m;
    const int b = blockIdx.x;
    PhaseFactors pf{phases + (size_t)b * 2 * nmzi, stage ? sh + 2 * m * m : nullptr};
    pf.stage(nmzi, threadIdx.x, blockDim.x);
    const int lane = threadIdx.x, gc = mesh_lanes_per_mzi(m), i = lane / gc, g = lane % gc;
    // Q = U (rebuilt here), P = G_U
    for (int e = lane; e < m * m; e += 64) {
        Q[e] = Cd{e / m == e % m ? 1.0 : 0.0, 0.0};
        const auto v = GU[(size_t)b * m * m + e];
        P[e] = Cd{(double)v.x, (double)v.y};
    }
    __syncthreads();
    int k0 = 0;
    for (int col = 0; col < m; ++col) {
        const int cnt = (m - col % 2) / 2;
        if (i < cnt) {
            const int p0 = col % 2 + 2 * i;
            Cd B[4], dA[4], dB[4];
            pf.block(k0 + i, B, dA, dB);
            for (int c = g; c < m; c += gc) {
                const Cd x0 = Q[p0 * m + c], x1 = Q[(p0 + 1) * m + c];
                Q[p0 * m + c] = cadd(cmul(B[0], x0), cmul(B[1], x1));
                Q[(p0 + 1) * m + c] = cadd(cmul(B[2], x0), cmul(B[3], x1));
            }
        }
        k0 += cnt;
        __syncthreads();
    }
    // columns in reverse
    for (int col = m - 1; col >= 0; --col) {
        const int cnt = (m - col % 2) / 2;
        k0 -= cnt;
        double va = 0.0, vb = 0.0;
        if (i < cnt) {
            const int p0 = col % 2 + 2 * i;
            Cd B[4], dA[4], dB[4];
            pf.block(k0 + i, B, dA, dB);
            // D = dT T^H restricted to rows p0, p0+1 (2x2): D = dB B^H
            Cd Da[4], Db[4];
            for (int r = 0; r < 2; ++r)
                for (int s2 = 0; s2 < 2; ++s2) {
                    Da[2 * r + s2] =
                        cadd(cmul(dA[2 * r], cconj(B[2 * s2])), cmul(dA[2 * r + 1], cconj(B[2 * s2 + 1])));
                    Db[2 * r + s2] =
                        cadd(cmul(dB[2 * r], cconj(B[2 * s2])), cmul(dB[2 * r + 1], cconj(B[2 * s2 + 1])));
                }
            for (int c = g; c < m; c += gc) {
                const Cd q0 = Q[p0 * m + c], q1 = Q[(p0 + 1) * m + c];
                const Cd pp0 = P[p0 * m + c], pp1 = P[(p0 + 1) * m + c];
                const Cd ya0 = cadd(cmul(Da[0], q0), cmul(Da[1], q1));
                const Cd ya1 = cadd(cmul(Da[2], q0), cmul(Da[3], q1));
                const Cd yb0 = cadd(cmul(Db[0], q0), cmul(Db[1], q1));
                const Cd yb1 = cadd(cmul(Db[2], q0), cmul(Db[3], q1));
                va += pp0.x * ya0.x + pp0.y * ya0.y + pp1.x * ya1.x + pp1.y * ya1.y;
                vb += pp0.x * yb0.x + pp0.y * yb0.y + pp1.x * yb1.x + pp1.y * yb1.y;
                // P <- T^H P, Q <- T^H Q on rows p0, p0+1
                Q[p0 * m + c] = cadd(cmul(cconj(B[0]), q0), cmul(cconj(B[2]), q1));
                Q[(p0 + 1) * m + c] = cadd(cmul(cconj(B[1]), q0), cmul(cconj(B[3]), q1));
                P[p0 * m + c] = cadd(cmul(cconj(B[0]), pp0), cmul(cconj(B[2]), pp1));
                P[(p0 + 1) * m + c] = cadd(cmul(cconj(B[1]), pp0), cmul(cconj(B[3]), pp1));
            }
        }
        // sum over the gc lanes of each MZI (aligned groups of a power of two)
        for (int o = gc / 2; o > 0; o >>= 1) {
            va += __shfl_xor(va, o, 64);
            vb += __shfl_xor(vb, o, 64);
        }
        if (i < cnt && g == 0) {
            gphases[(size_t)b * 2 * nmzi + 2 * (k0 + i)] = va;
            gphases[(size_t)b * 2 * nmzi + 2 * (k0 + i) + 1] = vb;
        }
        __syncthreads();
    }
}

} // namespace

int slos_launch_seed(const void *heads, uint64_t nleaves, uint32_t stride, const double *lowfac, const void *ga,
                     void *gn, int c64, void *stream, int batch, uint64_t ga_stride, uint64_t gn_stride)
{
    const int grid = (int)(nleaves < 1024 ? (nleaves + 3) / 4 : 256);
    const dim3 g(grid > 0 ? grid : 1, batch > 1 ? batch : 1);
    if (c64)
        hipLaunchKernelGGL(seed_kernel<float>, g, dim3(256), 0, (hipStream_t)stream, (const LeafDescHead *)heads,
                           nleaves, stride, lowfac, (const float2 *)ga, (float2 *)gn, ga_stride, gn_stride);
    else
        hipLaunchKernelGGL(seed_kernel<double>, g, dim3(256), 0, (hipStream_t)stream, (const LeafDescHead *)heads,
                           nleaves, stride, lowfac, (const double2 *)ga, (double2 *)gn, ga_stride, gn_stride);
    return (int)hipGetLastError();
}

// raise the dynamic-LDS limit of a kernel once per process
template <typename K>
static hipError_t allow_lds(K kernel, bool &done)
{
    if (done) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)SLOS_LDS_DYNAMIC_MAX);
    if (e == hipSuccess) done = true;
    return e;
}

int slos_launch_bwd_layer(const BwdParams &p, int c64, int grid, void *stream, int batch)
{
    static bool a32 = false, a64 = false;
    hipError_t e = c64 ? allow_lds(bwd_layer_kernel<float>, a32) : allow_lds(bwd_layer_kernel<double>, a64);
    if (e != hipSuccess) return (int)e;
    const size_t lds = (size_t)p.jn * 64 * sizeof(double2);
    const dim3 g(grid, batch > 1 ? batch : 1);
    if (c64)
        hipLaunchKernelGGL(bwd_layer_kernel<float>, g, dim3(64), lds, (hipStream_t)stream, p);
    else
        hipLaunchKernelGGL(bwd_layer_kernel<double>, g, dim3(64), lds, (hipStream_t)stream, p);
    return (int)hipGetLastError();
}

int slos_launch_colsum_gradu(const void *partials, const ColsumLayers &L, const int32_t *photons, int n, int m,
                             void *GU, int c64, void *stream, int batch, uint64_t partials_stride, uint64_t gu_stride)
{
    const dim3 g(m, batch > 1 ? batch : 1);
    if (c64)
        hipLaunchKernelGGL(colsum_gradu_kernel<float>, g, dim3(256), 0, (hipStream_t)stream, (const double2 *)partials,
                           L, photons, n, m, (float2 *)GU, partials_stride, gu_stride);
    else
        hipLaunchKernelGGL(colsum_gradu_kernel<double>, g, dim3(256), 0, (hipStream_t)stream,
                           (const double2 *)partials, L, photons, n, m, (double2 *)GU, partials_stride, gu_stride);
    return (int)hipGetLastError();
}

int slos_launch_sq_loss_seed(const void *a, uint64_t M, const int64_t *ranks, const double *scale, int64_t count,
                             const double *p_target, void *gn, uint64_t gn_stride, double *loss, int batch, int c64,
                             void *stream)
{
    const dim3 g((unsigned)((M + SLOS_SEED_SLICE - 1) / SLOS_SEED_SLICE), (unsigned)batch);
    if (c64)
        hipLaunchKernelGGL(sq_loss_seed_kernel<float>, g, dim3(256), 0, (hipStream_t)stream, (const float2 *)a, M,
                           ranks, scale, count, p_target, (float2 *)gn, gn_stride, loss);
    else
        hipLaunchKernelGGL(sq_loss_seed_kernel<double>, g, dim3(256), 0, (hipStream_t)stream, (const double2 *)a, M,
                           ranks, scale, count, p_target, (double2 *)gn, gn_stride, loss);
    return (int)hipGetLastError();
}

int slos_launch_sq_loss(const void *a, uint64_t M, const int64_t *ranks, int64_t count, const double *p_target,
                        void *grad_a, double *loss, int batch, int c64, void *stream)
{
    if (c64)
        hipLaunchKernelGGL(sq_loss_kernel<float>, dim3(batch), dim3(256), 0, (hipStream_t)stream, (const float2 *)a, M,
                           ranks, count, p_target, (float2 *)grad_a, loss);
    else
        hipLaunchKernelGGL(sq_loss_kernel<double>, dim3(batch), dim3(256), 0, (hipStream_t)stream,
                           (const double2 *)a, M, ranks, count, p_target, (double2 *)grad_a, loss);
    return (int)hipGetLastError();
}

int slos_launch_mesh_forward(int m, int batch, const double *phases, void *U, int c64, void *stream)
{
    const int nmzi = m * (m - 1) / 2;
    const size_t mat = (size_t)m * m * sizeof(Cd), fac = 2 * (size_t)nmzi * sizeof(Cd);
    const int stage = mat + fac <= SLOS_LDS_DYNAMIC_MAX;  // phase factors in LDS when they fit
    const size_t lds = mat + (stage ? fac : 0);
    static bool a32 = false, a64 = false;
    hipError_t e = c64 ? allow_lds(mesh_forward_kernel<float>, a32) : allow_lds(mesh_forward_kernel<double>, a64);
    if (e != hipSuccess) return (int)e;
    if (c64)
        hipLaunchKernelGGL(mesh_forward_kernel<float>, dim3(batch), dim3(64), lds, (hipStream_t)stream, m, nmzi,
                           phases, (float2 *)U, stage);
    else
        hipLaunchKernelGGL(mesh_forward_kernel<double>, dim3(batch), dim3(64), lds, (hipStream_t)stream, m, nmzi,
                           phases, (double2 *)U, stage);
    return (int)hipGetLastError();
}

int slos_launch_mesh_backward(int m, int batch, const double *phases, const void *GU, double *gphases, int c64,
                              void *stream)
{
    const int nmzi = m * (m - 1) / 2;
    const size_t mat = 2 * (size_t)m * m * sizeof(Cd), fac = 2 * (size_t)nmzi * sizeof(Cd);
    const int stage = mat + fac <= SLOS_LDS_DYNAMIC_MAX;
    const size_t lds = mat + (stage ? fac : 0);
    static bool a32 = false, a64 = false;
    hipError_t e = c64 ? allow_lds(mesh_backward_kernel<float>, a32) : allow_lds(mesh_backward_kernel<double>, a64);
    if (e != hipSuccess) return (int)e;
    if (c64)
        hipLaunchKernelGGL(mesh_backward_kernel<float>, dim3(batch), dim3(64), lds, (hipStream_t)stream, m, nmzi,
                           phases, (const float2 *)GU, gphases, stage);
    else
        hipLaunchKernelGGL(mesh_backward_kernel<double>, dim3(batch), dim3(64), lds, (hipStream_t)stream, m, nmzi,
                           phases, (const double2 *)GU, gphases, stage);
    return (int)hipGetLastError();
}
