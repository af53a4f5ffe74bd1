// Internal structures shared by the host plan (plan.cpp) and the HIP kernels
// (layer.hip).  Not part of the public ABI.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "slos.h"

// A leaf is a contiguous block of one Fock layer: the occupations of the
// "high" modes q..m-1 are fixed and the remaining K photons range over the q
// low modes.  In colex order such a block is contiguous, its states are
// ordered by the colex rank of their low part (0 .. C(q+K-1, K) - 1), and for
// a high mode j the predecessor block (high part minus e_j, same K) is a block
// of the previous layer with the same inner order.
struct LeafRec {
    uint64_t out_base;                 // rank (in layer k) of the leaf's first state
    uint32_t size;                     // C(q+K-1, K)
    uint32_t tab;                      // index into the inner-type table
    uint8_t q;                         // number of low modes
    uint8_t K;                         // photons in the low modes
    uint8_t nhp;                       // k - K photons in high modes
    uint8_t pad0;
    uint32_t pad1;
    double fac_hi;                     // sqrt(prod over high modes of o_j!) / sqrt(prod t_i!)
    uint8_t hm[SLOS_MAX_PHOTONS];      // modes of the high photons, descending
};
static_assert(sizeof(LeafRec) == 64, "LeafRec must stay 64 bytes");

// What a wave needs to compute one leaf, precomputed on the host so that a
// single coalesced load brings it in.  Group g (< nh) is the g-th occupied
// high mode (descending): its predecessor block starts at rank
// low_base - delta[g] of A_{k-1} and is multiplied by U[mode[g], i_k].
// The narrow form holds 16 groups with 32-bit deltas; the wide form 32 groups
// with 64-bit deltas (layers of 2^32 elements or more, or n > 16).
struct LeafDescHead {
    uint64_t out_base;   // rank of the leaf's first state in A_k
    uint64_t low_base;   // rank of the low block (same high part, K-1 low photons) in A_{k-1}
    double fac_hi;       // sqrt(prod high o_j!) / sqrt(prod t_i!)
    uint32_t size;       // states in the leaf, |F(q, K)|
    uint32_t low_size;   // states in the low block, |F(q, K-1)|
    uint32_t pred_off;   // inner table offset (elements) in the pred pool
    uint32_t fac_off;    // inner factorial offset in the lowfac pool
    uint8_t cmax;        // inner term-list length
    uint8_t nh;          // occupied high modes
    uint8_t q;
    uint8_t K;
    uint32_t pad;
};
static_assert(sizeof(LeafDescHead) == 48, "LeafDescHead must stay 48 bytes");

#define SLOS_NARROW_GROUPS 16
#define SLOS_WIDE_GROUPS 32
struct LeafDescNarrow {
    LeafDescHead h;
    uint32_t delta[SLOS_NARROW_GROUPS];
    uint8_t mode[SLOS_NARROW_GROUPS];
};
static_assert(sizeof(LeafDescNarrow) == 128, "LeafDescNarrow must stay 128 bytes");
struct LeafDescWide {
    LeafDescHead h;
    uint64_t delta[SLOS_WIDE_GROUPS];
    uint8_t mode[SLOS_WIDE_GROUPS];
};
static_assert(sizeof(LeafDescWide) == 336, "LeafDescWide must stay 336 bytes");

// Bytes of readable slack after every layer buffer: the low-block staging
// copies whole 16-byte chunks in 1 KiB wave-wide steps.
#define SLOS_BUFFER_SLACK 2048
// accumulation modes of the c64 layer kernel
#define SLOS_COMP_NONE 0
#define SLOS_COMP_BIASED 1
#define SLOS_COMP_TWOSUM 2
#define SLOS_COMP_F64 3
// per-layer leaf cap: min(leaf_max, max(SLOS_MIN_LEAF, N_k / SLOS_TARGET_LEAVES))
#define SLOS_MIN_LEAF 512
#define SLOS_TARGET_LEAVES 2048u

// Inner table of one (q, K) pair: for each low state x (colex rank within
// F(q, K)) the list of its occupied low modes j with the colex rank of
// x - e_j in F(q, K-1), packed as (j << 24) | rank, padded to cmax entries
// with (SLOS_ZERO_MODE << 24); stored term-major: pred[pred_off + c*size + x].
// lowfac[fac_off + x] = sqrt(prod_j x_j!) in FP64.
struct InnerType {
    uint16_t q;
    uint16_t K;
    uint32_t size;       // |F(q, K)|
    uint32_t cmax;       // longest term list
    uint32_t low_size;   // |F(q, K-1)| (0 when K = 0): the leaf's low block
    uint64_t pred_off;
    uint64_t fac_off;
};
static_assert(sizeof(InnerType) == 32, "InnerType must stay 32 bytes");

#define SLOS_ZERO_MODE 255u   // u[255] is held at zero in the kernels
#define SLOS_PRED_MASK 0x00FFFFFFu

#define SLOS_XCDS 8   // MI355X: 8 accelerator complex dies, workgroups dealt round-robin
#define SLOS_TICKET_STRIDE 64
// u32 index, within a layer's first ticket line, of that layer's recorded max
#define SLOS_VMAX_SLOT 32  // uint32 slots between ticket counters: one per 256-byte line

enum SlosLayerMode {
    SLOS_MODE_MID = 0,    // store A_k
    SLOS_MODE_AMPL = 1,   // last layer: normalise, store a(S), accumulate sum P
    SLOS_MODE_PROB = 2,   // last layer: normalise, store P(S), accumulate sum P
};

struct LayerParams {
    const void *X;          // A_{k-1} (device)
    void *Y;                // A_k, a or P (device)
    const void *U;          // m x m, row = output mode (device)
    const LeafRec *leaves;  // leaves of layer k (device)
    const void *desc;       // LeafDescNarrow or LeafDescWide array of layer k (device)
    uint64_t nleaves;
    const InnerType *types;
    const uint32_t *pred;
    const double *lowfac;
    const uint64_t *binom;  // binom[a * bstride + b] = C(a, b)
    int bstride;
    int m;
    int k;                  // layer index (photons in the output states)
    int col;                // input mode i_k of the photon added at this layer
    double norm_t;          // 1 / sqrt(prod_i t_i!)
    double *partials;       // one FP64 partial sum of P per leaf (last layer)
    uint32_t low_max;       // largest low block of the layer (elements)
    uint32_t lds_wave_bytes;// LDS bytes of one low-block staging slice
    // Leaves are dealt to XCDs in chunks of xcd_chunk consecutive leaves
    // (chunk c to the workgroups with blockIdx.x % SLOS_XCDS == c % SLOS_XCDS,
    // which the dispatcher places on one XCD): each L2 sees contiguous runs of
    // the colex order while all XCDs stay in the same region of the layer.
    uint32_t xcd_chunk;
    // One ticket counter per XCD (zeroed before every forward call): a wave
    // takes the XCD's next leaf in order, so the resident waves of an XCD
    // always work on neighbouring leaves and share the L2.
    uint32_t *tickets;
    uint32_t ticket_leaves;  // consecutive leaves per ticket
    // Compensated layers: max over A_{k-1} of |Re x| + |Im x| as float bits
    // (NULL: the vacuum, 1), and where this layer records the same for A_k
    // (NULL: not recorded).  Both live in the zeroed ticket area.
    const uint32_t *vmax_in;
    uint32_t *vmax_out;
    // Many unitaries through one plan: instance b = blockIdx.y reads X + b *
    // x_stride and U + b * u_stride, writes Y + b * y_stride (bytes), and uses
    // partials + b * partials_stride and tickets (with the vmax slots) +
    // b * ticket_stride.
    uint64_t x_stride, y_stride, u_stride;
    uint64_t partials_stride;
    uint64_t ticket_stride;
};

struct LayerLaunch {
    int c64;          // 1: complex64, 0: complex128
    int mode;         // SlosLayerMode
    int compensated;  // c64 only: SLOS_COMP_NONE / _BIASED / _TWOSUM
    int batch;        // instances (gridDim.y); 0 or 1: one
    int rr;           // outputs per lane per tile: 1, 2, 4
    int threads;      // workgroup size (multiple of 64, <= 256)
    int grid;         // workgroups
    uint32_t low_max; // largest low block of the layer (elements): one LDS slice
    int wide;         // 1: LeafDescWide descriptors
};

// LDS bytes one wave needs to stage a low block of low_max elements of es bytes
static inline uint32_t slos_lds_wave_bytes(uint32_t low_max, uint32_t es)
{
    return low_max ? ((low_max * es + 16u + 1023u) / 1024u) * 1024u : 0u;
}

// Dynamic LDS available to one workgroup of the layer kernel (gfx950: 160 KiB
// per CU, minus the kernel's static U column).
#define SLOS_LDS_DYNAMIC_MAX (160u * 1024u - 8u * 1024u)

// Kernel launchers (layer.hip).  Return a hipError_t value as int.
int slos_launch_layer(const LayerParams &p, const LayerLaunch &l, void *stream);
// stage: SLOS_REDUCE_STAGE doubles of scratch
#define SLOS_REDUCE_STAGE 256
int slos_launch_reduce(const double *partials, int64_t count, double *stage, double *out, void *stream,
                       int batch = 1, int64_t stride = 0);
int slos_launch_vacuum(void *out, int c64, int mode, double *sum_p, void *stream);
int slos_launch_zero_u32(uint32_t *buf, int count, void *stream);

// The static device scratch area (static_scratch.hip): SLOS_STATIC_SCRATCH_BYTES
// per GPU.  slos_static_scratch returns the current device's address of it
// (looked up once per device) and that device's index; a hipError_t as int.
#define SLOS_STATIC_SCRATCH_BYTES ((size_t)32 << 20)
int slos_static_scratch(void **ptr, int *device);

// ---- differentiation ----------------------------------------------------------

// One unit of the reverse layer k: the states y0 .. y0 + chunk - 1 (cut at
// low_size) of the low block of a forward leaf of layer k (same high part h,
// K-1 low photons), which lies at low_base in A_{k-1}; `chunk` is the layer's
// BwdParams::chunk.  The successor of low state y through low mode i < q is the
// forward leaf's state out_base + succ[succ_off + i*low_size + y]; through high
// mode j >= q it is hbase[hbase_off + j - q] + y (the block of high part h + e_j
// in layer k).
struct BwdUnit {
    uint64_t out_base;
    uint64_t low_base;
    uint64_t hbase_off;
    uint32_t low_size;
    uint32_t succ_off;
    uint32_t q;
    uint32_t y0;
};
static_assert(sizeof(BwdUnit) == 40, "BwdUnit must stay 40 bytes");

struct BwdParams {
    const void *gk;          // g_k (layer k), plan dtype
    void *gkm1;              // g_{k-1}
    const void *Akm1;        // kept A_{k-1}
    const void *U;           // m x m
    const BwdUnit *units;
    uint64_t nunits;
    const uint32_t *succ;
    const uint64_t *hbase;
    void *partials;          // double2 [nunits][m]
    int m;
    int col;                 // i_k
    uint32_t chunk;          // low states per unit (a multiple of 64)
    // Gradient partials of modes [jb, jb + jn) (jn <= SLOS_BWD_MODE_BLOCK); the
    // pass with write_g = 1 also forms g_{k-1} over every mode
    int jb, jn, write_g;
    // instance b = blockIdx.y: byte offsets b * stride of gk, gkm1, Akm1, U, partials
    uint64_t gk_stride, gkm1_stride, a_stride, u_stride, partials_stride;
};

#define SLOS_BWD_MODE_BLOCK 64  // modes whose 64 lanes' FP64 gradient partials one reverse pass keeps in LDS
#define SLOS_MESH_MAX_MODES 64  // the mesh kernels keep two m x m FP64 matrices in LDS

int slos_launch_seed(const void *heads, uint64_t nleaves, uint32_t stride, const double *lowfac, const void *ga,
                     void *gn, int c64, void *stream, int batch = 1, uint64_t ga_stride = 0, uint64_t gn_stride = 0);
int slos_launch_bwd_layer(const BwdParams &p, int c64, int grid, void *stream, int batch = 1);
// Per-layer partial-sum blocks of the reverse pass for the fused column sum:
// layer k + 1's partials start at off[k] (double2 elements) and hold nunits[k]
// rows of m values.
struct ColsumLayers {
    uint64_t off[SLOS_MAX_PHOTONS];
    uint64_t nunits[SLOS_MAX_PHOTONS];
};
int slos_launch_colsum_gradu(const void *partials, const ColsumLayers &L, const int32_t *photons, int n, int m,
                             void *GU, int c64, void *stream, int batch, uint64_t partials_stride, uint64_t gu_stride);
int slos_launch_sq_loss(const void *a, uint64_t M, const int64_t *ranks, int64_t count, const double *p_target,
                        void *grad_a, double *loss, int batch, int c64, void *stream);
int slos_launch_sq_loss_seed(const void *a, uint64_t M, const int64_t *ranks, const double *scale, int64_t count,
                             const double *p_target, void *gn, uint64_t gn_stride, double *loss, int batch, int c64,
                             void *stream);
int slos_launch_mesh_forward(int m, int batch, const double *phases, void *U, int c64, void *stream);
int slos_launch_mesh_backward(int m, int batch, const double *phases, const void *GU, double *gphases, int c64,
                              void *stream);

// ---- batches of independent instances -------------------------------------------

#define SLOS_BATCH_MAX_N 16

// One instance of a batch.  Layer k (1..n) has nleaves[k-1] narrow leaf
// descriptors starting at record desc_off[k-1]; its photon comes from input
// mode col[k-1].  U and the outputs live in packed arrays at U_off / out_off
// (elements).
struct BatchInst {
    uint64_t U_off;
    uint64_t out_off;
    uint32_t m;
    uint32_t n;
    uint32_t desc_off[SLOS_BATCH_MAX_N];
    uint32_t nleaves[SLOS_BATCH_MAX_N];
    uint8_t col[SLOS_BATCH_MAX_N];
};

// Two kinds of work per workgroup: instances large enough to occupy all its
// waves run cooperatively (all waves, a barrier between layers), first; then
// each wave runs its own list of small instances alone (wave-level ordering
// between layers), so no wave idles at a barrier on a one-leaf layer.
struct BatchParams {
    const void *U;              // packed U matrices
    void *out;                  // packed amplitudes
    double *sum_p;              // per instance, or NULL
    const BatchInst *inst;
    const uint32_t *wg_start;   // workgroup g runs wg_list[wg_start[g] .. wg_start[g+1]) cooperatively
    const uint32_t *wg_list;
    const uint32_t *wv_start;   // then wave w of g runs wv_list[wv_start[s] .. wv_start[s+1]), s = g W + w
    const uint32_t *wv_list;
    const LeafDescNarrow *desc;
    const uint32_t *pred;
    const double *lowfac;
    void *scratch;              // layer buffers (elements of the plan's type)
    const uint64_t *wg_scr;     // per workgroup: its cooperative pair of scratch_stride buffers
    uint64_t scratch_stride;    // elements per cooperative buffer, slack included
    uint64_t small_base;        // wave slot s: pair of small_stride buffers at small_base + 2 s small_stride
    uint64_t small_stride;
    const void *vac;            // A_0 = [1]
    uint32_t lds_wave_bytes;    // low-block slice per wave; a 256-entry U column per wave follows the slices
};

int slos_launch_batch(const BatchParams &p, int c64, int rr, int threads, int grid, void *stream);
int slos_prepare_batch_kernels(void);
