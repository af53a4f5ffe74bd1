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
    uint8_t hm[SLOS_MAX_PHOTONS];      // modes of the high photons, descending
    uint8_t pad1[12];
};
static_assert(sizeof(LeafRec) == 64, "LeafRec must stay 64 bytes");

// Inner table of one (q, K) pair: for each low state x (colex rank within
// F(q, K)) the list of its occupied low modes j with the colex rank of
// x - e_j in F(q, K-1), packed as (j << 24) | rank, padded to cmax entries
// with (SLOS_ZERO_MODE << 24); stored term-major: pred[pred_off + c*size + x].
// lowfac[fac_off + x] = sqrt(prod_j x_j!) in FP64.
struct InnerType {
    uint32_t q;
    uint32_t K;
    uint32_t size;
    uint32_t cmax;
    uint64_t pred_off;
    uint64_t fac_off;
};
static_assert(sizeof(InnerType) == 32, "InnerType must stay 32 bytes");

#define SLOS_ZERO_MODE 255u   // u[255] is held at zero in the kernels
#define SLOS_PRED_MASK 0x00FFFFFFu

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
    double *partials;       // one FP64 partial sum of P per wave (last layer)
};

struct LayerLaunch {
    int c64;          // 1: complex64, 0: complex128
    int mode;         // SlosLayerMode
    int compensated;  // c64 only
    int rr;           // outputs per lane per tile: 1, 2, 4
    int threads;      // workgroup size (multiple of 64, <= 256)
    int grid;         // workgroups
};

// Kernel launchers (layer.hip).  Return a hipError_t value as int.
int slos_launch_layer(const LayerParams &p, const LayerLaunch &l, void *stream);
int slos_launch_reduce(const double *partials, int count, double *out, void *stream);
int slos_launch_vacuum(void *out, int c64, int mode, double *sum_p, void *stream);
