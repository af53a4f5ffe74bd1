// Internal structures of the kernels beside the layer recurrence: weak
// simulation, post-selection, selected outputs and imperfect-source mixtures
// (sample.hip, postselect.hip, select.hip, source.hip) and the host code that
// launches them (plan.cpp).  Not part of the public ABI.
#pragma once

#include "slos_internal.h"

// states per block of the cumulative-probability table (multiple of 64)
#define SLOS_CDF_BLOCK 1024

// weak simulation (sample.hip)
// A 16-ary search tree over the block prefix bp (level 0, nb entries): level l
// holds bp[i * 16^l] for i < n[l] = ceil(nb / 16^l), up to the first level of
// at most 16 entries, so that every step of a search reads 16 consecutive
// values (one 128-byte line).  Levels 1.. are stored one after another at
// tree + off[l].
#define SLOS_CDF_TREE_MAX_LEVELS 12
struct CdfTree {
    int nlev;
    int64_t n[SLOS_CDF_TREE_MAX_LEVELS];
    int64_t off[SLOS_CDF_TREE_MAX_LEVELS];
    int64_t total;  // doubles in levels 1..nlev-1
};
inline CdfTree cdf_tree_layout(int64_t nb)
{
    CdfTree t{};
    t.n[0] = nb;
    t.nlev = 1;
    while (t.n[t.nlev - 1] > 16 && t.nlev < SLOS_CDF_TREE_MAX_LEVELS) {
        t.n[t.nlev] = (t.n[t.nlev - 1] + 15) / 16;
        t.off[t.nlev] = t.total;
        t.total += t.n[t.nlev];
        ++t.nlev;
    }
    return t;
}
int slos_launch_cdf(const void *P, int c64, int64_t M, double *bp, void *stream);
int slos_launch_marginals(const void *P, int c64, const double *bp, const int64_t *ends, int m, double *pk,
                          void *stream);
int slos_launch_sample(const void *P, int c64, int64_t M, const double *bp, const double *r, int64_t count,
                       int64_t *ranks, void *stream);

// post-selection (postselect.hip)
#define SLOS_PS_MAX_GROUPS 16
#define SLOS_PS_MAX_WAVES 8192  // partial sums per post-selection launch
#define SLOS_PS_LEAF_MAX 32768   // states per post-selection leaf
// an inner shape (q low modes, K low photons) of the post-selection leaves:
// its low states occupy table entries [off, off + size)
struct PsType {
    uint32_t off;
    uint32_t size;
    uint16_t q, K;
    uint32_t pad;
};
struct PostselectParams {
    const void *P;          // M probabilities (fp32 or fp64), colex order
    void *masked;           // P masked to the kept outputs, or NULL
    int64_t M;
    const uint64_t *binom;  // binom[a * bstride + b] = C(a, b)
    int bstride;
    int m, n, ngroups;
    uint64_t run;           // consecutive ranks per thread
    double *partials;       // one FP64 partial per wave
    int8_t group[256];      // group of each mode, -1: unconstrained
    uint8_t cmin[SLOS_PS_MAX_GROUPS], cmax[SLOS_PS_MAX_GROUPS];
    // leaf path: a leaf decomposition of the last layer of its own (leaves of
    // up to SLOS_PS_LEAF_MAX states), and per inner shape used by them a run of
    // the low-state table (SLOS_PS_MAX_GROUPS group counts per state)
    const LeafRec *leaves;
    uint64_t nleaves;
    const uint32_t *type_off;    // per inner-shape index: first table entry
    const PsType *types;         // ntypes entries, ascending off
    uint32_t ntypes;             // inner shapes of the leaves
    uint32_t entries;            // table entries (low states)
    uint8_t *low;                // entries x SLOS_PS_MAX_GROUPS group counts
};
int slos_launch_postselect(const PostselectParams &p, int c64, void *stream);
int slos_launch_postselect_table(const PostselectParams &p, int c64, const int64_t *ranks, int64_t nranks,
                                 const double *sum, double *table, void *stream);

// selected outputs (select.hip)
#define SLOS_SELECT_MAX_OCC 32
// A target's sub-lattice {t <= S} depends only on the multiset of its
// occupations once the occupied modes are put in a canonical order
// (occupation descending, then mode), so targets share one table per multiset:
// the states numbered in mixed radix over the digits (radix s_q + 1), listed by
// layer |t|, each with the mask of its non-zero digits.
struct SelectPattern {
    uint32_t R;                          // prod over digits of (s_q + 1)
    uint32_t nocc;                       // digits
    uint32_t off;                        // its states in the state and mask pools
    uint32_t lstart[SLOS_MAX_PHOTONS + 2];  // layer k: pool positions [off + lstart[k], off + lstart[k+1])
    uint32_t stride[SLOS_SELECT_MAX_OCC];   // t - e_q = index - stride[q]
};
struct SelectTarget {
    uint32_t pattern;                    // its sub-lattice table
    uint32_t nocc;                       // occupied modes of the target
    double fac;                          // sqrt(prod s_j!) / sqrt(prod t_i!)
    uint8_t mode[SLOS_SELECT_MAX_OCC];   // occupied modes in the pattern's digit order
};
struct SelectParams {
    const void *U;                // m x m, plan dtype
    const SelectTarget *targets;  // device
    const SelectPattern *patterns;  // device
    const uint16_t *state;        // per pattern, its states by layer (mixed-radix index)
    const uint32_t *mask;         // the non-zero digits of each listed state
    int64_t count;
    void *out;                    // count amplitudes, plan dtype
    uint32_t r_max;               // largest R of the call (LDS sizing)
    int m, n;
    uint8_t cols[SLOS_MAX_PHOTONS];  // i_k, k = 1..n
};
int slos_launch_select(const SelectParams &p, int c64, void *stream);

// imperfect-source mixtures (source.hip)
#define SLOS_SRC_MAX_SOURCES 12   // 2^12 emission subsets
#define SLOS_SRC_MAX_NMAX 16      // photon numbers kept: 0..nmax
#define SLOS_SRC_STATS_MAX_BLOCKS 16384  // statistics blocks: chunks of at least 1024 states
// Common-wavepacket groups, all subsets of the sources: the amplitude vector
// (monomial coefficients of the recurrence, no normalisation) of subset A is
// that of A minus its highest source advanced by one layer of the recurrence
// with that source's input mode: one launch per subset size a, blockIdx.y over
// the subsets of size a.  Vectors are compact (C(m+a-1, a) complex128 each, at
// amp_off[A]); the empty subset holds [1], written once at plan time.
struct SrcGroupParams {
    double2 *amp;
    const int64_t *amp_off;         // per subset mask
    const uint32_t *subsets;        // masks of this launch's size
    const LeafDescNarrow *desc;     // leaves of photon number a: [leaf_lo, leaf_hi)
    uint64_t leaf_lo, leaf_hi;
    uint64_t off_out, off_in;       // graded offsets of photon numbers a and a - 1
    const uint32_t *pred;
    const void *U;                  // complex128 m x m
    int m;
    uint8_t modes[SLOS_SRC_MAX_SOURCES];  // input mode of each source
};
// Common-group probabilities into the slots: slot s (bit b = source b in the
// common wavepacket) receives P = |A_s|^2 prod_j s_j! / prod_i t_i! on the
// states of popcount(s) photons, its whole support (prod s_j! from the leaf's
// high-mode factor and the inner table's low factors); the rest of the slot is
// never read.
struct SrcFillParams {
    double *slots;          // nslots x G
    uint64_t G;
    const double2 *amp;
    const int64_t *amp_off; // per slot: amplitude vector, or -1 (group above nmax)
    const double *inv_tfac; // per slot: 1 / prod_i t_i! of its group
    const LeafDescNarrow *desc;
    const double *lowfac;
    uint64_t leaves_upto[SLOS_SRC_MAX_NMAX + 1];  // leaves of photon numbers 1..k
    uint64_t off[SLOS_SRC_MAX_NMAX + 2];
    int nmax;
};
// y = gamma * L(in) + alpha * a + beta * b on graded vectors, one launch for
// all pairs r = blockIdx.y of a butterfly step.  (L in)[t] = sum over the
// occupied modes j of t of |U[j, col]|^2 in[t - e_j]: one distinguishable
// photon entering mode col.  y may alias a or b (same element only), never in.
// Supports: with c = popcount(r), operand X holds photon numbers
// [c + X_lo, c + X_lo + X_len] and is read only there; y is written on
// [c, c + y_len] (all clipped to [0, nmax]) and nowhere else.  Leaf records
// carry their photon number in h.pad.
struct SrcPassParams {
    const double *in;
    const double *a;
    const double *b;
    double *y;
    uint64_t s_in, s_a, s_b, s_y;   // elements between consecutive pairs
    double gamma, alpha, beta;
    const LeafDescNarrow *desc;     // leaves of photon numbers 1..nmax, graded ranks
    uint64_t nleaves;               // leaves this launch scans (a prefix: photon numbers 1..kmax)
    const uint32_t *pred;
    const void *U;                  // complex128 m x m
    int m, col, nmax;
    int in_lo, in_len, a_lo, a_len, b_lo, b_len, y_len;
};
struct SrcStatsParams {
    const double *P;
    const uint64_t *off;
    const uint64_t *binom;          // binom[a * bstride + b] = C(a, b)
    int bstride;
    int m, nmax, ngroups, min_modes;
    int8_t group[256];
    uint8_t cmin[SLOS_PS_MAX_GROUPS], cmax[SLOS_PS_MAX_GROUPS];
    uint64_t chunk;                               // states per block
    uint32_t blk_off[SLOS_SRC_MAX_NMAX + 2];      // first block of each photon number
    double *partials;               // blk_off[nmax + 1] x 3
    double *result;                 // [nmax + 1][3]: mass, physical, kept
};
int slos_launch_src_group(const SrcGroupParams &p, int nsub, void *stream);
int slos_launch_src_fill(const SrcFillParams &p, int nslots, void *stream);
int slos_launch_src_pass(const SrcPassParams &p, int npairs, void *stream);
int slos_launch_src_stats(const SrcStatsParams &p, void *stream);
