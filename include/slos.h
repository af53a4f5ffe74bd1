/*
 * slos.h -- C ABI of the MI355X SLOS strong-simulation library.
 *
 * The library computes, for an m-mode linear interferometer U and an n-photon
 * input Fock state T, the amplitude a(S) of every n-photon output Fock state S
 * (arXiv 2204.00602, Section 4.2.1, Eq. eqperm):
 *
 *     a(S) = Perm(U_{T,S}) / sqrt(s_1!..s_m! t_1!..t_m!),   P(S) = |a(S)|^2,
 *
 * by the layered photon-addition recurrence of the SLOS back-end (Section
 * 3.2.3, "SLOS" paragraph: the whole computation path is unfolded in memory,
 * time O(n C(m+n-1, n))).  With the photons of T listed as modes
 * i_1 <= ... <= i_n, A_0 = [1] and, for k = 1..n and every k-photon state t,
 *
 *     A_k[t] = sum_{j : t_j > 0} U[j, i_k] * A_{k-1}[t - e_j],
 *
 * then a(S) = A_n[S] * sqrt(prod_j s_j!) / sqrt(prod_i t_i!).
 *
 * Conventions shared by every entry point
 *   - U is row-major m x m, U[j*m + i] = amplitude from input mode i to output
 *     mode j (row = output mode), in the plan's complex type, interleaved
 *     (re, im).  U is not required to be unitary.
 *   - Output order: colex rank.  For a k-photon state with photon modes
 *     d_1 <= ... <= d_k, rank = sum_{r=1..k} C(d_r + r - 1, r); rank 0 holds all
 *     photons in mode 0.  slos_fock_rank / slos_fock_unrank convert.
 *   - Device pointers are HIP device allocations owned by the caller; the
 *     library never frees them.  `stream` is a hipStream_t (NULL = the null
 *     stream); calls that take one are asynchronous on it.
 *   - Every function returns SLOS_OK (0) or a negative SLOS_ERR_* code and
 *     never aborts; slos_last_error() describes the last failure on the
 *     calling thread.
 *   - A plan holds scratch memory: use it from one stream at a time.
 */
#ifndef SLOS_H
#define SLOS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define SLOS_OK 0
#define SLOS_ERR_INVALID_ARG (-1)   /* bad m, n, state, pointer or option        */
#define SLOS_ERR_SIZE_OVERFLOW (-2) /* C(m+n-1, n) or a buffer size overflows     */
#define SLOS_ERR_OOM (-3)           /* a device or host allocation failed         */
#define SLOS_ERR_DTYPE (-4)         /* call does not match the plan's dtype/flags */
#define SLOS_ERR_HIP (-5)           /* a HIP runtime call or launch failed        */
#define SLOS_ERR_NOT_KEPT (-6)      /* backward needs a plan with SLOS_KEEP_LAYERS */
#define SLOS_ERR_NO_DEVICE (-7)     /* no usable HIP device                       */

/* ---- plan flags ---------------------------------------------------------- */
#define SLOS_C64 0x1          /* complex64 recurrence, fp32 probabilities          */
#define SLOS_C128 0x2         /* complex128 recurrence, fp64 probabilities         */
#define SLOS_COMPENSATED 0x100 /* c64 only: compensated accumulation on layers
                                  k >= comp_from_layer.  Each FMA's rounding error
                                  is recovered exactly (the two-sum of the running
                                  sum and the product, made exact by starting the
                                  sum at a power-of-two bias >= 4 sum|products|,
                                  from the previous layer's recorded maximum) and
                                  summed in a second float; 4 flops per real
                                  product                                          */
#define SLOS_COMP_KNUTH 0x800  /* with SLOS_COMPENSATED: FMA two-product plus
                                  Knuth's branch-free two-sum instead (10 flops per
                                  real product; same error order)                  */
#define SLOS_COMP_FP64 0x1000  /* with SLOS_COMPENSATED: widen each term's factors
                                  to FP64 (their product is then exact) and sum
                                  with FP64 FMAs (4 FMAs and 2 conversions per
                                  complex term; one FP64 rounding per real
                                  product)                                         */
#define SLOS_KEEP_LAYERS 0x200 /* keep A_0..A_{n-1} on the device (for backward)   */
#define SLOS_HOST_ONLY 0x400   /* build the host tables only; no device memory;
                                  for slos_plan_info / slos_plan_leaf inspection  */

#define SLOS_MAX_MODES 255
#define SLOS_MAX_PHOTONS 32

typedef struct slos_plan_s *slos_plan_t;

/* Tuning options; a zero field takes its default. */
typedef struct slos_options {
    int32_t leaf_max;        /* max states per leaf tile, <= 65536 (default 16384 for
                                c64, 8192 for c128, 4096 with SLOS_KEEP_LAYERS); a
                                small layer uses smaller leaves so that it still
                                spreads over ~2048 workgroups                        */
    int32_t comp_from_layer; /* first compensated layer (default 1: every layer)     */
    int32_t block_threads;   /* threads per workgroup: 64, 128, 256 (default 256;
                                128 with SLOS_KEEP_LAYERS)                           */
    int32_t grid_blocks;     /* cap on workgroups per layer launch (default 2048)    */
    int32_t outputs_per_lane;/* 1, 2 or 4 outputs per lane per tile (default 2)       */
    int32_t xcd_chunk;       /* consecutive leaves dealt to one XCD at a time
                                (default 128; fewer when a layer has few leaves)    */
    int32_t ticket_leaves;   /* consecutive leaves a workgroup takes per work ticket
                                (default 1 for c64, 2 for c128)                      */
    int32_t max_batch;       /* unitaries per *_many call, 1..65535 (default 1): the
                                plan holds layer buffers for that many instances   */
    int32_t wide_descriptors;/* 1: use the 32-group, 64-bit-delta leaf descriptors on
                                every layer; 0 (default): only where a leaf needs
                                them (more than 16 occupied high modes, or a layer
                                of 2^32 states or more)                             */
    int32_t leaf_order;      /* order in which a layer's leaves are processed:
                                d = 1..4 groups the leaves whose high parts agree
                                once their d highest photons are removed (they
                                share predecessor blocks, which then stay in cache
                                while the group runs); 0: d = 1 (default); -1:
                                colex order                                      */
    int32_t low_block_max;   /* largest low block a leaf may stage in LDS (states);
                                leaves with larger ones are split further, so a
                                workgroup needs less LDS and more of them fit on
                                a CU.  0: default (3072 for c64, 24 KiB; 2560 for
                                c128, 40 KiB; no limit with SLOS_KEEP_LAYERS or
                                for batches); -1: none                           */
} slos_options_t;

/* ---- Fock-space arithmetic (host only; no device needed) ------------------ */

/* |S_{m,n}| = C(m+n-1, n) (Section 4.2.2).  SIZE_OVERFLOW if > INT64_MAX. */
int slos_fock_count(int m, int n, int64_t *count);

/* Colex rank of `state` (m int32 occupations summing to n). */
int slos_fock_rank(int m, int n, const int32_t *state, int64_t *rank);

/* Inverse of slos_fock_rank: writes m int32 occupations to `state`. */
int slos_fock_unrank(int m, int n, int64_t rank, int32_t *state);

/* ---- plans ---------------------------------------------------------------- */

/*
 * Build a plan for m modes (1..255) and the input Fock state `input_state`
 * (m int32 occupations, all >= 0, summing to n <= 32).  `flags` holds exactly
 * one of SLOS_C64 / SLOS_C128 plus optional SLOS_COMPENSATED (C64 only; with
 * SLOS_COMP_KNUTH), SLOS_KEEP_LAYERS, SLOS_HOST_ONLY.  Checks that C(m+n-1, n) and all buffers
 * fit, builds the photon list i_1 <= .. <= i_n (Section 2: photons are
 * creation operators, so their order does not change the result), the
 * binomial table, the leaf decomposition of every layer and the inner tables,
 * and allocates the layer buffers on the current HIP device.  The plan owns all
 * of this; release it with slos_plan_destroy.  `opts` may be NULL.
 */
int slos_plan(int m, int n, const int32_t *input_state, int flags, slos_plan_t *out);
int slos_plan_ex(int m, int n, const int32_t *input_state, int flags,
                 const slos_options_t *opts, slos_plan_t *out);

/* Frees everything the plan owns.  NULL is a no-op.  Synchronises the device. */
void slos_plan_destroy(slos_plan_t plan);

/* Number of outputs M = C(m+n-1, n); -1 for a NULL plan. */
int64_t slos_num_outputs(slos_plan_t plan);

/* Colex rank of an output state of the plan (m int32 occupations summing to
 * the plan's n): the index of a(state) in the arrays slos_amplitudes and
 * slos_probs write (Section 4.2.1 defines the output set S_{m,n}; the order is
 * colex, rank 0 holding every photon in mode 0).  INVALID_ARG for a NULL
 * pointer or a state of the wrong photon number.  Host only, no device work. */
int slos_rank(slos_plan_t plan, const int32_t *state, int64_t *rank);

/* Inverse of slos_rank: writes the plan's m occupations of output `rank`
 * (0 <= rank < slos_num_outputs) to `state`, which the caller owns. */
int slos_unrank(slos_plan_t plan, int64_t rank, int32_t *state);

/* Host-side inspection of the tiling of layer k (1..n): number of states N_k
 * and number of leaves.  Works on SLOS_HOST_ONLY plans. */
int slos_plan_info(slos_plan_t plan, int k, int64_t *n_states, int64_t *n_leaves);

/* Leaf `idx` of layer k: rank of its first state, low-mode count q, low photon
 * count K, and its k-K high photons' modes (descending) in high_modes[0..k-K). */
int slos_plan_leaf(slos_plan_t plan, int k, int64_t idx, int64_t *out_base,
                   int32_t *q, int32_t *K, int32_t *high_modes);

/* ---- forward -------------------------------------------------------------- */

/*
 * All M amplitudes: out[rank(S)] = a(S), M complex values in the plan's type
 * (device).  U: device, see conventions.  If sum_p (device, one double) is not
 * NULL it receives sum_S |a(S)|^2 accumulated in FP64 (Section 4.2.1: the P(S)
 * form a distribution, so this is 1 for unitary U).
 */
int slos_amplitudes(slos_plan_t plan, const void *U, void *out, double *sum_p, void *stream);

/*
 * All M probabilities P(S) = |a(S)|^2 (Eq. eqperm): probs[rank(S)], fp32 for a
 * C64 plan and fp64 for C128 (device).  sum_p as in slos_amplitudes.
 */
int slos_probs(slos_plan_t plan, const void *U, void *probs, double *sum_p, void *stream);

/*
 * slos_amplitudes for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, results bit for bit those of slos_amplitudes, and no
 * hipMalloc, hipFree or other allocating call: the pass's scratch (vacuum,
 * the two intermediate layers, the FP64 partial sums and the work counters)
 * lives in the library's static device area of 32 MiB per GPU, held from the
 * first call on a GPU until the process ends, instead of in the plan's own
 * buffers.  Plans whose scratch exceeds 32 MiB (about 4M complex64 states in
 * the two largest intermediate layers together, e.g. m = 16, n = 8 fits and
 * m = 20, n = 10 does not) are rejected with SLOS_ERR_SIZE_OVERFLOW, and plans
 * built with SLOS_KEEP_LAYERS with SLOS_ERR_INVALID_ARG; the plan's device must
 * be current.  Every call on one GPU shares that one area: calls that overlap
 * in time on a GPU (on different streams, or from different threads) race and
 * must be ordered by the caller.  Each call starts from what it writes itself,
 * not from what an earlier call left.
 */
int slos_amplitudes_noalloc(slos_plan_t plan, const void *U, void *out, double *sum_p, void *stream);

/*
 * The same input state through `batch` unitaries in one pass (one launch per
 * layer; instance b is blockIdx.y).  U: device, batch x m x m (instance b at
 * U + b*m*m); out / probs: device, batch x M (instance b at b*M); sum_p:
 * device, batch doubles, or NULL.  1 <= batch <= the plan's max_batch option.
 * Instance b's result equals slos_amplitudes / slos_probs on U_b.
 */
int slos_amplitudes_many(slos_plan_t plan, int batch, const void *U, void *out, double *sum_p, void *stream);
int slos_probs_many(slos_plan_t plan, int batch, const void *U, void *probs, double *sum_p, void *stream);

/*
 * Record one forward pass (slos_amplitudes_many, or slos_probs_many when
 * `probs` is non-zero, over `batch` instances) for these buffers into a HIP
 * graph owned by the plan, replacing an earlier one; slos_plan_replay launches
 * it on a stream.  Nothing runs at capture time.  The buffers stay bound to the
 * graph and must outlive it (until the next capture or slos_plan_destroy).  The
 * graph holds kernel nodes only (the ticket counters are cleared by a kernel).
 * Small plans are bound by launch latency: one graph launch replaces the n
 * layer launches and the sum.  SLOS_ERR_INVALID_ARG while timing is on.
 */
int slos_plan_capture(slos_plan_t plan, int batch, int probs, const void *U, void *out, double *sum_p);
int slos_plan_replay(slos_plan_t plan, void *stream);

/* ---- weak simulation from the strong one ------------------------------------ */

/*
 * Cumulative probability table of `probs` (device, 16-byte aligned, M values in
 * colex order: fp32 for a C64 plan, fp64 for C128, e.g. the output of
 * slos_probs; need not be normalised).  FP64 sums of blocks of 1024 states and
 * their exclusive prefix, plus the sums of each block's 16 chunks of 64 states
 * (about 3% of P in FP64 for complex64 plans) and a 16-ary search tree over the
 * block prefix (every 16^l-th prefix, levels down to 16 entries), kept by the
 * plan (one table per plan; a later call replaces it).  Deterministic.
 * slos_marginals and slos_sample read this table together with the same
 * `probs`.
 */
int slos_cdf(slos_plan_t plan, const void *probs, void *stream);

/*
 * Partial certificates (Section 4.2.2, Eq. eqpk): pk[K-1] = P(K), the total
 * probability that modes K..m-1 (0-based) are empty, for K = 1..m, in FP64
 * (device, m doubles).  In colex order those states are the first C(K+n-1, n),
 * so P(K) is a prefix sum.  Needs slos_cdf on the same `probs` first.
 */
int slos_marginals(slos_plan_t plan, const void *probs, double *pk, void *stream);

/*
 * Sampling (the sampler built on a strong back-end, Section 3.2): for each of
 * `count` uniforms r[i] in [0, 1) (device FP64, supplied by the caller),
 * ranks[i] (device int64) = colex rank of the first output whose cumulative
 * probability exceeds r[i] * sum P.  States of zero probability are never
 * returned.  Needs slos_cdf on the same `probs` first.
 */
int slos_sample(slos_plan_t plan, const void *probs, const double *r, int64_t count, int64_t *ranks,
                void *stream);

/* ---- selected outputs ------------------------------------------------------------ */

/*
 * Amplitudes a(S) of `count` chosen outputs only (targets: host, count x m
 * int32 occupations, each summing to n), without the full distribution: for
 * each target the recurrence of Section 3.2.3 runs over the states t <= S
 * alone, prod_j (s_j + 1) of them (2^n without bunching).  One workgroup per
 * target holds that sub-lattice's amplitudes in LDS, so prod_j (s_j + 1) must
 * stay within 19,456 states (c64) or 9,728 (c128); larger targets are
 * rejected.  Targets with the same multiset of occupations share one
 * layer-sorted table of their sub-lattice, built per call.  U: device
 * m x m (plan dtype); out: device, count amplitudes (plan dtype), out[i] =
 * a(target i).  Synchronises the stream before returning (the target
 * descriptors are uploaded from host memory).
 */
int slos_select(slos_plan_t plan, const void *U, const int32_t *targets, int64_t count, void *out, void *stream);

/* ---- post-selection ------------------------------------------------------------ */

/*
 * Heralds and post-selection (Section 3.2.7, the CNOT analysis; Processor
 * appendix) as a conjunction over groups of modes: output S is kept iff for
 * every group g, count_min[g] <= sum of s_j over the modes j with
 * group_of_mode[j] == g <= count_max[g].  group_of_mode: host, m ints, -1 for
 * an unconstrained mode (NULL: no constraint); count_min/count_max: host,
 * ngroups ints each, 0 <= min <= max <= 255; ngroups <= 16.
 * probs: device, M values (fp32 for C64, fp64 for C128), colex order.
 * kept_sum (device, 1 double) = sum of P over the kept outputs (the
 * performance of a post-selected gate), summed in FP64 in a fixed order.
 * masked (device, M values, or NULL) receives P with the dropped outputs set
 * to 0 (e.g. for slos_cdf / slos_sample over the post-selected distribution).
 * ranks (device int64, nranks) / table (device FP64, nranks): table[i] =
 * P(ranks[i]) / kept_sum when output ranks[i] is kept, else 0: the rows of
 * the Analyzer's conditional table.
 */
int slos_postselect(slos_plan_t plan, const void *probs, const int32_t *group_of_mode, int ngroups,
                    const int32_t *count_min, const int32_t *count_max, double *kept_sum, void *masked,
                    const int64_t *ranks, int64_t nranks, double *table, void *stream);

/* ---- differentiation ---------------------------------------------------------- */

/*
 * Reverse pass of the recurrence (adjoint of every layer, then of the
 * normalisation).  grad_a: device, M complex in the plan's type: the gradient
 * of a real loss L with respect to the amplitudes in the PyTorch convention
 * (dL/dRe a + i dL/dIm a).  grad_U: device, m x m complex, overwritten with the
 * gradient with respect to U in the same convention.  Uses the layers
 * A_0..A_{n-1} kept by the last slos_amplitudes / slos_probs call on this plan,
 * which must have used the same U.  Needs SLOS_KEEP_LAYERS (else
 * SLOS_ERR_NOT_KEPT); any m the plan takes (the gradient partials of each
 * reverse layer are formed 64 modes per pass).  Deterministic: no atomics.
 */
int slos_backward(slos_plan_t plan, const void *U, const void *grad_a, void *grad_U, void *stream);

/* slos_backward for the `batch` instances of the last slos_amplitudes_many /
 * slos_probs_many call: grad_a batch x M, grad_U batch x m x m. */
int slos_backward_many(slos_plan_t plan, int batch, const void *U, const void *grad_a, void *grad_U, void *stream);

/*
 * The squared-error loss on selected outputs and its gradient with respect to
 * the amplitudes, for `batch` instances of this plan's output set (the loss of
 * the differentiation workload; Section 4.6 trains on squared residuals of
 * output probabilities).  a: device, batch x M amplitudes in the plan's type
 * (instance b at b * M); ranks: device, `count` distinct output ranks (colex,
 * see slos_rank); p_target: device FP64, batch x count; grad_a: device, batch x
 * M, written in full: 4 (|a_b(S)|^2 - p_target[b, t]) a_b(S) at S = ranks[t]
 * and 0 elsewhere, the PyTorch-convention gradient of
 * L_b = sum_t (|a_b(ranks[t])|^2 - p_target[b, t])^2 that slos_backward_many
 * takes; loss: device FP64, batch values L_b summed in a fixed order, or NULL.
 * One launch, no allocation.  Ranks outside [0, M) are ignored.  The caller
 * owns every buffer; grad_a must not alias a.
 */
int slos_sq_loss_grad_many(slos_plan_t plan, int batch, const void *a, const int64_t *ranks, int64_t count,
                           const double *p_target, void *grad_a, double *loss, void *stream);

/*
 * Normalisation factors of chosen outputs: scales[t] = c_S for S = ranks[t],
 * where a(S) = c_S A_n[S] with c_S = sqrt(prod_j s_j!) / sqrt(prod_i t_i!)
 * (Eq. eqperm's normalisation of the permanent), the same double the adjoint's
 * seed applies.  ranks, scales: host arrays of `count` entries; a rank outside
 * [0, M) gets 0.  Host arithmetic only (host-only plans are accepted).
 */
int slos_output_scales(slos_plan_t plan, const int64_t *ranks, int64_t count, double *scales);

/*
 * slos_sq_loss_grad_many followed by slos_backward_many without the dense
 * dL/da in between: the loss kernel writes the adjoint's seed
 * g_n = c_S * 4 (|a_b(S)|^2 - p_target[b, t]) a_b(S) at S = ranks[t] (0
 * elsewhere) straight into the plan's last-layer gradient buffer, then the
 * reverse layers run as in slos_backward_many.  grad_U and loss come out
 * bit-identical to the two calls.  scales: device FP64, `count` values from
 * slos_output_scales for the same ranks (computed once for a fixed target
 * set).  a, ranks, p_target, grad_U, loss: as in the two calls.  Needs
 * SLOS_KEEP_LAYERS, batch <= max_batch and n >= 1 (the vacuum has no adjoint
 * layers: SLOS_ERR_INVALID_ARG).  Launches only, no allocation.
 */
int slos_sq_loss_backward_many(slos_plan_t plan, int batch, const void *U, const void *a, const int64_t *ranks,
                               const double *scales, int64_t count, const double *p_target, void *grad_U,
                               double *loss, void *stream);

/*
 * Rectangular MZI mesh (Section 2: any unitary decomposes into beam splitters
 * and phase shifters in a square array).  MZI k = PS_1(phi_b) BS PS_0(phi_a) BS
 * with BS of Eq. eq:bs at theta = pi/2 (the composition BS, PS(phi_a) on mode 0,
 * BS, PS(phi_b) on mode 1).  Column c = 0..m-1 holds MZIs on modes (p, p+1),
 * p = c mod 2, c mod 2 + 2, ..., p + 1 < m, taken in that order; U = T_last ...
 * T_first.  phases: device FP64, batch x 2K with K = m(m-1)/2, (phi_a, phi_b)
 * per MZI.  U: device, batch x m x m complex (dtype SLOS_C64 or SLOS_C128).
 * 2 <= m <= 64.  Computed in FP64.
 */
int slos_mesh_unitary(int m, int batch, const double *phases, void *U, int dtype, void *stream);

/*
 * Gradient of a real loss with respect to the mesh phases, given grad_U
 * (batch x m x m, PyTorch convention): grad_phases[b, l] = Re sum conj(G_U) o
 * dU/dphi_l, written to device FP64 batch x 2K.  Reverse sweep over the MZIs.
 */
int slos_mesh_backward(int m, int batch, const double *phases, const void *grad_U, double *grad_phases, int dtype,
                       void *stream);

/* ---- batches of independent instances --------------------------------------- */

typedef struct slos_batch_s *slos_batch_t;

/*
 * Plan `count` independent instances of uneven size (the QML loop of Appendix
 * B.6 evaluates many unitaries per loss).  Instance i has ms[i] modes and its
 * input occupations follow those of instance i-1 in `inputs` (sum of ms[i]
 * int32 in total), with at most 16 photons.  flags: SLOS_C64 or SLOS_C128.
 * opts: leaf_max (default 1024), block_threads (64 to 1024; the larger give
 * the big instances more waves), grid_blocks (workgroups, default 1024),
 * outputs_per_lane (default 2); other fields are ignored.
 * The whole batch runs in one kernel launch.  An instance whose last layer has
 * at least four tiles per wave runs on a whole workgroup (its waves share each
 * layer, a barrier between layers); every other instance runs on a single
 * wave.  The host assigns both kinds largest-first to the least loaded
 * workgroup or wave, so no workgroup waits on another.
 */
int slos_batch_plan(int count, const int32_t *ms, const int32_t *inputs, int flags, const slos_options_t *opts,
                    slos_batch_t *out);
void slos_batch_destroy(slos_batch_t batch);

/* Packed layouts: U of instance i starts at element u_offsets[i] (row-major
 * m_i x m_i), its C(m_i+n_i-1, n_i) amplitudes at out_offsets[i] (colex
 * order).  Both arrays take count + 1 entries (the last is the total). */
int slos_batch_offsets(slos_batch_t batch, int64_t *u_offsets, int64_t *out_offsets);

/* All amplitudes of every instance (device, packed).  sum_p: device, count
 * doubles (sum of P per instance, FP64), or NULL. */
int slos_batch_amplitudes(slos_batch_t batch, const void *U, void *out, double *sum_p, void *stream);

/* Capture the batch launch for these buffers into a HIP graph owned by the
 * batch (replacing an earlier one); slos_batch_replay launches it on a stream.
 * The buffers stay bound to the graph. */
int slos_batch_capture(slos_batch_t batch, const void *U, void *out, double *sum_p);
int slos_batch_replay(slos_batch_t batch, void *stream);

/* ---- imperfect sources ------------------------------------------------------- */

/*
 * Source model (Section 3.2.4: a Processor's source tunes its emission
 * probability, multi-photon emission and indistinguishability; Appendix A.4,
 * Fig. slos_output2, prints their effect on the Ralph CNOT).  Every photon of
 * the input state comes from a source of its own, which emits nothing (p0),
 * one photon (p1) or two (p2), with p1 + p2 = emission_probability and
 * multiphoton_component = g2 = 2 p2 / (p1 + 2 p2)^2.  An emitted first photon
 * shares the common wavepacket with probability sqrt(indistinguishability)
 * (two such photons interfere with probability V, the HOM visibility), else it
 * is distinguishable from every other photon; the second photon of a pair is
 * always distinguishable.  Photons of different wavepackets do not interfere.
 * Defaults (src = NULL): a perfect source (1, 0, 1).
 */
typedef struct {
    double emission_probability;   /* (0, 1]                              */
    double multiphoton_component;  /* g2 in [0, 1], with its product by the
                                      emission probability at most 1/2     */
    double indistinguishability;   /* V in [0, 1]                          */
} slos_source_params_t;

typedef struct slos_source_s *slos_source_t;

/*
 * Plan the output distribution of the source mixture behind input_state (host,
 * m int32, n = sum <= 12 photons, i.e. sources) over the photon numbers
 * 0..nmax (nmax < 0: 2n when pairs are possible, else n; nmax <= min(2n, 16); the
 * states of photon numbers above nmax are dropped, those below are exact).
 * Output layout ("graded"): photon number k occupies elements
 * [offsets[k], offsets[k+1]) in colex order, offsets from slos_source_info;
 * fewer than 2^32 states in all.  opts: leaf_max (default 256) only.  The
 * plan allocates 1.5 x 2^n graded FP64 vectors of device scratch, the leaf
 * tables of photon numbers 1..nmax and a batch of the 2^n common-wavepacket
 * groups; it owns them until slos_source_destroy.
 * Errors: INVALID_ARG (bad sizes or source parameters), SIZE_OVERFLOW, OOM,
 * NO_DEVICE.
 */
int slos_source_plan(int m, const int32_t *input_state, const slos_source_params_t *src, int nmax,
                     const slos_options_t *opts, slos_source_t *out);
void slos_source_destroy(slos_source_t source);
/* Total states over photon numbers 0..nmax (-1 for a NULL plan). */
int64_t slos_source_num_outputs(slos_source_t source);
/* offsets (host, nmax + 2 int64, or NULL); emission (host, 3 doubles: p0,
 * p1, p2 of one source, or NULL). */
int slos_source_info(slos_source_t source, int64_t *offsets, double *emission);

/*
 * probs (device, num_outputs FP64, graded layout) = the mixture's output
 * probabilities for U (device, complex128 m x m, row = output mode).  The
 * common-wavepacket group of every subset of sources runs through the batch
 * kernel; a distinguishable photon entering mode i is the real-weight layer
 * P'[t] = sum_{j: t_j > 0} |U[j, i]|^2 P[t - e_j]; the subsets fold source by
 * source in 3 (2^n - 1) such passes.  FP64 throughout.  Asynchronous.
 */
int slos_source_probs(slos_source_t source, const void *U, double *probs, void *stream);

/*
 * Per photon number k = 0..nmax, result[3k .. 3k+2] (host) = total
 * probability, its part over the outputs with at least min_modes occupied
 * modes ("physical": at least min_modes detectors click), and the part of
 * that which passes the mode-group bounds of slos_postselect (group_of_mode,
 * ngroups, count_min, count_max, same conventions).  With min_modes = n and the
 * gate's heralds and groups, the sums over k give the physical performance and
 * (kept / physical) the gate performance of Fig. slos_output2.  FP64 in a fixed
 * order; synchronises the stream.
 */
int slos_source_postselect(slos_source_t source, const double *probs, const int32_t *group_of_mode, int ngroups,
                           const int32_t *count_min, const int32_t *count_max, int min_modes, double *result,
                           void *stream);

/* ---- timing ----------------------------------------------------------------- */

/*
 * Turn per-layer timing on (1) or off (0).  While on, each forward call
 * records a HIP event on its stream before layer 1, after every layer k and
 * after the final FP64 sum; slos_plan_layer_ms then waits for the last event
 * and writes ms[k-1] = duration of layer k (k = 1..n) and ms[n] = duration of
 * the sum reduction (0 if it did not run).  `count` must be >= n + 1.  Events
 * are owned by the plan.  Leave it off under stream capture.
 */
int slos_plan_set_timing(slos_plan_t plan, int on);
int slos_plan_layer_ms(slos_plan_t plan, float *ms, int count);

/* Last error message on the calling thread ("" if none). */
const char *slos_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SLOS_H */
