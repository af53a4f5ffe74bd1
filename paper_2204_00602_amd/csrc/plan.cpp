// Host side of the SLOS library: argument checks, Fock-space arithmetic
// (colex rank / unrank), the leaf tiling of every layer, inner tables, device
// buffers and the launch sequence of the layer recurrence.
//
// Method: arXiv 2204.00602, Section 3.2.3 (SLOS back-end: unfold the whole
// computation path, time O(n C(m+n-1, n))) and Section 4.2.1 (Eq. eqperm, the
// amplitude each output must equal).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <tuple>
#include <unordered_map>
#include <new>
#include <queue>
#include <string>
#include <thread>
#include <vector>

#include "slos_ext.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? SLOS_ERR_OOM : SLOS_ERR_HIP, "%s: %s", what,
                hipGetErrorString(e));
}

constexpr uint64_t kSat = ~uint64_t(0);

// Pascal table C(a, b), 0 <= a <= amax, 0 <= b <= bmax; saturates at kSat.
struct Binom {
    int amax = 0, bmax = 0, stride = 0;
    std::vector<uint64_t> t;
    void build(int amax_, int bmax_)
    {
        amax = amax_;
        bmax = bmax_;
        stride = bmax + 1;
        t.assign((size_t)(amax + 1) * stride, 0);
        for (int a = 0; a <= amax; ++a) {
            t[(size_t)a * stride] = 1;
            for (int b = 1; b <= std::min(a, bmax); ++b) {
                uint64_t x = t[(size_t)(a - 1) * stride + b - 1];
                uint64_t y = t[(size_t)(a - 1) * stride + b];
                uint64_t s;
                t[(size_t)a * stride + b] =
                    (x == kSat || y == kSat || __builtin_add_overflow(x, y, &s)) ? kSat : s;
            }
        }
    }
    uint64_t operator()(int a, int b) const
    {
        if (a < 0 || b < 0 || b > a) return 0;
        return t[(size_t)a * stride + b];
    }
};

// Exact C(a, b) with overflow detection (for the public count/rank helpers).
bool binom_exact(int a, int b, uint64_t *out)
{
    if (b < 0 || a < 0 || b > a) {
        *out = 0;
        return true;
    }
    b = std::min(b, a - b);
    unsigned __int128 r = 1;
    for (int i = 1; i <= b; ++i) {
        r = r * (unsigned __int128)(a - b + i) / (unsigned __int128)i;
        if (r > (unsigned __int128)INT64_MAX) return false;
    }
    *out = (uint64_t)r;
    return true;
}

int check_state(int m, int n, const int32_t *s, const char *what)
{
    if (!s) return fail(SLOS_ERR_INVALID_ARG, "%s is NULL", what);
    long tot = 0;
    for (int j = 0; j < m; ++j) {
        if (s[j] < 0) return fail(SLOS_ERR_INVALID_ARG, "%s[%d] = %d is negative", what, j, s[j]);
        tot += s[j];
    }
    if (tot != n)
        return fail(SLOS_ERR_INVALID_ARG, "%s holds %ld photons, expected %d", what, tot, n);
    return SLOS_OK;
}

// Colex rank of the k-photon state occ (m modes) with a saturating table.
uint64_t colex_rank(const Binom &B, int m, const int32_t *occ)
{
    uint64_t r = 0;
    int pos = 0;
    for (int j = 0; j < m; ++j)
        for (int c = 0; c < occ[j]; ++c) {
            ++pos;
            r += B(j + pos - 1, pos);
        }
    return r;
}

// Inverse: photon positions r = k..1 take the largest c_r < c_{r+1} with
// C(c_r, r) <= remaining rank; the photon's mode is c_r - r + 1.
void colex_unrank(const Binom &B, int m, int k, uint64_t rank, int32_t *occ)
{
    std::fill(occ, occ + m, 0);
    int c = m + k - 1;  // exclusive upper bound for c_k
    for (int r = k; r >= 1; --r) {
        int cc = c - 1;
        while (cc >= r && B(cc, r) > rank) --cc;
        if (cc < r - 1) cc = r - 1;
        rank -= B(cc, r);
        occ[cc - r + 1] += 1;
        c = cc;
    }
}

// Process order of a layer's leaves: group the leaves of one inner shape (q, K)
// whose high parts agree once their d highest photons (hm[0..d), the modes are
// descending) are removed, so that a group's shared predecessor blocks are read
// while they are still in cache; colex order puts such leaves far apart (the
// top photon is the most significant).  Groups in lexicographic order of the
// remaining photons, leaves within a group by their top photons.
void order_leaves(std::vector<LeafRec> &lv, int d)
{
    std::stable_sort(lv.begin(), lv.end(), [d](const LeafRec &a, const LeafRec &b) {
        if (a.q != b.q) return a.q < b.q;
        if (a.K != b.K) return a.K < b.K;
        const int n = a.nhp;  // equal: the same layer and K
        for (int i = d; i < n; ++i)
            if (a.hm[i] != b.hm[i]) return a.hm[i] < b.hm[i];
        for (int i = 0; i < std::min(d, n); ++i)
            if (a.hm[i] != b.hm[i]) return a.hm[i] < b.hm[i];
        return a.out_base < b.out_base;
    });
}

} // namespace

// FNV-1a over the bytes of a short key
struct ByteVecHash {
    size_t operator()(const std::vector<uint8_t> &v) const
    {
        uint64_t h = 1469598103934665603ull;
        for (uint8_t b : v) h = (h ^ b) * 1099511628211ull;
        return (size_t)h;
    }
};

struct slos_plan_s {
    int m = 0, n = 0, flags = 0;
    bool c64 = true, comp = false, keep = false, host_only = false;
    slos_options_t opts{};
    std::vector<int> photons;      // i_1 <= ... <= i_n
    double norm_t = 1.0;           // 1 / sqrt(prod t!)
    Binom B;
    std::vector<uint64_t> Nk;      // N_0 .. N_n
    std::vector<std::vector<LeafRec>> leaves;  // index k = 1..n
    std::vector<uint32_t> low_max;             // per layer: largest low block
    std::vector<InnerType> types;
    std::vector<uint32_t> pred;
    std::vector<double> lowfac;
    std::map<std::pair<int, int>, uint32_t> type_of;

    // device
    int device = -1;
    uint64_t *d_binom = nullptr;
    LeafRec *d_leaves = nullptr;
    std::vector<uint64_t> leaf_off;   // per layer offset into d_leaves
    unsigned char *d_desc = nullptr;  // leaf descriptors of all layers
    std::vector<uint64_t> desc_off;   // per layer byte offset into d_desc
    std::vector<int> desc_wide;       // per layer: wide descriptors
    InnerType *d_types = nullptr;
    uint32_t *d_pred = nullptr;
    double *d_lowfac = nullptr;
    void *d_vac = nullptr;            // A_0 = [1]
    void *d_buf[2] = {nullptr, nullptr};
    void *d_keep = nullptr;           // A_0..A_{n-1} when KEEP_LAYERS
    std::vector<uint64_t> keep_off;   // element offsets of A_k in d_keep
    double *d_partials = nullptr;
    int64_t n_partials = 0;
    int batch_cap = 1;                // instances per call (opts.max_batch)
    uint64_t keep_stride = 0;         // elements per instance in d_keep
    uint64_t buf_stride[2] = {0, 0};  // elements per instance in d_buf[b]
    uint64_t g_stride = 0;            // elements per instance in d_g[b]
    uint64_t bpart_stride = 0;        // double2 per instance in d_bpart
    uint32_t *d_tickets = nullptr;    // SLOS_XCDS ticket counters per layer
    double *d_cdf = nullptr;          // block prefix of the last slos_cdf input (nb + 1), run prefixes, chunk sums, search tree
    int64_t *d_pk_ends = nullptr;     // C(K+n-1, n) for K = 1..m
    double *d_ps_partials = nullptr;  // post-selection partial sums + reduction stage
    SelectTarget *d_sel = nullptr;    // target descriptors of the last slos_select call
    SelectTarget *h_sel = nullptr;    // their pinned host staging (sel_cap entries)
    std::vector<SelectTarget> sel_build;  // built here, then copied to the staging
    // sub-lattice tables of every occupation multiset seen by slos_select so
    // far (kept across calls; re-uploaded when a call adds one)
    std::unordered_map<std::vector<uint8_t>, uint32_t, ByteVecHash> sel_pat_of;
    std::unordered_map<uint64_t, uint32_t> sel_key;  // multiset key -> pattern
    std::vector<SelectPattern> sel_pats;
    std::vector<uint16_t> sel_state;
    std::vector<uint32_t> sel_mask;
    size_t sel_uploaded = 0;          // patterns on the device
    unsigned char *d_sel_tab = nullptr;  // patterns, then states, then masks
    size_t sel_tab_cap = 0, sel_st_bytes = 0;
    PsType *d_ps_types = nullptr;     // inner types of the last layer, table runs
    uint32_t *d_ps_type_off = nullptr;// first table entry per inner-type index
    uint8_t *d_ps_low = nullptr;      // group counts of every low state (per call)
    uint32_t ps_ntypes = 0, ps_entries = 0;
    // post-selection's own leaves of the last layer: it stages nothing in LDS,
    // so they have no low-block cap and may be larger than the recurrence's
    // (fewer per-leaf set-ups, while the low-state table of their shapes still
    // fits the L2); their tab indexes ps_type_list, inner shapes only
    std::vector<LeafRec> ps_leaves;
    std::vector<PsType> ps_type_list;
    std::map<std::pair<int, int>, uint32_t> ps_type_of;
    bool ps_pass = false;             // gen_leaves is building ps_leaves
    uint64_t ps_leaf_off = 0;         // ps_leaves in d_leaves
    size_t sel_cap = 0;
    // differentiation (SLOS_KEEP_LAYERS plans)
    std::vector<std::vector<BwdUnit>> units;   // per layer
    std::vector<uint32_t> succ;                // inner successor tables
    std::vector<uint64_t> hbase;               // high-mode successor block bases
    std::map<std::pair<int, int>, uint32_t> succ_of;
    BwdUnit *d_units = nullptr;
    std::vector<uint64_t> unit_off;
    uint32_t *d_succ = nullptr;
    uint64_t *d_hbase = nullptr;
    void *d_g[2] = {nullptr, nullptr};         // adjoint layers (ping-pong)
    void *d_bpart = nullptr;                   // double2 partials, all layers
    std::vector<uint64_t> bpart_off;           // per layer, in double2 units
    int32_t *d_photons = nullptr;
    bool timing = false;
    bool timed_reduce = false;
    std::vector<hipEvent_t> events;   // n + 2 when timing is on
    hipGraphExec_t graph = nullptr;   // slos_plan_capture

    size_t elem() const { return c64 ? 8 : 16; }

    uint32_t inner_type(int q, int K)
    {
        auto key = std::make_pair(q, K);
        auto it = type_of.find(key);
        if (it != type_of.end()) return it->second;
        InnerType ty{};
        ty.q = (uint16_t)q;
        ty.K = (uint16_t)K;
        ty.size = (uint32_t)B(q + K - 1, K);
        ty.low_size = K > 0 ? (uint32_t)B(q + K - 2, K - 1) : 0u;
        std::vector<int32_t> occ(q), sub(q);
        // first pass: cmax
        uint32_t cmax = 0;
        for (uint32_t x = 0; x < ty.size; ++x) {
            colex_unrank(B, q, K, x, occ.data());
            uint32_t cnt = 0;
            for (int j = 0; j < q; ++j) cnt += occ[j] > 0;
            cmax = std::max(cmax, cnt);
        }
        ty.cmax = cmax;
        ty.pred_off = pred.size();
        ty.fac_off = lowfac.size();
        pred.resize(pred.size() + (size_t)cmax * ty.size, SLOS_ZERO_MODE << 24);
        lowfac.resize(lowfac.size() + ty.size, 1.0);
        for (uint32_t x = 0; x < ty.size; ++x) {
            colex_unrank(B, q, K, x, occ.data());
            uint32_t c = 0;
            double f = 1.0;
            for (int j = 0; j < q; ++j) {
                for (int v = 2; v <= occ[j]; ++v) f *= v;
                if (occ[j] == 0) continue;
                sub = occ;
                sub[j] -= 1;
                uint64_t p = colex_rank(B, q, sub.data());
                pred[ty.pred_off + (size_t)c * ty.size + x] = ((uint32_t)j << 24) | (uint32_t)p;
                ++c;
            }
            lowfac[ty.fac_off + x] = std::sqrt(f);
        }
        uint32_t id = (uint32_t)types.size();
        types.push_back(ty);
        type_of[key] = id;
        return id;
    }

    // inner shape (q, K) of a post-selection leaf: only its size is needed
    uint32_t ps_type(int q, int K)
    {
        auto key = std::make_pair(q, K);
        auto it = ps_type_of.find(key);
        if (it != ps_type_of.end()) return it->second;
        const uint32_t id = (uint32_t)ps_type_list.size();
        ps_type_list.push_back(PsType{0, (uint32_t)B(q + K - 1, K), (uint16_t)q, (uint16_t)K, 0});
        ps_type_of[key] = id;
        return id;
    }

    // Leaves of layer k: split F(j+1, K) by the occupation of mode j (blocks
    // t_j = 0, 1, .., K in colex order) until a block holds <= cap states.
    uint64_t low_cap = ~uint64_t(0);   // largest low block a leaf may have (elements)

    void gen_leaves(int k, int j, int K, uint64_t cap, std::vector<uint8_t> &hm, std::vector<LeafRec> &out)
    {
        uint64_t size = B(j + K, K);
        const uint64_t low = K > 0 ? B(j + K - 1, K - 1) : 0;
        if (K == 0 || j == 0 || (size <= cap && low <= low_cap)) {
            LeafRec L{};
            L.q = (uint8_t)(j + 1);
            L.K = (uint8_t)K;
            L.nhp = (uint8_t)hm.size();
            for (size_t i = 0; i < hm.size(); ++i) L.hm[i] = hm[i];
            L.size = (uint32_t)size;
            L.tab = ps_pass ? ps_type(j + 1, K) : inner_type(j + 1, K);
            // rank of the leaf's first state: low photons all in mode 0 add
            // C(r-1, r) = 0; high photon at position r = k - idx adds C(d+r-1, r)
            uint64_t base = 0;
            for (size_t idx = 0; idx < hm.size(); ++idx) {
                int r = k - (int)idx;
                base += B(hm[idx] + r - 1, r);
            }
            L.out_base = base;
            // FP64 normalisation of the high part: sqrt(prod o_j!) / sqrt(prod t_i!)
            double f = 1.0;
            int run = 0;
            for (size_t idx = 0; idx < hm.size(); ++idx) {
                run = (idx > 0 && hm[idx] == hm[idx - 1]) ? run + 1 : 1;
                f *= (double)run;
            }
            L.fac_hi = std::sqrt(f) * norm_t;
            out.push_back(L);
            return;
        }
        for (int s = 0; s <= K; ++s) {
            for (int c = 0; c < s; ++c) hm.push_back((uint8_t)j);
            gen_leaves(k, j - 1, K - s, cap, hm, out);
            for (int c = 0; c < s; ++c) hm.pop_back();
        }
    }

    // Host-side expansion of a leaf into its descriptor head and groups:
    // for the top photon of high mode d at position r (c = d + r - 1),
    //   rank(t) - rank(t - e_d) = C(c, r) + sum_{r' > r} C(c_{r'} - 1, r'),
    // and the low block (same high part, K-1 low photons) starts at
    //   out_base - sum_{r > K} C(c_r - 1, r).
    void describe(int k, const LeafRec &L, LeafDescHead &h, std::vector<uint64_t> &deltas,
                  std::vector<uint8_t> &modes) const
    {
        const InnerType &ty = types[L.tab];
        uint64_t S = 0;
        int prev = -1;
        std::vector<uint64_t> bases;
        deltas.clear();
        modes.clear();
        for (int idx = 0; idx < L.nhp; ++idx) {
            const int r = k - idx;
            const int d = L.hm[idx];
            const int c = d + r - 1;
            if (d != prev) {
                bases.push_back(L.out_base - (B(c, r) + S));
                modes.push_back((uint8_t)d);
                prev = d;
            }
            S += B(c - 1, r);
        }
        h = LeafDescHead{};
        h.out_base = L.out_base;
        h.low_base = L.out_base - S;
        h.fac_hi = L.fac_hi;
        h.size = L.size;
        h.low_size = ty.low_size;
        h.pred_off = (uint32_t)ty.pred_off;
        h.fac_off = (uint32_t)ty.fac_off;
        h.cmax = (uint8_t)ty.cmax;
        h.nh = (uint8_t)modes.size();
        h.q = L.q;
        h.K = L.K;
        for (uint64_t b : bases) deltas.push_back(h.low_base - b);
    }

    // succ[i*low_size + y] = colex rank in F(q, K) of y + e_i, y in F(q, K-1)
    uint32_t succ_table(int q, int K)
    {
        auto key = std::make_pair(q, K);
        auto it = succ_of.find(key);
        if (it != succ_of.end()) return it->second;
        const uint32_t ls = (uint32_t)B(q + K - 2, K - 1);
        const uint32_t off = (uint32_t)succ.size();
        succ.resize(succ.size() + (size_t)q * ls);
        std::vector<int32_t> occ(q);
        for (uint32_t y = 0; y < ls; ++y) {
            colex_unrank(B, q, K - 1, y, occ.data());
            for (int i = 0; i < q; ++i) {
                occ[i] += 1;
                succ[off + (size_t)i * ls + y] = (uint32_t)colex_rank(B, q, occ.data());
                occ[i] -= 1;
            }
        }
        succ_of[key] = off;
        return off;
    }

    // reverse-layer units of layer k: one per forward leaf with K >= 1
    // low states per reverse unit of layer k: 128, doubled (up to 1024) while
    // the layer would still have more than 8192 units for a full batch
    std::vector<uint32_t> unit_chunk;

    void build_units(int k)
    {
        if ((int)unit_chunk.size() <= k) unit_chunk.resize(k + 1, 128u);
        uint32_t ch = 128;
        while (ch < 1024 && (Nk[k - 1] / ch) * (uint64_t)batch_cap > 8192) ch *= 2;
        unit_chunk[k] = ch;
        // The units come from a leaf split of their own, at the full leaf size:
        // the forward splits small layers into many small leaves to spread
        // them over the chip, which would leave many units of a few states
        // each (the chunks above spread the reverse layer instead).
        std::vector<LeafRec> lv;
        std::vector<uint8_t> hm0;
        gen_leaves(k, m - 1, k, (uint64_t)opts.leaf_max, hm0, lv);
        std::vector<int32_t> occ(m);
        for (const LeafRec &L : lv) {
            if (L.K == 0) continue;
            BwdUnit u{};
            LeafDescHead h;
            std::vector<uint64_t> dl;
            std::vector<uint8_t> md;
            describe(k, L, h, dl, md);
            u.out_base = h.out_base;
            u.low_base = h.low_base;
            u.low_size = h.low_size;
            u.q = L.q;
            u.succ_off = succ_table(L.q, L.K);
            u.hbase_off = hbase.size();
            // state (h + e_j, K-1 low photons in mode 0) for each high mode j
            std::fill(occ.begin(), occ.end(), 0);
            for (int i = 0; i < L.nhp; ++i) occ[L.hm[i]] += 1;
            occ[0] += L.K - 1;
            for (int j = L.q; j < m; ++j) {
                occ[j] += 1;
                hbase.push_back(colex_rank(B, m, occ.data()));
                occ[j] -= 1;
            }
            // one unit per chunk of the low block, so that small layers still
            // spread over many waves
            for (uint32_t y0 = 0; y0 < u.low_size; y0 += unit_chunk[k]) {
                u.y0 = y0;
                units[k].push_back(u);
            }
        }
    }

    void free_device()
    {
        auto f = [](void *p) {
            if (p) (void)hipFree(p);
        };
        f(d_binom);
        f(d_leaves);
        f(d_desc);
        d_desc = nullptr;
        f(d_types);
        f(d_pred);
        f(d_lowfac);
        f(d_vac);
        f(d_buf[0]);
        f(d_buf[1]);
        f(d_keep);
        f(d_partials);
        f(d_tickets);
        d_tickets = nullptr;
        f(d_cdf);
        d_cdf = nullptr;
        f(d_pk_ends);
        d_pk_ends = nullptr;
        f(d_ps_partials);
        d_ps_partials = nullptr;
        f(d_sel);
        d_sel = nullptr;
        if (h_sel) (void)hipHostFree(h_sel);
        h_sel = nullptr;
        f(d_sel_tab);
        d_sel_tab = nullptr;
        sel_tab_cap = 0;
        sel_uploaded = 0;
        f(d_ps_types);
        d_ps_types = nullptr;
        f(d_ps_type_off);
        d_ps_type_off = nullptr;
        f(d_ps_low);
        d_ps_low = nullptr;
        sel_cap = 0;
        f(d_units);
        f(d_succ);
        f(d_hbase);
        f(d_g[0]);
        f(d_g[1]);
        f(d_bpart);
        f(d_photons);
        d_units = nullptr;
        d_succ = nullptr;
        d_hbase = nullptr;
        d_g[0] = d_g[1] = nullptr;
        d_bpart = nullptr;
        d_photons = nullptr;
        d_binom = nullptr;
        d_leaves = nullptr;
        d_types = nullptr;
        d_pred = nullptr;
        d_lowfac = nullptr;
        d_vac = nullptr;
        d_buf[0] = d_buf[1] = nullptr;
        d_keep = nullptr;
        d_partials = nullptr;
        for (hipEvent_t ev : events) (void)hipEventDestroy(ev);
        events.clear();
        if (graph) (void)hipGraphExecDestroy(graph);
        graph = nullptr;
    }
};

namespace {

template <typename T>
int dev_upload(T **dst, const T *src, size_t count, const char *what)
{
    size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc((void **)dst, bytes);
    if (e != hipSuccess) return hip_fail(e, what);
    if (count) {
        e = hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, what);
    }
    return SLOS_OK;
}

int alloc_dev(void **dst, size_t bytes, const char *what)
{
    hipError_t e = hipMalloc(dst, std::max<size_t>(bytes, 1));
    if (e != hipSuccess) return hip_fail(e, what);
    return SLOS_OK;
}

int check_plan(slos_plan_t p)
{
    if (!p) return fail(SLOS_ERR_INVALID_ARG, "plan is NULL");
    if (p->host_only) return fail(SLOS_ERR_INVALID_ARG, "plan was built with SLOS_HOST_ONLY");
    return SLOS_OK;
}

} // namespace

extern "C" {

const char *slos_last_error(void) { return g_last_error.c_str(); }

int slos_fock_count(int m, int n, int64_t *count)
{
    if (m < 1 || n < 0 || !count) return fail(SLOS_ERR_INVALID_ARG, "need m >= 1, n >= 0, count != NULL");
    uint64_t c;
    if (!binom_exact(m + n - 1, n, &c))
        return fail(SLOS_ERR_SIZE_OVERFLOW, "C(%d, %d) exceeds int64", m + n - 1, n);
    *count = (int64_t)c;
    return SLOS_OK;
}

int slos_fock_rank(int m, int n, const int32_t *state, int64_t *rank)
{
    if (m < 1 || n < 0 || !rank) return fail(SLOS_ERR_INVALID_ARG, "need m >= 1, n >= 0, rank != NULL");
    int rc = check_state(m, n, state, "state");
    if (rc) return rc;
    int64_t cnt;
    if ((rc = slos_fock_count(m, n, &cnt))) return rc;
    Binom B;
    B.build(m + n, n);
    *rank = (int64_t)colex_rank(B, m, state);
    return SLOS_OK;
}

int slos_fock_unrank(int m, int n, int64_t rank, int32_t *state)
{
    if (m < 1 || n < 0 || !state) return fail(SLOS_ERR_INVALID_ARG, "need m >= 1, n >= 0, state != NULL");
    int64_t cnt;
    int rc = slos_fock_count(m, n, &cnt);
    if (rc) return rc;
    if (rank < 0 || rank >= cnt)
        return fail(SLOS_ERR_INVALID_ARG, "rank %lld outside [0, %lld)", (long long)rank, (long long)cnt);
    Binom B;
    B.build(m + n, n);
    colex_unrank(B, m, n, (uint64_t)rank, state);
    return SLOS_OK;
}

int slos_plan(int m, int n, const int32_t *input_state, int flags, slos_plan_t *out)
{
    return slos_plan_ex(m, n, input_state, flags, nullptr, out);
}

int slos_plan_ex(int m, int n, const int32_t *input_state, int flags, const slos_options_t *opts,
                 slos_plan_t *out)
{
    if (!out) return fail(SLOS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (m < 1 || m > SLOS_MAX_MODES)
        return fail(SLOS_ERR_INVALID_ARG, "m = %d outside [1, %d]", m, SLOS_MAX_MODES);
    if (n < 0 || n > SLOS_MAX_PHOTONS)
        return fail(SLOS_ERR_INVALID_ARG, "n = %d outside [0, %d]", n, SLOS_MAX_PHOTONS);
    int rc = check_state(m, n, input_state, "input_state");
    if (rc) return rc;
    const int known = SLOS_C64 | SLOS_C128 | SLOS_COMPENSATED | SLOS_COMP_KNUTH | SLOS_COMP_FP64 | SLOS_KEEP_LAYERS |
                      SLOS_HOST_ONLY;
    if (flags & ~known) return fail(SLOS_ERR_INVALID_ARG, "unknown flag bits 0x%x", flags & ~known);
    int dt = flags & (SLOS_C64 | SLOS_C128);
    if (dt != SLOS_C64 && dt != SLOS_C128)
        return fail(SLOS_ERR_DTYPE, "flags must hold exactly one of SLOS_C64, SLOS_C128");
    if ((flags & SLOS_COMPENSATED) && dt != SLOS_C64)
        return fail(SLOS_ERR_DTYPE, "SLOS_COMPENSATED applies to SLOS_C64 plans only");
    if ((flags & SLOS_COMP_KNUTH) && !(flags & SLOS_COMPENSATED))
        return fail(SLOS_ERR_INVALID_ARG, "SLOS_COMP_KNUTH needs SLOS_COMPENSATED");
    if ((flags & SLOS_COMP_FP64) && !(flags & SLOS_COMPENSATED))
        return fail(SLOS_ERR_INVALID_ARG, "SLOS_COMP_FP64 needs SLOS_COMPENSATED");
    if ((flags & SLOS_COMP_FP64) && (flags & SLOS_COMP_KNUTH))
        return fail(SLOS_ERR_INVALID_ARG, "SLOS_COMP_FP64 and SLOS_COMP_KNUTH exclude each other");
    int64_t M;
    if ((rc = slos_fock_count(m, n, &M))) return rc;

    slos_options_t o{};
    if (opts) o = *opts;
    // defaults: the fastest settings of a coordinate-descent search at
    // m=24, n=12 on gfx950 (a c128 low block of an 8192-state leaf takes
    // enough LDS to halve the resident workgroups, hence the smaller leaves)
    // plans that keep their layers (gradients, many small unitaries) default to
    // the fastest settings measured on the m=12, n=6 mesh gradient of 64
    // unitaries: 4096-state leaves, two outputs per lane, 128-thread workgroups
    if (o.leaf_max == 0) o.leaf_max = (flags & SLOS_KEEP_LAYERS) ? 4096 : (dt == SLOS_C64 ? 16384 : 8192);
    // low blocks of at most 24 KiB (c64: six workgroups of two-output tiles
    // per CU, the occupancy their 80 VGPRs allow) or 40 KiB (c128: three); the
    // leaves with larger low blocks are split further
    if (o.low_block_max == 0) o.low_block_max = (flags & SLOS_KEEP_LAYERS) ? -1 : (dt == SLOS_C64 ? 3072 : 2560);
    if (o.comp_from_layer == 0) o.comp_from_layer = 1;
    if (o.block_threads == 0) o.block_threads = (flags & SLOS_KEEP_LAYERS) ? 128 : 256;
    if (o.grid_blocks == 0) o.grid_blocks = 2048;
    if (o.outputs_per_lane == 0) o.outputs_per_lane = 2;
    if (o.xcd_chunk == 0) o.xcd_chunk = 128;
    if (o.ticket_leaves == 0) o.ticket_leaves = dt == SLOS_C64 ? 1 : 2;  // c64: the smaller leaves of its cap favour 1
    if (o.max_batch == 0) o.max_batch = 1;
    if (o.wide_descriptors < 0 || o.wide_descriptors > 1)
        return fail(SLOS_ERR_INVALID_ARG, "wide_descriptors must be 0 or 1");
    if (o.leaf_order < -1 || o.leaf_order > 4)
        return fail(SLOS_ERR_INVALID_ARG, "leaf_order = %d outside [-1, 4]", o.leaf_order);
    if (o.low_block_max < -1)
        return fail(SLOS_ERR_INVALID_ARG, "low_block_max = %d is below -1", o.low_block_max);
    if (o.max_batch < 1 || o.max_batch > 65535)
        return fail(SLOS_ERR_INVALID_ARG, "max_batch = %d outside [1, 65535]", o.max_batch);
    if (o.ticket_leaves < 1 || o.ticket_leaves > 4096)
        return fail(SLOS_ERR_INVALID_ARG, "ticket_leaves = %d outside [1, 4096]", o.ticket_leaves);
    if (o.xcd_chunk < 1 || o.xcd_chunk > (1 << 24))
        return fail(SLOS_ERR_INVALID_ARG, "xcd_chunk = %d outside [1, 2^24]", o.xcd_chunk);
    if (o.leaf_max < 1 || o.leaf_max > 65536)
        return fail(SLOS_ERR_INVALID_ARG, "leaf_max = %d outside [1, 65536]", o.leaf_max);
    if (o.block_threads != 64 && o.block_threads != 128 && o.block_threads != 256)
        return fail(SLOS_ERR_INVALID_ARG, "block_threads must be 64, 128 or 256");
    if (o.grid_blocks < 1 || o.grid_blocks > (1 << 20))
        return fail(SLOS_ERR_INVALID_ARG, "grid_blocks = %d outside [1, 2^20]", o.grid_blocks);
    if (o.outputs_per_lane != 1 && o.outputs_per_lane != 2 && o.outputs_per_lane != 4)
        return fail(SLOS_ERR_INVALID_ARG, "outputs_per_lane must be 1, 2 or 4");
    if (o.comp_from_layer < 1)
        return fail(SLOS_ERR_INVALID_ARG, "comp_from_layer must be >= 1");

    slos_plan_s *p = new (std::nothrow) slos_plan_s;
    if (!p) return fail(SLOS_ERR_OOM, "host allocation of the plan failed");
    p->m = m;
    p->n = n;
    p->flags = flags;
    p->c64 = dt == SLOS_C64;
    p->comp = (flags & SLOS_COMPENSATED) != 0;
    p->keep = (flags & SLOS_KEEP_LAYERS) != 0;
    p->host_only = (flags & SLOS_HOST_ONLY) != 0;
    p->opts = o;
    p->batch_cap = o.max_batch;

    if (o.low_block_max > 0) p->low_cap = (uint64_t)o.low_block_max;
    try {
        double tf = 1.0;
        for (int i = 0; i < m; ++i) {
            for (int c = 0; c < input_state[i]; ++c) p->photons.push_back(i);
            for (int v = 2; v <= input_state[i]; ++v) tf *= v;
        }
        p->norm_t = 1.0 / std::sqrt(tf);
        p->B.build(m + n, n);
        p->Nk.resize(n + 1);
        for (int k = 0; k <= n; ++k) p->Nk[k] = p->B(m + k - 1, k);

        // size checks: every buffer in bytes must fit size_t with room to spare
        uint64_t maxN = *std::max_element(p->Nk.begin(), p->Nk.end());
        if (maxN > (uint64_t(1) << 58))
            throw std::pair<int, std::string>(SLOS_ERR_SIZE_OVERFLOW, "layer too large for a device buffer");

        p->leaves.resize(n + 1);
        p->low_max.assign(n + 1, 0);
        for (int k = 1; k <= n; ++k) {
            // small layers get smaller leaves so that they still spread over
            // about SLOS_TARGET_LEAVES workgroups
            const uint64_t cap = std::min<uint64_t>((uint64_t)o.leaf_max,
                                                    std::max<uint64_t>(SLOS_MIN_LEAF, p->Nk[k] / SLOS_TARGET_LEAVES));
            std::vector<uint8_t> hm;
            p->gen_leaves(k, m - 1, k, cap, hm, p->leaves[k]);
            for (const LeafRec &L : p->leaves[k])
                p->low_max[k] = std::max(p->low_max[k], p->types[L.tab].low_size);
            // grouped order by default (depth 1: leaves that share the block
            // reached by removing their top photon run together)
            if (o.leaf_order >= 0) order_leaves(p->leaves[k], o.leaf_order > 0 ? o.leaf_order : 1);
        }
        if (n > 0) {
            const uint64_t saved = p->low_cap;
            p->low_cap = ~uint64_t(0);
            p->ps_pass = true;
            std::vector<uint8_t> hm;
            p->gen_leaves(n, m - 1, n, SLOS_PS_LEAF_MAX, hm, p->ps_leaves);
            order_leaves(p->ps_leaves, 1);  // the grouped order (measured faster than colex here too)
            p->ps_pass = false;
            p->low_cap = saved;
        }
        if (p->keep) {
            p->units.resize(n + 1);
            for (int k = 1; k <= n; ++k) p->build_units(k);
        }
        // one wave must be able to hold its low block in LDS
        const size_t es_ = (dt == SLOS_C64) ? 8 : 16;
        for (int k = 1; k <= n; ++k)
            if (slos_lds_wave_bytes(p->low_max[k], (uint32_t)es_) > SLOS_LDS_DYNAMIC_MAX)
                throw std::pair<int, std::string>(SLOS_ERR_INVALID_ARG,
                                                  "leaf_max too large: a low block does not fit in LDS");
    } catch (std::bad_alloc &) {
        delete p;
        return fail(SLOS_ERR_OOM, "host allocation failed while building tables");
    } catch (std::pair<int, std::string> &e) {
        delete p;
        return fail(e.first, "%s", e.second.c_str());
    }

    if (p->pred.size() >= (size_t(1) << 32) || p->lowfac.size() >= (size_t(1) << 32)) {
        delete p;
        return fail(SLOS_ERR_SIZE_OVERFLOW, "inner tables exceed 2^32 entries; lower leaf_max");
    }
    if (p->host_only) {
        *out = p;
        return SLOS_OK;
    }

    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev < 1) {
        delete p;
        return fail(SLOS_ERR_NO_DEVICE, "no HIP device (%s)", hipGetErrorString(e));
    }
    (void)hipGetDevice(&p->device);

    // upload tables
    std::vector<LeafRec> all;
    p->leaf_off.assign(n + 2, 0);
    for (int k = 1; k <= n; ++k) {
        p->leaf_off[k] = all.size();
        all.insert(all.end(), p->leaves[k].begin(), p->leaves[k].end());
    }
    p->leaf_off[n + 1] = all.size();
    p->ps_leaf_off = all.size();
    all.insert(all.end(), p->ps_leaves.begin(), p->ps_leaves.end());
    std::vector<unsigned char> descs;
    p->desc_off.assign(n + 2, 0);
    p->desc_wide.assign(n + 1, 0);
    try {
        std::vector<uint64_t> deltas;
        std::vector<uint8_t> modes;
        for (int k = 1; k <= n; ++k) {
            // narrow unless a leaf has more than 16 groups or a 64-bit delta
            int wide = p->opts.wide_descriptors > 0 ? 1 : 0;
            for (const LeafRec &L : p->leaves[k]) {
                LeafDescHead h;
                p->describe(k, L, h, deltas, modes);
                if (h.nh > SLOS_NARROW_GROUPS) wide = 1;
                for (uint64_t d : deltas)
                    if (d > 0xFFFFFFFFull) wide = 1;
                if (wide) break;
            }
            p->desc_wide[k] = wide;
            p->desc_off[k] = descs.size();
            const size_t rec = wide ? sizeof(LeafDescWide) : sizeof(LeafDescNarrow);
            descs.resize(descs.size() + rec * p->leaves[k].size());
            unsigned char *dst = descs.data() + p->desc_off[k];
            for (const LeafRec &L : p->leaves[k]) {
                LeafDescHead h;
                p->describe(k, L, h, deltas, modes);
                if (wide) {
                    LeafDescWide w{};
                    w.h = h;
                    for (size_t g = 0; g < deltas.size(); ++g) {
                        w.delta[g] = deltas[g];
                        w.mode[g] = modes[g];
                    }
                    std::memcpy(dst, &w, sizeof w);
                } else {
                    LeafDescNarrow w{};
                    w.h = h;
                    for (size_t g = 0; g < deltas.size(); ++g) {
                        w.delta[g] = (uint32_t)deltas[g];
                        w.mode[g] = modes[g];
                    }
                    std::memcpy(dst, &w, sizeof w);
                }
                dst += rec;
            }
        }
        p->desc_off[n + 1] = descs.size();
    } catch (std::bad_alloc &) {
        delete p;
        return fail(SLOS_ERR_OOM, "host allocation failed while building leaf descriptors");
    }
    if ((rc = dev_upload(&p->d_binom, p->B.t.data(), p->B.t.size(), "binomial table")) ||
        (rc = dev_upload(&p->d_leaves, all.data(), all.size(), "leaf table")) ||
        (rc = dev_upload(&p->d_desc, descs.data(), descs.size(), "leaf descriptors")) ||
        (rc = dev_upload(&p->d_types, p->types.data(), p->types.size(), "inner types")) ||
        (rc = dev_upload(&p->d_pred, p->pred.data(), p->pred.size(), "inner predecessor table")) ||
        (rc = dev_upload(&p->d_lowfac, p->lowfac.data(), p->lowfac.size(), "inner factorial table"))) {
        p->free_device();
        delete p;
        return rc;
    }

    // A_0 = [1]
    const size_t es = p->elem();
    {
        double one_d[2] = {1.0, 0.0};
        float one_f[2] = {1.0f, 0.0f};
        if ((rc = alloc_dev(&p->d_vac, es + SLOS_BUFFER_SLACK, "vacuum layer"))) {
            p->free_device();
            delete p;
            return rc;
        }
        e = hipMemcpy(p->d_vac, p->c64 ? (const void *)one_f : (const void *)one_d, es,
                      hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            rc = hip_fail(e, "vacuum upload");
            p->free_device();
            delete p;
            return rc;
        }
    }
    // intermediate layers 1..n-1
    if (p->keep) {
        p->keep_off.assign(n + 1, 0);
        uint64_t tot = 0;
        for (int k = 0; k < n; ++k) {
            p->keep_off[k] = tot;
            tot += (p->Nk[k] + 15) / 16 * 16;  // 128-byte aligned layers
        }
        p->keep_off[n] = tot;
        p->keep_stride = tot;
        if ((rc = alloc_dev(&p->d_keep, tot * es * p->batch_cap + SLOS_BUFFER_SLACK, "kept layers"))) {
            p->free_device();
            delete p;
            return rc;
        }
        for (int b = 0; b < p->batch_cap; ++b) {
            e = hipMemcpy((char *)p->d_keep + (size_t)b * tot * es, p->d_vac, es, hipMemcpyDeviceToDevice);
            if (e != hipSuccess) {
                rc = hip_fail(e, "kept vacuum layer");
                p->free_device();
                delete p;
                return rc;
            }
        }
    } else {
        uint64_t need[2] = {0, 0};
        for (int k = 1; k < n; ++k) need[k & 1] = std::max(need[k & 1], p->Nk[k]);
        for (int b = 0; b < 2; ++b) {
            need[b] = (need[b] + 31) / 32 * 32;  // 256-byte aligned instances
            p->buf_stride[b] = need[b];
        }
        for (int b = 0; b < 2; ++b)
            if (need[b] && (rc = alloc_dev(&p->d_buf[b], need[b] * es * p->batch_cap + SLOS_BUFFER_SLACK,
                                           "layer buffer"))) {
                p->free_device();
                delete p;
                return rc;
            }
    }
    p->n_partials = n > 0 ? (int64_t)p->leaves[n].size() * (p->opts.block_threads / 64) : 1;
    if ((rc = alloc_dev((void **)&p->d_partials,
                        (size_t)(p->n_partials + SLOS_REDUCE_STAGE) * p->batch_cap * sizeof(double), "partial sums")) ||
        (rc = alloc_dev((void **)&p->d_tickets,
                        (size_t)(n + 1) * SLOS_XCDS * SLOS_TICKET_STRIDE * p->batch_cap * sizeof(uint32_t),
                        "ticket counters"))) {
        p->free_device();
        delete p;
        return rc;
    }
    {
        const uint64_t nb = (p->Nk[n] + SLOS_CDF_BLOCK - 1) / SLOS_CDF_BLOCK;
        const uint64_t nsup = (nb + SLOS_CDF_BLOCK - 1) / SLOS_CDF_BLOCK;
        std::vector<int64_t> ends(m);
        for (int K = 1; K <= m; ++K) ends[K - 1] = (int64_t)p->B(K + n - 1, n);
        if ((rc = alloc_dev((void **)&p->d_cdf,
                            (nb + 1 + nsup + 1 + (uint64_t)(SLOS_CDF_BLOCK / 64) * nb +
                             (uint64_t)cdf_tree_layout((int64_t)nb).total) * sizeof(double),
                            "cumulative probability table")) ||
            (rc = dev_upload(&p->d_pk_ends, ends.data(), ends.size(), "marginal bounds")) ||
            (rc = alloc_dev((void **)&p->d_ps_partials, (SLOS_PS_MAX_WAVES + SLOS_REDUCE_STAGE) * sizeof(double),
                            "post-selection partial sums"))) {
            p->free_device();
            delete p;
            return rc;
        }
    }
    if (n > 0) {
        // post-selection tables: one run of low states per inner shape of
        // its leaves, in the order the shapes were met (ascending off)
        std::vector<uint32_t> off(p->ps_type_list.size(), 0);
        std::vector<PsType> pt = p->ps_type_list;
        uint64_t entries = 0;
        for (size_t i = 0; i < pt.size(); ++i) {
            off[i] = (uint32_t)entries;
            pt[i].off = (uint32_t)entries;
            entries += pt[i].size;
        }
        if (entries >= (1ull << 32)) {
            p->free_device();
            delete p;
            return fail(SLOS_ERR_SIZE_OVERFLOW, "post-selection table exceeds 2^32 entries");
        }
        p->ps_ntypes = (uint32_t)pt.size();
        p->ps_entries = (uint32_t)entries;
        if ((rc = dev_upload(&p->d_ps_types, pt.data(), pt.size(), "post-selection types")) ||
            (rc = dev_upload(&p->d_ps_type_off, off.data(), off.size(), "post-selection offsets")) ||
            (rc = alloc_dev((void **)&p->d_ps_low, entries * SLOS_PS_MAX_GROUPS, "post-selection table"))) {
            p->free_device();
            delete p;
            return rc;
        }
    }
    if (p->keep && n > 0) {
        std::vector<BwdUnit> allu;
        p->unit_off.assign(n + 2, 0);
        p->bpart_off.assign(n + 2, 0);
        uint64_t bp = 0;
        for (int k = 1; k <= n; ++k) {
            p->unit_off[k] = allu.size();
            p->bpart_off[k] = bp;
            allu.insert(allu.end(), p->units[k].begin(), p->units[k].end());
            bp += (uint64_t)p->units[k].size() * (uint64_t)m;
        }
        p->bpart_off[n + 1] = bp;
        uint64_t gmax = *std::max_element(p->Nk.begin(), p->Nk.end());
        gmax = (gmax + 31) / 32 * 32;
        p->g_stride = gmax;
        p->bpart_stride = std::max<uint64_t>(bp, 1);
        std::vector<int32_t> ph(p->photons.begin(), p->photons.end());
        if ((rc = dev_upload(&p->d_units, allu.data(), allu.size(), "reverse units")) ||
            (rc = dev_upload(&p->d_succ, p->succ.data(), p->succ.size(), "successor tables")) ||
            (rc = dev_upload(&p->d_hbase, p->hbase.data(), p->hbase.size(), "successor bases")) ||
            (rc = dev_upload(&p->d_photons, ph.data(), ph.size(), "photon list")) ||
            (rc = alloc_dev(&p->d_g[0], gmax * es * p->batch_cap, "adjoint layer")) ||
            (rc = alloc_dev(&p->d_g[1], gmax * es * p->batch_cap, "adjoint layer")) ||
            (rc = alloc_dev(&p->d_bpart, p->bpart_stride * 16 * p->batch_cap, "gradient partials"))) {
            p->free_device();
            delete p;
            return rc;
        }
    }
    *out = p;
    return SLOS_OK;
}

void slos_plan_destroy(slos_plan_t p)
{
    if (!p) return;
    if (!p->host_only) {
        (void)hipDeviceSynchronize();
        p->free_device();
    }
    delete p;
}

int64_t slos_num_outputs(slos_plan_t p)
{
    if (!p) return -1;
    return (int64_t)p->Nk[p->n];
}

int slos_rank(slos_plan_t p, const int32_t *state, int64_t *rank)
{
    // host arithmetic only: host-only plans are accepted
    if (!p) return fail(SLOS_ERR_INVALID_ARG, "plan is NULL");
    int rc;
    if (!rank) return fail(SLOS_ERR_INVALID_ARG, "rank is NULL");
    if ((rc = check_state(p->m, p->n, state, "state"))) return rc;
    *rank = (int64_t)colex_rank(p->B, p->m, state);
    return SLOS_OK;
}

int slos_unrank(slos_plan_t p, int64_t rank, int32_t *state)
{
    // host arithmetic only: host-only plans are accepted
    if (!p) return fail(SLOS_ERR_INVALID_ARG, "plan is NULL");
    if (!state) return fail(SLOS_ERR_INVALID_ARG, "state is NULL");
    const int64_t cnt = (int64_t)p->Nk[p->n];
    if (rank < 0 || rank >= cnt)
        return fail(SLOS_ERR_INVALID_ARG, "rank %lld outside [0, %lld)", (long long)rank, (long long)cnt);
    colex_unrank(p->B, p->m, p->n, (uint64_t)rank, state);
    return SLOS_OK;
}

int slos_plan_info(slos_plan_t p, int k, int64_t *n_states, int64_t *n_leaves)
{
    if (!p) return fail(SLOS_ERR_INVALID_ARG, "plan is NULL");
    if (k < 1 || k > p->n) return fail(SLOS_ERR_INVALID_ARG, "layer %d outside [1, %d]", k, p->n);
    if (n_states) *n_states = (int64_t)p->Nk[k];
    if (n_leaves) *n_leaves = (int64_t)p->leaves[k].size();
    return SLOS_OK;
}

int slos_plan_leaf(slos_plan_t p, int k, int64_t idx, int64_t *out_base, int32_t *q, int32_t *K,
                   int32_t *high_modes)
{
    if (!p) return fail(SLOS_ERR_INVALID_ARG, "plan is NULL");
    if (k < 1 || k > p->n) return fail(SLOS_ERR_INVALID_ARG, "layer %d outside [1, %d]", k, p->n);
    if (idx < 0 || (size_t)idx >= p->leaves[k].size())
        return fail(SLOS_ERR_INVALID_ARG, "leaf %lld out of range", (long long)idx);
    const LeafRec &L = p->leaves[k][idx];
    if (out_base) *out_base = (int64_t)L.out_base;
    if (q) *q = L.q;
    if (K) *K = L.K;
    if (high_modes)
        for (int i = 0; i < L.nhp; ++i) high_modes[i] = L.hm[i];
    return SLOS_OK;
}

// Device buffers of one forward pass beyond its inputs and outputs: the vacuum
// A_0, the two ping-pong layers, the FP64 partial sums (plus the reduction
// stage after them) and the ticket counters.
struct ForwardScratch {
    void *vac;
    void *buf[2];
    double *partials;
    uint32_t *tickets;
};

static int run_forward(slos_plan_t p, int batch, const void *U, void *out, double *sum_p, void *stream,
                       int last_mode, const ForwardScratch *over = nullptr)
{
    int rc = check_plan(p);
    if (rc) return rc;
    if (!U || !out) return fail(SLOS_ERR_INVALID_ARG, "U and out must be device pointers");
    if (batch < 1 || batch > p->batch_cap)
        return fail(SLOS_ERR_INVALID_ARG, "batch = %d outside [1, max_batch = %d]", batch, p->batch_cap);
    const int n = p->n;
    // bytes of one instance's output
    const size_t out_bytes = (size_t)p->Nk[n] * (last_mode == SLOS_MODE_PROB ? p->elem() / 2 : p->elem());
    if (n == 0) {
        for (int b = 0; b < batch; ++b) {
            int e = slos_launch_vacuum((char *)out + b * out_bytes, p->c64, last_mode, sum_p ? sum_p + b : nullptr,
                                       stream);
            if (e) return hip_fail((hipError_t)e, "vacuum kernel");
        }
        return SLOS_OK;
    }
    const size_t es = p->elem();
    const int wpb = p->opts.block_threads / 64;
    hipStream_t hs = (hipStream_t)stream;
    const uint64_t tstride = (uint64_t)(n + 1) * SLOS_XCDS * SLOS_TICKET_STRIDE;
    const ForwardScratch sc = over ? *over : ForwardScratch{p->d_vac, {p->d_buf[0], p->d_buf[1]}, p->d_partials,
                                                            p->d_tickets};
    {
        int e = slos_launch_zero_u32(sc.tickets, (int)(tstride * batch), stream);
        if (e) return hip_fail((hipError_t)e, "ticket reset kernel");
    }
    if (p->timing) {
        hipError_t e = hipEventRecord(p->events[0], hs);
        if (e != hipSuccess) return hip_fail(e, "timing event");
        p->timed_reduce = false;
    }
    for (int k = 1; k <= n; ++k) {
        LayerParams lp{};
        if (p->keep) {
            lp.X = (const char *)p->d_keep + p->keep_off[k - 1] * es;
            lp.Y = k == n ? out : (void *)((char *)p->d_keep + p->keep_off[k] * es);
            lp.x_stride = p->keep_stride * es;
            lp.y_stride = k == n ? out_bytes : p->keep_stride * es;
        } else {
            lp.X = k == 1 ? sc.vac : sc.buf[(k - 1) & 1];
            lp.Y = k == n ? out : sc.buf[k & 1];
            lp.x_stride = k == 1 ? 0 : p->buf_stride[(k - 1) & 1] * es;  // every instance reads the one vacuum
            lp.y_stride = k == n ? out_bytes : p->buf_stride[k & 1] * es;
        }
        lp.u_stride = (uint64_t)p->m * p->m * es;
        lp.partials_stride = (uint64_t)p->n_partials;
        lp.ticket_stride = tstride;
        lp.U = U;
        lp.leaves = p->d_leaves + p->leaf_off[k];
        lp.desc = p->d_desc + p->desc_off[k];
        lp.nleaves = p->leaves[k].size();
        lp.types = p->d_types;
        lp.pred = p->d_pred;
        lp.lowfac = p->d_lowfac;
        lp.binom = p->d_binom;
        lp.bstride = p->B.stride;
        lp.m = p->m;
        lp.k = k;
        lp.col = p->photons[k - 1];
        lp.norm_t = p->norm_t;
        lp.partials = sc.partials;
        LayerLaunch ll{};
        ll.c64 = p->c64;
        ll.mode = k == n ? last_mode : SLOS_MODE_MID;
        ll.compensated = (p->comp && k >= p->opts.comp_from_layer)
                             ? ((p->flags & SLOS_COMP_KNUTH)  ? SLOS_COMP_TWOSUM
                                : (p->flags & SLOS_COMP_FP64) ? SLOS_COMP_F64
                                                              : SLOS_COMP_BIASED)
                             : SLOS_COMP_NONE;
        ll.rr = p->opts.outputs_per_lane;
        ll.batch = batch;
        ll.threads = p->opts.block_threads;
        ll.low_max = p->low_max[k];
        ll.wide = p->desc_wide[k];
        lp.low_max = ll.low_max;
        lp.lds_wave_bytes = slos_lds_wave_bytes(ll.low_max, (uint32_t)es);
        // a workgroup shares one low block: LDS does not limit its wave count
        const int wpb_k = wpb;
        ll.threads = 64 * wpb_k;
        uint64_t want = lp.nleaves;  // one leaf per workgroup at a time
        ll.grid = (int)std::min<uint64_t>(want, (uint64_t)p->opts.grid_blocks);
        // a whole number of workgroups per XCD
        ll.grid = std::max(SLOS_XCDS, (ll.grid + SLOS_XCDS - 1) / SLOS_XCDS * SLOS_XCDS);
        // a layer with few leaves deals smaller chunks, so that every XCD gets some
        lp.xcd_chunk = (uint32_t)std::max<uint64_t>(
            1, std::min<uint64_t>((uint64_t)p->opts.xcd_chunk, lp.nleaves / (4 * SLOS_XCDS)));
        lp.tickets = sc.tickets + (size_t)k * SLOS_XCDS * SLOS_TICKET_STRIDE;
        const bool comp_k = ll.compensated == SLOS_COMP_BIASED;
        const bool comp_next = k < n && p->comp && !(p->flags & (SLOS_COMP_KNUTH | SLOS_COMP_FP64)) &&
                               k + 1 >= p->opts.comp_from_layer;
        lp.vmax_in = (comp_k && k >= 2)
                         ? sc.tickets + (size_t)(k - 1) * SLOS_XCDS * SLOS_TICKET_STRIDE + SLOS_VMAX_SLOT
                         : nullptr;
        lp.vmax_out = comp_next ? lp.tickets + SLOS_VMAX_SLOT : nullptr;
        lp.ticket_leaves = (uint32_t)p->opts.ticket_leaves;

        int e = slos_launch_layer(lp, ll, stream);
        if (e) return hip_fail((hipError_t)e, "layer kernel");
        if (p->timing && (e = (int)hipEventRecord(p->events[k], hs)))
            return hip_fail((hipError_t)e, "timing event");
        if (k == n && sum_p) {
            e = slos_launch_reduce(sc.partials, p->n_partials, sc.partials + p->n_partials * p->batch_cap, sum_p,
                                   stream, batch, p->n_partials);
            if (e) return hip_fail((hipError_t)e, "sum reduction kernel");
            if (p->timing) {
                if ((e = (int)hipEventRecord(p->events[n + 1], hs)))
                    return hip_fail((hipError_t)e, "timing event");
                p->timed_reduce = true;
            }
        }
    }
    return SLOS_OK;
}

int slos_plan_set_timing(slos_plan_t p, int on)
{
    int rc = check_plan(p);
    if (rc) return rc;
    if (on && p->events.empty()) {
        p->events.resize(p->n + 2);
        for (auto &ev : p->events) {
            hipError_t e = hipEventCreate(&ev);
            if (e != hipSuccess) {
                ev = nullptr;
                return hip_fail(e, "hipEventCreate");
            }
        }
    }
    p->timing = on != 0;
    return SLOS_OK;
}

int slos_plan_layer_ms(slos_plan_t p, float *ms, int count)
{
    int rc = check_plan(p);
    if (rc) return rc;
    if (!p->timing) return fail(SLOS_ERR_INVALID_ARG, "timing is off for this plan");
    if (!ms || count < p->n + 1) return fail(SLOS_ERR_INVALID_ARG, "ms needs n + 1 = %d entries", p->n + 1);
    if (p->n == 0) {
        ms[0] = 0.f;
        return SLOS_OK;
    }
    hipEvent_t last = p->timed_reduce ? p->events[p->n + 1] : p->events[p->n];
    hipError_t e = hipEventSynchronize(last);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    for (int k = 1; k <= p->n; ++k) {
        e = hipEventElapsedTime(&ms[k - 1], p->events[k - 1], p->events[k]);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    }
    ms[p->n] = 0.f;
    if (p->timed_reduce) {
        e = hipEventElapsedTime(&ms[p->n], p->events[p->n], p->events[p->n + 1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    }
    return SLOS_OK;
}

// The reverse layers n..1 from g_n (already in d_g[n & 1]) and the assembly of
// G_U; n >= 1.
static int run_reverse(slos_plan_t p, int batch, const void *U, void *grad_U, void *stream)
{
    const int n = p->n, m = p->m;
    const int c64 = p->c64 ? 1 : 0;
    const size_t es = p->elem();
    const uint64_t mm = (uint64_t)m * m;
    int e;
    for (int k = n; k >= 1; --k) {
        BwdParams bp{};
        bp.gk = p->d_g[k & 1];
        bp.gkm1 = p->d_g[(k - 1) & 1];
        bp.Akm1 = (const char *)p->d_keep + p->keep_off[k - 1] * es;
        bp.U = U;
        bp.units = p->d_units + p->unit_off[k];
        bp.nunits = p->units[k].size();
        bp.succ = p->d_succ;
        bp.hbase = p->d_hbase;
        bp.partials = (char *)p->d_bpart + p->bpart_off[k] * 16;
        bp.m = m;
        bp.col = p->photons[k - 1];
        bp.chunk = p->unit_chunk[k];
        bp.gk_stride = bp.gkm1_stride = p->g_stride * es;
        bp.a_stride = p->keep_stride * es;
        bp.u_stride = mm * es;
        bp.partials_stride = p->bpart_stride * 16;
        const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>(bp.nunits, 4096));
        // one pass per block of SLOS_BWD_MODE_BLOCK modes' gradient partials;
        // the first also forms g_{k-1}, which the next layer's passes read
        for (int jb = 0; jb < m; jb += SLOS_BWD_MODE_BLOCK) {
            bp.jb = jb;
            bp.jn = std::min(SLOS_BWD_MODE_BLOCK, m - jb);
            bp.write_g = jb == 0;
            if ((e = slos_launch_bwd_layer(bp, c64, grid, stream, batch)))
                return hip_fail((hipError_t)e, "reverse layer");
        }
    }
    // every layer's column sums and G_U in one launch
    ColsumLayers cl{};
    for (int k = 1; k <= n; ++k) {
        cl.off[k - 1] = p->bpart_off[k];
        cl.nunits[k - 1] = p->units[k].size();
    }
    if ((e = slos_launch_colsum_gradu(p->d_bpart, cl, p->d_photons, n, m, grad_U, c64, stream, batch,
                                      p->bpart_stride, mm)))
        return hip_fail((hipError_t)e, "gradient assembly");
    return SLOS_OK;
}

static int check_backward(slos_plan_t p, int batch, const void *U, void *grad_U)
{
    int rc = check_plan(p);
    if (rc) return rc;
    if (!p->keep) return fail(SLOS_ERR_NOT_KEPT, "slos_backward needs a plan built with SLOS_KEEP_LAYERS");
    if (!U || !grad_U) return fail(SLOS_ERR_INVALID_ARG, "U and grad_U must be device pointers");
    if (batch < 1 || batch > p->batch_cap)
        return fail(SLOS_ERR_INVALID_ARG, "batch = %d outside [1, max_batch = %d]", batch, p->batch_cap);
    return SLOS_OK;
}

// G_U = 0 for the vacuum: a(vacuum) = 1 does not depend on U
static int zero_grad_u(slos_plan_t p, int batch, void *grad_U, void *stream)
{
    const uint64_t mm = (uint64_t)p->m * p->m;
    int e = slos_launch_zero_u32((uint32_t *)grad_U, (int)(mm * p->elem() * batch / 4), stream);
    return e ? hip_fail((hipError_t)e, "zero kernel") : SLOS_OK;
}

static int run_backward(slos_plan_t p, int batch, const void *U, const void *grad_a, void *grad_U, void *stream)
{
    int rc = check_backward(p, batch, U, grad_U);
    if (rc) return rc;
    if (!grad_a) return fail(SLOS_ERR_INVALID_ARG, "grad_a must be a device pointer");
    const int n = p->n;
    if (n == 0) return zero_grad_u(p, batch, grad_U, stream);
    const size_t rec = p->desc_wide[n] ? sizeof(LeafDescWide) : sizeof(LeafDescNarrow);
    // g_n = c_S g_a
    int e;
    if ((e = slos_launch_seed(p->d_desc + p->desc_off[n], p->leaves[n].size(), (uint32_t)rec, p->d_lowfac, grad_a,
                              p->d_g[n & 1], p->c64 ? 1 : 0, stream, batch, p->Nk[n], p->g_stride)))
        return hip_fail((hipError_t)e, "seed kernel");
    return run_reverse(p, batch, U, grad_U, stream);
}

int slos_backward(slos_plan_t p, const void *U, const void *grad_a, void *grad_U, void *stream)
{
    return run_backward(p, 1, U, grad_a, grad_U, stream);
}

int slos_backward_many(slos_plan_t p, int batch, const void *U, const void *grad_a, void *grad_U, void *stream)
{
    return run_backward(p, batch, U, grad_a, grad_U, stream);
}

int slos_sq_loss_grad_many(slos_plan_t p, int batch, const void *a, const int64_t *ranks, int64_t count,
                           const double *p_target, void *grad_a, double *loss, void *stream)
{
    int rc = check_plan(p);
    if (rc) return rc;
    if (batch < 1 || batch > 65535) return fail(SLOS_ERR_INVALID_ARG, "batch = %d outside [1, 65535]", batch);
    if (count < 0) return fail(SLOS_ERR_INVALID_ARG, "count = %lld is negative", (long long)count);
    if (!a || !grad_a || (count > 0 && (!ranks || !p_target)))
        return fail(SLOS_ERR_INVALID_ARG, "a, grad_a (and ranks, p_target when count > 0) must be device pointers");
    int e = slos_launch_sq_loss(a, p->Nk[p->n], ranks, count, p_target, grad_a, loss, batch, p->c64 ? 1 : 0, stream);
    if (e) return hip_fail((hipError_t)e, "squared-loss kernel");
    return SLOS_OK;
}

int slos_output_scales(slos_plan_t p, const int64_t *ranks, int64_t count, double *scales)
{
    // host arithmetic only: host-only plans are accepted
    if (!p) return fail(SLOS_ERR_INVALID_ARG, "plan is NULL");
    if (count < 0) return fail(SLOS_ERR_INVALID_ARG, "count = %lld is negative", (long long)count);
    if (count > 0 && (!ranks || !scales)) return fail(SLOS_ERR_INVALID_ARG, "ranks and scales must be host arrays");
    const int n = p->n;
    const uint64_t M = p->Nk[n];
    if (n == 0) {
        for (int64_t t = 0; t < count; ++t) scales[t] = ranks[t] == 0 ? 1.0 : 0.0;
        return SLOS_OK;
    }
    // the last layer's leaves tile [0, N_n) by their first ranks
    const std::vector<LeafRec> &lv = p->leaves[n];
    std::vector<uint32_t> ord(lv.size());
    for (uint32_t i = 0; i < (uint32_t)ord.size(); ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](uint32_t x, uint32_t y) { return lv[x].out_base < lv[y].out_base; });
    for (int64_t t = 0; t < count; ++t) {
        const int64_t r = ranks[t];
        if (r < 0 || (uint64_t)r >= M) {
            scales[t] = 0.0;  // outside the output set (the loss ignores it)
            continue;
        }
        // last leaf whose first rank is <= r
        size_t lo = 0, hi = ord.size();
        while (hi - lo > 1) {
            const size_t mid = (lo + hi) / 2;
            if (lv[ord[mid]].out_base <= (uint64_t)r) lo = mid;
            else hi = mid;
        }
        const LeafRec &L = lv[ord[lo]];
        const uint64_t x = (uint64_t)r - L.out_base;
        // the factor the seed of the adjoint applies: fac_hi * inner factor
        scales[t] = L.fac_hi * p->lowfac[p->types[L.tab].fac_off + x];
    }
    return SLOS_OK;
}

int slos_sq_loss_backward_many(slos_plan_t p, int batch, const void *U, const void *a, const int64_t *ranks,
                               const double *scales, int64_t count, const double *p_target, void *grad_U,
                               double *loss, void *stream)
{
    int rc = check_backward(p, batch, U, grad_U);
    if (rc) return rc;
    if (count < 0) return fail(SLOS_ERR_INVALID_ARG, "count = %lld is negative", (long long)count);
    if (!a || (count > 0 && (!ranks || !scales || !p_target)))
        return fail(SLOS_ERR_INVALID_ARG, "a (and ranks, scales, p_target when count > 0) must be device pointers");
    const int n = p->n;
    if (n == 0) return fail(SLOS_ERR_INVALID_ARG, "n = 0: the vacuum has no adjoint layers");
    int e = slos_launch_sq_loss_seed(a, p->Nk[n], ranks, scales, count, p_target, p->d_g[n & 1], p->g_stride, loss,
                                     batch, p->c64 ? 1 : 0, stream);
    if (e) return hip_fail((hipError_t)e, "squared-loss seed kernel");
    return run_reverse(p, batch, U, grad_U, stream);
}

int slos_mesh_unitary(int m, int batch, const double *phases, void *U, int dtype, void *stream)
{
    if (m < 2 || m > SLOS_MESH_MAX_MODES || batch < 1 || !phases || !U)
        return fail(SLOS_ERR_INVALID_ARG, "need 2 <= m <= %d, batch >= 1 and device pointers", SLOS_MESH_MAX_MODES);
    if (dtype != SLOS_C64 && dtype != SLOS_C128) return fail(SLOS_ERR_DTYPE, "dtype must be SLOS_C64 or SLOS_C128");
    int e = slos_launch_mesh_forward(m, batch, phases, U, dtype == SLOS_C64, stream);
    if (e) return hip_fail((hipError_t)e, "mesh kernel");
    return SLOS_OK;
}

int slos_mesh_backward(int m, int batch, const double *phases, const void *grad_U, double *grad_phases, int dtype,
                       void *stream)
{
    if (m < 2 || m > SLOS_MESH_MAX_MODES || batch < 1 || !phases || !grad_U || !grad_phases)
        return fail(SLOS_ERR_INVALID_ARG, "need 2 <= m <= %d, batch >= 1 and device pointers", SLOS_MESH_MAX_MODES);
    if (dtype != SLOS_C64 && dtype != SLOS_C128) return fail(SLOS_ERR_DTYPE, "dtype must be SLOS_C64 or SLOS_C128");
    int e = slos_launch_mesh_backward(m, batch, phases, grad_U, grad_phases, dtype == SLOS_C64, stream);
    if (e) return hip_fail((hipError_t)e, "mesh reverse kernel");
    return SLOS_OK;
}

int slos_amplitudes(slos_plan_t p, const void *U, void *out, double *sum_p, void *stream)
{
    return run_forward(p, 1, U, out, sum_p, stream, SLOS_MODE_AMPL);
}

int slos_probs(slos_plan_t p, const void *U, void *probs, double *sum_p, void *stream)
{
    return run_forward(p, 1, U, probs, sum_p, stream, SLOS_MODE_PROB);
}

static size_t round256(size_t b) { return (b + 255) / 256 * 256; }

int slos_amplitudes_noalloc(slos_plan_t p, const void *U, void *out, double *sum_p, void *stream)
{
    int rc = check_plan(p);
    if (rc) return rc;
    if (p->keep)
        return fail(SLOS_ERR_INVALID_ARG, "slos_amplitudes_noalloc: the plan keeps its layers (SLOS_KEEP_LAYERS); "
                                          "use slos_amplitudes");
    if (!U || !out) return fail(SLOS_ERR_INVALID_ARG, "U and out must be device pointers");
    const int n = p->n;
    const size_t es = p->elem();
    // the plan's own buffers for one instance, carved from the static area:
    // vacuum | layer buffer 0 | layer buffer 1 | partials + reduction stage | tickets
    const size_t b_vac = round256(es + SLOS_BUFFER_SLACK);
    const size_t b_buf0 = p->buf_stride[0] ? round256(p->buf_stride[0] * es + SLOS_BUFFER_SLACK) : 0;
    const size_t b_buf1 = p->buf_stride[1] ? round256(p->buf_stride[1] * es + SLOS_BUFFER_SLACK) : 0;
    // (the reduction stage follows the partials of max_batch instances)
    const size_t b_part = round256((size_t)(p->n_partials * p->batch_cap + SLOS_REDUCE_STAGE) * sizeof(double));
    const size_t b_tick = round256((size_t)(n + 1) * SLOS_XCDS * SLOS_TICKET_STRIDE * sizeof(uint32_t));
    const size_t need = b_vac + b_buf0 + b_buf1 + b_part + b_tick;
    if (need > SLOS_STATIC_SCRATCH_BYTES)
        return fail(SLOS_ERR_SIZE_OVERFLOW,
                    "slos_amplitudes_noalloc: m = %d, n = %d needs %zu bytes of scratch; the static area holds %zu",
                    p->m, n, need, (size_t)SLOS_STATIC_SCRATCH_BYTES);
    void *base = nullptr;
    int dev = -1;
    int e = slos_static_scratch(&base, &dev);
    if (e) return hip_fail((hipError_t)e, "static scratch address");
    if (dev != p->device)
        return fail(SLOS_ERR_INVALID_ARG, "slos_amplitudes_noalloc: the plan lives on device %d, device %d is current",
                    p->device, dev);
    char *c = (char *)base;
    ForwardScratch sc{};
    sc.vac = c;
    sc.buf[0] = b_buf0 ? c + b_vac : nullptr;
    sc.buf[1] = b_buf1 ? c + b_vac + b_buf0 : nullptr;
    sc.partials = (double *)(c + b_vac + b_buf0 + b_buf1);
    sc.tickets = (uint32_t *)(c + b_vac + b_buf0 + b_buf1 + b_part);
    if (n > 0) {
        // the area keeps whatever the last call left: A_0 = [1] is written afresh
        // (the ticket counters are zeroed by the pass itself, and the partials
        // and the reduction stage are written before they are read)
        e = slos_launch_vacuum(sc.vac, p->c64, SLOS_MODE_AMPL, nullptr, stream);
        if (e) return hip_fail((hipError_t)e, "vacuum kernel");
    }
    return run_forward(p, 1, U, out, sum_p, stream, SLOS_MODE_AMPL, &sc);
}

int slos_amplitudes_many(slos_plan_t p, int batch, const void *U, void *out, double *sum_p, void *stream)
{
    return run_forward(p, batch, U, out, sum_p, stream, SLOS_MODE_AMPL);
}

int slos_probs_many(slos_plan_t p, int batch, const void *U, void *probs, double *sum_p, void *stream)
{
    return run_forward(p, batch, U, probs, sum_p, stream, SLOS_MODE_PROB);
}

int slos_plan_capture(slos_plan_t p, int batch, int probs, const void *U, void *out, double *sum_p)
{
    int rc = check_plan(p);
    if (rc) return rc;
    if (p->timing) return fail(SLOS_ERR_INVALID_ARG, "turn timing off before capturing the pass");
    if (p->graph) {
        (void)hipGraphExecDestroy(p->graph);
        p->graph = nullptr;
    }
    hipStream_t s;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "capture stream");
    hipGraph_t g = nullptr;
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(s);
        return hip_fail(e, "begin capture");
    }
    rc = run_forward(p, batch, U, out, sum_p, s, probs ? SLOS_MODE_PROB : SLOS_MODE_AMPL);
    const hipError_t ee = hipStreamEndCapture(s, &g);
    if (!rc && ee == hipSuccess) e = hipGraphInstantiate(&p->graph, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(s);
    if (rc) {
        p->graph = nullptr;
        return rc;  // run_forward set the message
    }
    if (ee != hipSuccess || e != hipSuccess) {
        p->graph = nullptr;
        return hip_fail(ee != hipSuccess ? ee : e, "graph capture of the forward pass");
    }
    return SLOS_OK;
}

int slos_plan_replay(slos_plan_t p, void *stream)
{
    int rc = check_plan(p);
    if (rc) return rc;
    if (!p->graph) return fail(SLOS_ERR_INVALID_ARG, "no captured graph: call slos_plan_capture first");
    const hipError_t e = hipGraphLaunch(p->graph, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    return SLOS_OK;
}

int slos_cdf(slos_plan_t p, const void *probs, void *stream)
{
    int rc = check_plan(p);
    if (rc) return rc;
    if (!probs) return fail(SLOS_ERR_INVALID_ARG, "probs is NULL");
    if ((uintptr_t)probs % 16) return fail(SLOS_ERR_INVALID_ARG, "probs must be 16-byte aligned");
    int e = slos_launch_cdf(probs, p->c64 ? 1 : 0, (int64_t)p->Nk[p->n], p->d_cdf, stream);
    if (e) return hip_fail((hipError_t)e, "cumulative probability kernels");
    return SLOS_OK;
}

int slos_marginals(slos_plan_t p, const void *probs, double *pk, void *stream)
{
    int rc = check_plan(p);
    if (rc) return rc;
    if (!probs || !pk) return fail(SLOS_ERR_INVALID_ARG, "probs and pk must be device pointers");
    int e = slos_launch_marginals(probs, p->c64 ? 1 : 0, p->d_cdf, p->d_pk_ends, p->m, pk, stream);
    if (e) return hip_fail((hipError_t)e, "marginal kernel");
    return SLOS_OK;
}

int slos_postselect(slos_plan_t p, const void *probs, const int32_t *group_of_mode, int ngroups,
                    const int32_t *count_min, const int32_t *count_max, double *kept_sum, void *masked,
                    const int64_t *ranks, int64_t nranks, double *table, void *stream)
{
    int rc = check_plan(p);
    if (rc) return rc;
    if (!probs || !kept_sum) return fail(SLOS_ERR_INVALID_ARG, "probs and kept_sum must be device pointers");
    if (ngroups < 0 || ngroups > SLOS_PS_MAX_GROUPS)
        return fail(SLOS_ERR_INVALID_ARG, "ngroups = %d outside [0, %d]", ngroups, SLOS_PS_MAX_GROUPS);
    if (ngroups > 0 && (!group_of_mode || !count_min || !count_max))
        return fail(SLOS_ERR_INVALID_ARG, "groups need group_of_mode, count_min and count_max");
    if (nranks < 0 || (nranks > 0 && (!ranks || !table)))
        return fail(SLOS_ERR_INVALID_ARG, "nranks must be >= 0, with ranks and table when > 0");
    PostselectParams ps{};
    ps.P = probs;
    ps.masked = masked;
    ps.M = (int64_t)p->Nk[p->n];
    ps.binom = p->d_binom;
    ps.bstride = p->B.stride;
    ps.m = p->m;
    ps.n = p->n;
    ps.ngroups = ngroups;
    for (int j = 0; j < p->m; ++j) {
        const int g = group_of_mode ? group_of_mode[j] : -1;
        if (g < -1 || g >= ngroups)
            return fail(SLOS_ERR_INVALID_ARG, "group_of_mode[%d] = %d outside [-1, ngroups)", j, g);
        ps.group[j] = (int8_t)g;
    }
    for (int g = 0; g < ngroups; ++g) {
        if (count_min[g] < 0 || count_max[g] > 255 || count_min[g] > count_max[g])
            return fail(SLOS_ERR_INVALID_ARG, "group %d: need 0 <= count_min <= count_max <= 255", g);
        ps.cmin[g] = (uint8_t)count_min[g];
        ps.cmax[g] = (uint8_t)count_max[g];
    }
    const uint64_t M = (uint64_t)ps.M;
    const uint64_t threads = std::min<uint64_t>((M + 63) / 64, (uint64_t)SLOS_PS_MAX_WAVES * 64);
    ps.run = (M + threads - 1) / threads;
    ps.partials = p->d_ps_partials;
    if (p->n > 0) {
        ps.leaves = p->d_leaves + p->ps_leaf_off;
        ps.nleaves = p->ps_leaves.size();
        ps.type_off = p->d_ps_type_off;
        ps.types = p->d_ps_types;
        ps.ntypes = p->ps_ntypes;
        ps.entries = p->ps_entries;
        ps.low = p->d_ps_low;
    }
    int e = slos_launch_postselect(ps, p->c64 ? 1 : 0, stream);
    if (e) return hip_fail((hipError_t)e, "post-selection kernel");
    const uint64_t waves = ps.nleaves > 0 ? (uint64_t)SLOS_PS_MAX_WAVES : (((M + ps.run - 1) / ps.run + 255) / 256) * 4;
    e = slos_launch_reduce(p->d_ps_partials, (int64_t)waves, p->d_ps_partials + SLOS_PS_MAX_WAVES, kept_sum,
                           stream);
    if (e) return hip_fail((hipError_t)e, "post-selection sum");
    if (nranks > 0) {
        e = slos_launch_postselect_table(ps, p->c64 ? 1 : 0, ranks, nranks, kept_sum, table, stream);
        if (e) return hip_fail((hipError_t)e, "post-selection table kernel");
    }
    return SLOS_OK;
}

// The sub-lattice of one occupation multiset (occupations descending): its
// states in mixed radix, listed layer by layer, each with the mask of its
// non-zero digits; appended to the plan's pools.
static uint32_t select_pattern(slos_plan_s *p, const std::vector<uint8_t> &key, uint32_t R)
{
    auto it = p->sel_pat_of.find(key);
    if (it != p->sel_pat_of.end()) return it->second;
    const int n = p->n;
    SelectPattern pt{};
    pt.R = R;
    pt.nocc = (uint32_t)key.size();
    pt.off = (uint32_t)p->sel_state.size();
    uint32_t st = 1;
    for (size_t q = 0; q < key.size(); ++q) {
        pt.stride[q] = st;
        st *= (uint32_t)key[q] + 1u;
    }
    std::vector<uint8_t> layer(R);
    std::vector<uint32_t> msk(R), cnt(n + 2, 0);
    std::vector<uint32_t> digit(key.size(), 0);  // digits of x, counted up in mixed radix
    for (uint32_t x = 0; x < R; ++x) {
        uint32_t k = 0, mk = 0;
        for (size_t q = 0; q < key.size(); ++q) {
            k += digit[q];
            if (digit[q]) mk |= 1u << q;
        }
        layer[x] = (uint8_t)k;
        msk[x] = mk;
        ++cnt[k];
        for (size_t q = 0; q < key.size(); ++q) {  // x + 1
            if (++digit[q] <= key[q]) break;
            digit[q] = 0;
        }
    }
    uint32_t run = 0;
    for (int k = 0; k <= n; ++k) {
        pt.lstart[k] = run;
        run += cnt[k];
        cnt[k] = pt.lstart[k];
    }
    pt.lstart[n + 1] = run;
    p->sel_state.resize(p->sel_state.size() + R);
    p->sel_mask.resize(p->sel_mask.size() + R);
    for (uint32_t x = 0; x < R; ++x) {
        const uint32_t pos = pt.off + cnt[layer[x]]++;
        p->sel_state[pos] = (uint16_t)x;
        p->sel_mask[pos] = msk[x];
    }
    const uint32_t pi = (uint32_t)p->sel_pats.size();
    p->sel_pats.push_back(pt);
    p->sel_pat_of.emplace(key, pi);
    return pi;
}

int slos_select(slos_plan_t p, const void *U, const int32_t *targets, int64_t count, void *out, void *stream)
{
    int rc = check_plan(p);
    if (rc) return rc;
    if (count < 0) return fail(SLOS_ERR_INVALID_ARG, "count = %lld is negative", (long long)count);
    if (count == 0) return SLOS_OK;
    if (!U || !targets || !out) return fail(SLOS_ERR_INVALID_ARG, "U, targets and out must not be NULL");
    const int m = p->m, n = p->n;
    const size_t es = p->elem();
    // largest sub-lattice whose amplitudes fit a workgroup's LDS
    const uint64_t r_cap = SLOS_LDS_DYNAMIC_MAX / es;
    if ((size_t)count > p->sel_cap) {
        if (p->d_sel) (void)hipFree(p->d_sel);
        if (p->h_sel) (void)hipHostFree(p->h_sel);
        p->d_sel = nullptr;
        p->h_sel = nullptr;
        p->sel_cap = 0;
        if ((rc = alloc_dev((void **)&p->d_sel, (size_t)count * sizeof(SelectTarget), "target descriptors")))
            return rc;
        hipError_t he = hipHostMalloc((void **)&p->h_sel, (size_t)count * sizeof(SelectTarget), hipHostMallocDefault);
        if (he != hipSuccess) {
            p->h_sel = nullptr;
            return hip_fail(he, "pinned staging of the target descriptors");
        }
        p->sel_cap = (size_t)count;
    }
    // Targets are prepared in parallel (host threads over contiguous ranges):
    // occupied modes in canonical order, the normalisation, and the multiset of
    // occupations as a 64-bit key (the occupations in descending order, each
    // written as that many one bits and a zero: at most n + 32 bits).  Patterns
    // are then assigned in one serial pass over the keys.
    std::vector<uint64_t> keys;
    std::vector<uint32_t> rs;
    try {
        p->sel_build.resize((size_t)count);
        keys.resize((size_t)count);
        rs.resize((size_t)count);
    } catch (std::bad_alloc &) {
        return fail(SLOS_ERR_OOM, "host allocation of %lld target descriptors failed", (long long)count);
    }
    std::vector<int64_t> bad_at(1, -1);
    std::vector<int> bad_kind(1, 0);
    auto prepare = [&](int64_t lo, int64_t hi, int64_t &bad, int &kind) {
        int occ_n[SLOS_SELECT_MAX_OCC], occ_j[SLOS_SELECT_MAX_OCC];
        for (int64_t i = lo; i < hi; ++i) {
            const int32_t *s = targets + (size_t)i * m;
            int tot = 0, nocc = 0;
            double f = 1.0;
            uint64_t R = 1;
            for (int j = 0; j < m; ++j) {
                const int v = s[j];
                if (v == 0) continue;
                if (v < 0 || tot + v > n) {
                    tot = v < 0 ? -1 : n + 1;
                    break;
                }
                tot += v;
                int q = nocc++;  // insert: occupation descending, then mode ascending
                while (q > 0 && occ_n[q - 1] < v) {
                    occ_n[q] = occ_n[q - 1];
                    occ_j[q] = occ_j[q - 1];
                    --q;
                }
                occ_n[q] = v;
                occ_j[q] = j;
                R *= (uint64_t)v + 1;
                for (int w = 2; w <= v; ++w) f *= w;
                if (R > r_cap) break;
            }
            if (tot != n || R > r_cap) {
                bad = i;
                kind = tot < 0 ? 1 : (R > r_cap ? 2 : 3);
                return;
            }
            uint64_t key = 0;
            for (int q = 0; q < nocc; ++q) key = (key << (occ_n[q] + 1)) | (((1ull << occ_n[q]) - 1) << 1);
            keys[(size_t)i] = key;
            rs[(size_t)i] = (uint32_t)R;
            SelectTarget &t = p->sel_build[(size_t)i];
            t = SelectTarget{};
            t.nocc = (uint32_t)nocc;
            for (int q = 0; q < nocc; ++q) t.mode[q] = (uint8_t)occ_j[q];
            t.fac = std::sqrt(f) * p->norm_t;
        }
    };
    const int nth = count >= 4096 ? (int)std::min<unsigned>(8u, std::max(1u, std::thread::hardware_concurrency())) : 1;
    bad_at.assign(nth, -1);
    bad_kind.assign(nth, 0);
    if (nth == 1) {
        prepare(0, count, bad_at[0], bad_kind[0]);
    } else {
        std::vector<std::thread> pool;
        try {
            for (int w = 0; w < nth; ++w)
                pool.emplace_back(prepare, count * w / nth, count * (w + 1) / nth, std::ref(bad_at[w]),
                                  std::ref(bad_kind[w]));
        } catch (...) {
            for (auto &th : pool) th.join();
            return fail(SLOS_ERR_OOM, "could not start the host threads that prepare the targets");
        }
        for (auto &th : pool) th.join();
    }
    for (int w = 0; w < nth; ++w) {
        if (bad_at[w] < 0) continue;
        const long long i = (long long)bad_at[w];
        if (bad_kind[w] == 1) return fail(SLOS_ERR_INVALID_ARG, "target %lld has a negative occupation", i);
        if (bad_kind[w] == 2)
            return fail(SLOS_ERR_INVALID_ARG, "target %lld: prod(s_j + 1) exceeds %llu states (one workgroup's LDS)",
                        i, (unsigned long long)r_cap);
        return fail(SLOS_ERR_INVALID_ARG, "target %lld does not hold n = %d photons", i, n);
    }
    uint32_t r_max = 1;
    try {
        std::vector<uint8_t> mult;
        for (int64_t i = 0; i < count; ++i) {
            auto it = p->sel_key.find(keys[(size_t)i]);
            uint32_t pi;
            if (it != p->sel_key.end()) {
                pi = it->second;
            } else {
                mult.clear();  // decode the key: runs of ones, most significant first
                const SelectTarget &t = p->sel_build[(size_t)i];
                const int32_t *s = targets + (size_t)i * m;
                for (uint32_t q = 0; q < t.nocc; ++q) mult.push_back((uint8_t)s[t.mode[q]]);
                pi = select_pattern(p, mult, rs[(size_t)i]);
                p->sel_key.emplace(keys[(size_t)i], pi);
            }
            p->sel_build[(size_t)i].pattern = pi;
            r_max = std::max(r_max, rs[(size_t)i]);
        }
    } catch (std::bad_alloc &) {
        return fail(SLOS_ERR_OOM, "host allocation of the sub-lattice tables failed");
    }
    // tables: patterns, then the state pool (2-byte entries, padded to 16
    // bytes), then the masks; uploaded again only when this call added patterns
    const size_t npat = p->sel_pats.size();
    const size_t pat_bytes = npat * sizeof(SelectPattern);
    const size_t st_bytes = (p->sel_state.size() * sizeof(uint16_t) + 15) / 16 * 16;
    const size_t tab_bytes = pat_bytes + st_bytes + p->sel_mask.size() * sizeof(uint32_t);
    if (npat != p->sel_uploaded) {
        if (tab_bytes > p->sel_tab_cap) {
            if (p->d_sel_tab) (void)hipFree(p->d_sel_tab);
            p->d_sel_tab = nullptr;
            p->sel_tab_cap = 0;
            if ((rc = alloc_dev((void **)&p->d_sel_tab, 2 * tab_bytes, "sub-lattice tables"))) return rc;
            p->sel_tab_cap = 2 * tab_bytes;
        }
        hipError_t e = hipMemcpy(p->d_sel_tab, p->sel_pats.data(), pat_bytes, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(p->d_sel_tab + pat_bytes, p->sel_state.data(), p->sel_state.size() * sizeof(uint16_t),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(p->d_sel_tab + pat_bytes + st_bytes, p->sel_mask.data(),
                          p->sel_mask.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "sub-lattice table upload");
        p->sel_uploaded = npat;
        p->sel_st_bytes = st_bytes;
    }
    std::memcpy(p->h_sel, p->sel_build.data(), (size_t)count * sizeof(SelectTarget));
    hipError_t e = hipMemcpyAsync(p->d_sel, p->h_sel, (size_t)count * sizeof(SelectTarget), hipMemcpyHostToDevice,
                                  (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "target upload");
    SelectParams sp{};
    sp.U = U;
    sp.targets = p->d_sel;
    sp.patterns = (const SelectPattern *)p->d_sel_tab;
    sp.state = (const uint16_t *)(p->d_sel_tab + pat_bytes);
    sp.mask = (const uint32_t *)(p->d_sel_tab + pat_bytes + p->sel_st_bytes);
    sp.count = count;
    sp.out = out;
    sp.r_max = r_max;
    sp.m = m;
    sp.n = n;
    for (int k = 0; k < n; ++k) sp.cols[k] = (uint8_t)p->photons[k];
    int ke = slos_launch_select(sp, p->c64 ? 1 : 0, stream);
    if (ke) return hip_fail((hipError_t)ke, "selected-output kernel");
    e = hipStreamSynchronize((hipStream_t)stream);  // the staging buffer is reused by the next call
    if (e != hipSuccess) return hip_fail(e, "selected-output synchronisation");
    return SLOS_OK;
}

int slos_sample(slos_plan_t p, const void *probs, const double *r, int64_t count, int64_t *ranks, void *stream)
{
    int rc = check_plan(p);
    if (rc) return rc;
    if (count < 0) return fail(SLOS_ERR_INVALID_ARG, "count = %lld is negative", (long long)count);
    if (count == 0) return SLOS_OK;
    if (!probs || !r || !ranks) return fail(SLOS_ERR_INVALID_ARG, "probs, r and ranks must be device pointers");
    int e = slos_launch_sample(probs, p->c64 ? 1 : 0, (int64_t)p->Nk[p->n], p->d_cdf, r, count, ranks, stream);
    if (e) return hip_fail((hipError_t)e, "sampling kernel");
    return SLOS_OK;
}

} // extern "C"

// ---- batches ----------------------------------------------------------------------

struct slos_batch_s {
    int count = 0;
    bool c64 = true;
    slos_options_t opts{};
    slos_plan_s builder;                 // shared binomials, leaves and inner tables
    std::vector<BatchInst> inst;
    std::vector<int64_t> out_off, u_off; // count + 1 each
    std::vector<LeafDescNarrow> desc;
    std::vector<uint32_t> wg_start, wg_list;   // cooperative instances per workgroup
    std::vector<uint32_t> wv_start, wv_list;   // small instances per wave slot
    std::vector<uint64_t> wg_scr;              // per workgroup: its cooperative scratch pair
    uint64_t scratch_stride = 0;         // elements per cooperative scratch buffer
    uint64_t small_base = 0, small_stride = 0;
    uint64_t scratch_elems = 0;
    uint32_t lds_wave_bytes = 0;
    int grid = 0;
    // device
    BatchInst *d_inst = nullptr;
    uint32_t *d_wg_start = nullptr, *d_wg_list = nullptr;
    uint32_t *d_wv_start = nullptr, *d_wv_list = nullptr;
    uint64_t *d_wg_scr = nullptr;
    LeafDescNarrow *d_desc = nullptr;
    uint32_t *d_pred = nullptr;
    double *d_lowfac = nullptr;
    void *d_scratch = nullptr;
    void *d_vac = nullptr;
    hipGraphExec_t exec = nullptr;

    void free_device()
    {
        auto f = [](void *q) {
            if (q) (void)hipFree(q);
        };
        f(d_inst);
        f(d_wg_start);
        f(d_wg_list);
        f(d_wv_start);
        f(d_wv_list);
        f(d_wg_scr);
        f(d_desc);
        f(d_pred);
        f(d_lowfac);
        f(d_scratch);
        f(d_vac);
        if (exec) (void)hipGraphExecDestroy(exec);
        d_inst = nullptr;
        d_wg_start = d_wg_list = nullptr;
        d_wv_start = d_wv_list = nullptr;
        d_wg_scr = nullptr;
        d_desc = nullptr;
        d_pred = nullptr;
        d_lowfac = nullptr;
        d_scratch = d_vac = nullptr;
        exec = nullptr;
    }

    BatchParams params(const void *U, void *out, double *sum_p) const
    {
        BatchParams bp{};
        bp.U = U;
        bp.out = out;
        bp.sum_p = sum_p;
        bp.inst = d_inst;
        bp.wg_start = d_wg_start;
        bp.wg_list = d_wg_list;
        bp.wv_start = d_wv_start;
        bp.wv_list = d_wv_list;
        bp.wg_scr = d_wg_scr;
        bp.small_base = small_base;
        bp.small_stride = small_stride;
        bp.desc = d_desc;
        bp.pred = d_pred;
        bp.lowfac = d_lowfac;
        bp.scratch = d_scratch;
        bp.scratch_stride = scratch_stride;
        bp.vac = d_vac;
        bp.lds_wave_bytes = lds_wave_bytes;
        return bp;
    }
};

extern "C" {

int slos_batch_plan(int count, const int32_t *ms, const int32_t *inputs, int flags, const slos_options_t *opts,
                    slos_batch_t *out)
{
    if (!out) return fail(SLOS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (count < 1 || !ms || !inputs) return fail(SLOS_ERR_INVALID_ARG, "need count >= 1, ms and inputs");
    if (flags & ~(SLOS_C64 | SLOS_C128))
        return fail(SLOS_ERR_INVALID_ARG, "batch flags take SLOS_C64 or SLOS_C128 only");
    const int dt = flags & (SLOS_C64 | SLOS_C128);
    if (dt != SLOS_C64 && dt != SLOS_C128)
        return fail(SLOS_ERR_DTYPE, "flags must hold exactly one of SLOS_C64, SLOS_C128");
    slos_options_t o{};
    if (opts) o = *opts;
    if (o.leaf_max == 0) o.leaf_max = 1024;
    if (o.block_threads == 0) o.block_threads = 256;
    if (o.grid_blocks == 0) o.grid_blocks = 1024;
    if (o.outputs_per_lane == 0) o.outputs_per_lane = 2;
    if (o.leaf_max < 1 || o.leaf_max > 65536 ||
        (o.block_threads != 64 && o.block_threads != 128 && o.block_threads != 256 && o.block_threads != 512 &&
         o.block_threads != 1024) ||
        o.grid_blocks < 1 || o.grid_blocks > (1 << 20) ||
        (o.outputs_per_lane != 1 && o.outputs_per_lane != 2 && o.outputs_per_lane != 4) || o.low_block_max < -1)
        return fail(SLOS_ERR_INVALID_ARG, "invalid batch options");

    int maxm = 0, maxn = 0;
    int64_t pos = 0;
    for (int i = 0; i < count; ++i) {
        const int m = ms[i];
        if (m < 1 || m > SLOS_MAX_MODES) return fail(SLOS_ERR_INVALID_ARG, "instance %d: m = %d", i, m);
        long tot = 0;
        for (int j = 0; j < m; ++j) {
            if (inputs[pos + j] < 0) return fail(SLOS_ERR_INVALID_ARG, "instance %d: negative occupation", i);
            tot += inputs[pos + j];
        }
        if (tot > SLOS_BATCH_MAX_N)
            return fail(SLOS_ERR_INVALID_ARG, "instance %d: %ld photons, batches take at most %d", i, tot,
                        SLOS_BATCH_MAX_N);
        maxm = std::max(maxm, m);
        maxn = std::max(maxn, (int)tot);
        pos += m;
    }

    slos_batch_s *b = new (std::nothrow) slos_batch_s;
    if (!b) return fail(SLOS_ERR_OOM, "host allocation of the batch failed");
    b->count = count;
    b->c64 = dt == SLOS_C64;
    b->opts = o;
    const size_t es = b->c64 ? 8 : 16;
    try {
        slos_plan_s &P = b->builder;
        P.opts = o;
        if (o.low_block_max > 0) P.low_cap = (uint64_t)o.low_block_max;  // default: no cap
        P.B.build(maxm + maxn, maxn);
        b->inst.resize(count);
        b->out_off.assign(count + 1, 0);
        b->u_off.assign(count + 1, 0);
        uint32_t low_max = 0;
        std::map<std::tuple<int, int, double>, std::pair<uint32_t, uint32_t>> shared;  // descriptor sets
        std::vector<double> cost(count);
        std::vector<uint64_t> inter(count, 0), last(count, 1);  // largest layer below n, layer n
        pos = 0;
        for (int i = 0; i < count; ++i) {
            const int m = ms[i];
            BatchInst &I = b->inst[i];
            I = BatchInst{};
            I.m = (uint32_t)m;
            std::vector<int> photons;
            double tf = 1.0;
            for (int j = 0; j < m; ++j) {
                for (int c = 0; c < inputs[pos + j]; ++c) photons.push_back(j);
                for (int v = 2; v <= inputs[pos + j]; ++v) tf *= v;
            }
            const int n = (int)photons.size();
            I.n = (uint32_t)n;
            P.norm_t = 1.0 / std::sqrt(tf);
            uint64_t M = P.B(m + n - 1, n);
            b->u_off[i + 1] = b->u_off[i] + (int64_t)m * m;
            b->out_off[i + 1] = b->out_off[i] + (int64_t)M;
            I.U_off = (uint64_t)b->u_off[i];
            I.out_off = (uint64_t)b->out_off[i];
            double c = 0.0;
            for (int k = 1; k <= n; ++k) {
                I.col[k - 1] = (uint8_t)photons[k - 1];
                // A layer's descriptors depend on (m, k) only, except the last
                // layer's normalisation, which also takes 1/sqrt(prod t!):
                // instances that agree on those share one descriptor set.
                const auto key = std::make_tuple(m, k, k == n ? P.norm_t : -1.0);
                const auto hit = shared.find(key);
                if (hit != shared.end()) {
                    I.desc_off[k - 1] = hit->second.first;
                    I.nleaves[k - 1] = hit->second.second;
                }
                std::vector<LeafRec> lv;
                std::vector<uint8_t> hm;
                if (hit == shared.end()) {
                    P.gen_leaves(k, m - 1, k, (uint64_t)o.leaf_max, hm, lv);
                    I.desc_off[k - 1] = (uint32_t)b->desc.size();
                    I.nleaves[k - 1] = (uint32_t)lv.size();
                    shared[key] = {I.desc_off[k - 1], I.nleaves[k - 1]};
                }
                std::vector<uint64_t> deltas;
                std::vector<uint8_t> modes;
                for (const LeafRec &L : lv) {
                    LeafDescHead h;
                    P.describe(k, L, h, deltas, modes);
                    if (h.nh > SLOS_NARROW_GROUPS) throw std::pair<int, std::string>(SLOS_ERR_INVALID_ARG, "too many groups");
                    LeafDescNarrow w{};
                    w.h = h;
                    for (size_t g = 0; g < deltas.size(); ++g) {
                        w.delta[g] = (uint32_t)deltas[g];
                        w.mode[g] = modes[g];
                    }
                    b->desc.push_back(w);
                    low_max = std::max(low_max, h.low_size);
                }
                const uint64_t Nk = P.B(m + k - 1, k);
                if (k < n) inter[i] = std::max(inter[i], Nk);
                else last[i] = Nk;
                c += (double)(P.B(m + k - 2, k - 1) + Nk);
            }
            cost[i] = c + 64.0 * n;
            pos += m;
        }
        // Instances whose last layer has at least four tiles per wave run
        // cooperatively on a workgroup; the rest run on single waves.  Both
        // lists are filled largest first, each instance to the least loaded
        // workgroup (load in wave time: cost / W) or wave slot (whose load
        // starts at its workgroup's cooperative load).
        const int G = std::min(o.grid_blocks, count);
        const int W = o.block_threads / 64;
        const uint64_t coop_min = 4ull * (uint64_t)W * 64u * (uint64_t)o.outputs_per_lane;
        std::vector<int> order(count);
        for (int i = 0; i < count; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
        std::vector<double> load(G, 0.0);
        std::vector<std::vector<uint32_t>> lists(G), wlists((size_t)G * W);
        uint64_t coop_inter = 0, small_inter = 0;
        typedef std::pair<double, uint32_t> Slot;
        std::vector<int> small;
        for (int i : order) {
            if (W > 1 && last[i] >= coop_min) {
                int g = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                load[g] += cost[i] / W;
                lists[g].push_back((uint32_t)i);
                coop_inter = std::max(coop_inter, inter[i]);
            } else {
                small.push_back(i);
                small_inter = std::max(small_inter, inter[i]);
            }
        }
        std::priority_queue<Slot, std::vector<Slot>, std::greater<Slot>> heap;
        for (int g = 0; g < G; ++g)
            for (int w = 0; w < W; ++w) heap.push(Slot(load[g], (uint32_t)(g * W + w)));
        for (int i : small) {
            Slot sl = heap.top();
            heap.pop();
            wlists[sl.second].push_back((uint32_t)i);
            sl.first += cost[i];
            heap.push(sl);
        }
        b->grid = G;
        b->wg_start.assign(G + 1, 0);
        for (int g = 0; g < G; ++g) {
            b->wg_start[g + 1] = b->wg_start[g] + (uint32_t)lists[g].size();
            b->wg_list.insert(b->wg_list.end(), lists[g].begin(), lists[g].end());
        }
        b->wv_start.assign((size_t)G * W + 1, 0);
        for (size_t sl = 0; sl < (size_t)G * W; ++sl) {
            b->wv_start[sl + 1] = b->wv_start[sl] + (uint32_t)wlists[sl].size();
            b->wv_list.insert(b->wv_list.end(), wlists[sl].begin(), wlists[sl].end());
        }
        // scratch: a cooperative pair for each workgroup that has cooperative
        // instances, then a small pair for every wave slot
        const uint64_t slack = (SLOS_BUFFER_SLACK + es - 1) / es;
        b->scratch_stride = std::max<uint64_t>(coop_inter, 1) + slack;
        b->small_stride = std::max<uint64_t>(small_inter, 1) + slack;
        b->wg_scr.assign(G, 0);
        uint64_t pos_scr = 0;
        for (int g = 0; g < G; ++g)
            if (!lists[g].empty()) {
                b->wg_scr[g] = pos_scr;
                pos_scr += 2 * b->scratch_stride;
            }
        b->small_base = pos_scr;
        b->scratch_elems = pos_scr + (uint64_t)G * W * 2 * b->small_stride;
        b->lds_wave_bytes = slos_lds_wave_bytes(low_max, (uint32_t)es);
        if ((b->lds_wave_bytes + 256 * es) * (size_t)W > SLOS_LDS_DYNAMIC_MAX)
            throw std::pair<int, std::string>(SLOS_ERR_INVALID_ARG, "leaf_max too large for the LDS of a workgroup");
        if (P.pred.size() >= (size_t(1) << 32) || b->desc.size() >= (size_t(1) << 32))
            throw std::pair<int, std::string>(SLOS_ERR_SIZE_OVERFLOW, "batch tables too large");
    } catch (std::bad_alloc &) {
        delete b;
        return fail(SLOS_ERR_OOM, "host allocation failed while building the batch");
    } catch (std::pair<int, std::string> &e) {
        delete b;
        return fail(e.first, "%s", e.second.c_str());
    }

    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev < 1) {
        delete b;
        return fail(SLOS_ERR_NO_DEVICE, "no HIP device (%s)", hipGetErrorString(e));
    }
    int rc;
    double one_d[2] = {1.0, 0.0};
    float one_f[2] = {1.0f, 0.0f};
    if ((rc = dev_upload(&b->d_inst, b->inst.data(), b->inst.size(), "batch instances")) ||
        (rc = dev_upload(&b->d_wg_start, b->wg_start.data(), b->wg_start.size(), "batch schedule")) ||
        (rc = dev_upload(&b->d_wg_list, b->wg_list.data(), b->wg_list.size(), "batch schedule")) ||
        (rc = dev_upload(&b->d_wv_start, b->wv_start.data(), b->wv_start.size(), "batch schedule")) ||
        (rc = dev_upload(&b->d_wv_list, b->wv_list.data(), b->wv_list.size(), "batch schedule")) ||
        (rc = dev_upload(&b->d_wg_scr, b->wg_scr.data(), b->wg_scr.size(), "batch schedule")) ||
        (rc = dev_upload(&b->d_desc, b->desc.data(), b->desc.size(), "batch descriptors")) ||
        (rc = dev_upload(&b->d_pred, b->builder.pred.data(), b->builder.pred.size(), "batch inner tables")) ||
        (rc = dev_upload(&b->d_lowfac, b->builder.lowfac.data(), b->builder.lowfac.size(), "batch factorials")) ||
        (rc = alloc_dev(&b->d_scratch, (size_t)b->scratch_elems * es + SLOS_BUFFER_SLACK, "batch scratch")) ||
        (rc = alloc_dev(&b->d_vac, es + SLOS_BUFFER_SLACK, "vacuum layer"))) {
        b->free_device();
        delete b;
        return rc;
    }
    if ((e = hipMemcpy(b->d_vac, b->c64 ? (const void *)one_f : (const void *)one_d, es, hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = (hipError_t)slos_prepare_batch_kernels()) != hipSuccess) {
        rc = hip_fail(e, "batch set-up");
        b->free_device();
        delete b;
        return rc;
    }
    *out = b;
    return SLOS_OK;
}

void slos_batch_destroy(slos_batch_t b)
{
    if (!b) return;
    (void)hipDeviceSynchronize();
    b->free_device();
    delete b;
}

int slos_batch_offsets(slos_batch_t b, int64_t *u_offsets, int64_t *out_offsets)
{
    if (!b) return fail(SLOS_ERR_INVALID_ARG, "batch is NULL");
    for (int i = 0; i <= b->count; ++i) {
        if (u_offsets) u_offsets[i] = b->u_off[i];
        if (out_offsets) out_offsets[i] = b->out_off[i];
    }
    return SLOS_OK;
}

int slos_batch_amplitudes(slos_batch_t b, const void *U, void *out, double *sum_p, void *stream)
{
    if (!b) return fail(SLOS_ERR_INVALID_ARG, "batch is NULL");
    if (!U || !out) return fail(SLOS_ERR_INVALID_ARG, "U and out must be device pointers");
    const BatchParams bp = b->params(U, out, sum_p);
    int e = slos_launch_batch(bp, b->c64, b->opts.outputs_per_lane, b->opts.block_threads, b->grid, stream);
    if (e) return hip_fail((hipError_t)e, "batch kernel");
    return SLOS_OK;
}

int slos_batch_capture(slos_batch_t b, const void *U, void *out, double *sum_p)
{
    if (!b) return fail(SLOS_ERR_INVALID_ARG, "batch is NULL");
    if (!U || !out) return fail(SLOS_ERR_INVALID_ARG, "U and out must be device pointers");
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    hipStream_t s;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "capture stream");
    hipGraph_t g = nullptr;
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const BatchParams bp = b->params(U, out, sum_p);
        int le = slos_launch_batch(bp, b->c64, b->opts.outputs_per_lane, b->opts.block_threads, b->grid, s);
        hipError_t ee = hipStreamEndCapture(s, &g);
        e = le ? (hipError_t)le : ee;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(s);
    if (e != hipSuccess) {
        b->exec = nullptr;
        return hip_fail(e, "graph capture of the batch");
    }
    return SLOS_OK;
}

int slos_batch_replay(slos_batch_t b, void *stream)
{
    if (!b) return fail(SLOS_ERR_INVALID_ARG, "batch is NULL");
    if (!b->exec) return fail(SLOS_ERR_INVALID_ARG, "no captured graph: call slos_batch_capture first");
    hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    return SLOS_OK;
}

} // extern "C"

// ---- imperfect-source mixtures ------------------------------------------------------

struct slos_source_s {
    int m = 0, n = 0, nmax = 0;
    double p0 = 0.0, p1 = 1.0, p2 = 0.0, x = 1.0;
    std::vector<int> modes;         // input mode of source b (ascending)
    std::vector<uint64_t> off;      // first state of photon number k, k = 0..nmax+1
    uint64_t G = 0;
    uint64_t nleaves = 0;
    std::vector<uint64_t> leaves_upto;  // leaves of photon numbers 1..k, k = 0..nmax
    std::vector<int64_t> amp_off;   // per subset: its common group's vector in d_amp, or -1
    std::vector<uint32_t> sub_off;  // subsets of size a: sub_masks[sub_off[a] .. sub_off[a+1])
    std::vector<uint32_t> sub_masks;
    std::vector<double> inv_tfac;   // per subset: 1 / prod_i t_i! of its common group
    int64_t namp = 0;
    slos_plan_s builder;            // binomials, leaves and inner tables of photon numbers 1..nmax
    // device
    LeafDescNarrow *d_desc = nullptr;
    uint32_t *d_pred = nullptr;
    uint64_t *d_off = nullptr;
    int64_t *d_amp_off = nullptr;
    uint32_t *d_sub = nullptr;
    double *d_inv_tfac = nullptr;
    double *d_lowfac = nullptr;
    uint64_t *d_binom = nullptr;
    void *d_amp = nullptr;
    double *d_slots = nullptr;      // 2^n graded vectors
    double *d_temp = nullptr;       // 2^(n-1) graded vectors (at least one)
    double *d_part = nullptr;
    double *d_res = nullptr;

    void free_device()
    {
        auto f = [](void *q) {
            if (q) (void)hipFree(q);
        };
        f(d_desc);
        f(d_pred);
        f(d_off);
        f(d_amp_off);
        f(d_sub);
        f(d_inv_tfac);
        f(d_lowfac);
        f(d_binom);
        f(d_amp);
        f(d_slots);
        f(d_temp);
        f(d_part);
        f(d_res);
        d_desc = nullptr;
        d_pred = nullptr;
        d_off = nullptr;
        d_amp_off = nullptr;
        d_sub = nullptr;
        d_inv_tfac = nullptr;
        d_lowfac = nullptr;
        d_binom = nullptr;
        d_amp = nullptr;
        d_slots = d_temp = d_part = d_res = nullptr;
    }
};

extern "C" {

int slos_source_plan(int m, const int32_t *input_state, const slos_source_params_t *src, int nmax,
                     const slos_options_t *opts, slos_source_t *out)
{
    if (!out) return fail(SLOS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (m < 1 || m > SLOS_MAX_MODES) return fail(SLOS_ERR_INVALID_ARG, "m = %d outside [1, %d]", m, SLOS_MAX_MODES);
    if (!input_state) return fail(SLOS_ERR_INVALID_ARG, "input_state is NULL");
    long n = 0;
    for (int j = 0; j < m; ++j) {
        if (input_state[j] < 0) return fail(SLOS_ERR_INVALID_ARG, "input_state[%d] = %d is negative", j, input_state[j]);
        n += input_state[j];
    }
    if (n > SLOS_SRC_MAX_SOURCES)
        return fail(SLOS_ERR_INVALID_ARG, "%ld photons: at most %d sources", n, SLOS_SRC_MAX_SOURCES);
    slos_source_params_t sp{1.0, 0.0, 1.0};
    if (src) sp = *src;
    const double beta = sp.emission_probability, g2 = sp.multiphoton_component, V = sp.indistinguishability;
    if (!(beta > 0.0 && beta <= 1.0)) return fail(SLOS_ERR_INVALID_ARG, "emission_probability %g outside (0, 1]", beta);
    if (!(g2 >= 0.0 && g2 <= 1.0)) return fail(SLOS_ERR_INVALID_ARG, "multiphoton_component %g outside [0, 1]", g2);
    if (beta * g2 > 0.5)
        return fail(SLOS_ERR_INVALID_ARG, "emission_probability x multiphoton_component = %g exceeds 1/2",
                    beta * g2);
    if (!(V >= 0.0 && V <= 1.0)) return fail(SLOS_ERR_INVALID_ARG, "indistinguishability %g outside [0, 1]", V);
    // p1 + p2 = beta, g2 = 2 p2 / (p1 + 2 p2)^2: the root of
    // g2 p2^2 - (1 - beta g2) p2 + beta^2 g2 / 2 = 0 that vanishes with g2,
    // written without the cancellation of 1 - beta g2 - sqrt(1 - 2 beta g2)
    const double disc = std::sqrt(1.0 - 2.0 * beta * g2);
    const double p2 = g2 > 0.0 ? beta * beta * g2 / ((1.0 - beta * g2) + disc) : 0.0;
    if (nmax < 0) nmax = (int)(p2 > 0.0 ? 2 * n : n);
    if (nmax > SLOS_SRC_MAX_NMAX)
        return fail(SLOS_ERR_INVALID_ARG, "nmax = %d above %d photons", nmax, SLOS_SRC_MAX_NMAX);
    if (nmax > 2 * n) return fail(SLOS_ERR_INVALID_ARG, "nmax = %d above 2n = %ld photons", nmax, 2 * n);

    slos_source_s *s = new (std::nothrow) slos_source_s;
    if (!s) return fail(SLOS_ERR_OOM, "host allocation of the source plan failed");
    s->m = m;
    s->n = (int)n;
    s->nmax = nmax;
    s->p2 = p2;
    s->p1 = beta - p2;
    s->p0 = 1.0 - beta;
    s->x = std::sqrt(V);
    std::vector<LeafDescNarrow> desc;
    std::vector<int32_t> ms, inputs;
    int rc = SLOS_OK;
    try {
        for (int j = 0; j < m; ++j)
            for (int c = 0; c < input_state[j]; ++c) s->modes.push_back(j);
        slos_plan_s &P = s->builder;
        P.m = m;
        P.norm_t = 1.0;
        P.B.build(m + nmax, nmax);
        s->off.assign(nmax + 2, 0);
        for (int k = 0; k <= nmax; ++k) {
            const uint64_t Nk = P.B(m + k - 1, k);
            if (Nk == kSat || s->off[k] + Nk < s->off[k])
                throw std::pair<int, std::string>(SLOS_ERR_SIZE_OVERFLOW, "state count overflows");
            s->off[k + 1] = s->off[k] + Nk;
        }
        s->G = s->off[nmax + 1];
        if (s->G >= (uint64_t(1) << 32))
            throw std::pair<int, std::string>(SLOS_ERR_SIZE_OVERFLOW, "more than 2^32 states up to nmax photons");
        const uint64_t cap = (opts && opts->leaf_max > 0) ? (uint64_t)opts->leaf_max : 256u;
        std::vector<uint64_t> deltas;
        std::vector<uint8_t> md;
        s->leaves_upto.assign(nmax + 1, 0);
        for (int k = 1; k <= nmax; ++k) {
            std::vector<LeafRec> lv;
            std::vector<uint8_t> hm;
            P.gen_leaves(k, m - 1, k, cap, hm, lv);
            for (const LeafRec &L : lv) {
                LeafDescHead h;
                P.describe(k, L, h, deltas, md);
                if (h.nh > SLOS_NARROW_GROUPS)
                    throw std::pair<int, std::string>(SLOS_ERR_INVALID_ARG, "too many occupied high modes");
                LeafDescNarrow w{};
                w.h = h;
                w.h.out_base += s->off[k];
                w.h.low_base += s->off[k - 1];
                w.h.pad = (uint32_t)k;
                for (size_t g = 0; g < deltas.size(); ++g) {
                    w.delta[g] = (uint32_t)deltas[g];
                    w.mode[g] = md[g];
                }
                desc.push_back(w);
            }
            s->leaves_upto[k] = desc.size();
        }
        s->nleaves = desc.size();
        if (P.pred.size() >= (size_t(1) << 32))
            throw std::pair<int, std::string>(SLOS_ERR_SIZE_OVERFLOW, "inner tables exceed 2^32 entries");
        // common groups: a compact vector per subset whose group fits in nmax photons
        const uint32_t nsub = 1u << n;
        s->amp_off.assign(nsub, -1);
        s->inv_tfac.assign(nsub, 1.0);
        s->sub_off.assign(n + 2, 0);
        int64_t pos = 0;
        for (int a = 0; a <= n; ++a) {
            s->sub_off[a] = (uint32_t)s->sub_masks.size();
            for (uint32_t A = 0; A < nsub; ++A) {
                if (__builtin_popcount(A) != a) continue;
                s->sub_masks.push_back(A);
                if (a > nmax) continue;
                s->amp_off[A] = pos;
                pos += (int64_t)(s->off[a + 1] - s->off[a]);
                std::vector<int> occ(m, 0);
                double tf = 1.0;
                for (int b = 0; b < n; ++b)
                    if (A >> b & 1u) tf *= (double)(++occ[s->modes[b]]);
                s->inv_tfac[A] = 1.0 / tf;
            }
        }
        s->sub_off[n + 1] = (uint32_t)s->sub_masks.size();
        s->namp = pos;
    } catch (std::bad_alloc &) {
        delete s;
        return fail(SLOS_ERR_OOM, "host allocation failed while building the source plan");
    } catch (std::pair<int, std::string> &e) {
        delete s;
        return fail(e.first, "%s", e.second.c_str());
    }
    const size_t G = (size_t)s->G;
    const size_t nslots = (size_t)1 << s->n, ntemp = std::max<size_t>(1, nslots / 2);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        delete s;
        return fail(SLOS_ERR_NO_DEVICE, "no HIP device");
    }
    if ((rc = dev_upload(&s->d_desc, desc.data(), desc.size(), "source leaf descriptors")) ||
        (rc = dev_upload(&s->d_lowfac, s->builder.lowfac.data(), s->builder.lowfac.size(), "source factorials")) ||
        (rc = dev_upload(&s->d_sub, s->sub_masks.data(), s->sub_masks.size(), "source subsets")) ||
        (rc = dev_upload(&s->d_inv_tfac, s->inv_tfac.data(), s->inv_tfac.size(), "source group factors")) ||
        (rc = dev_upload(&s->d_pred, s->builder.pred.data(), s->builder.pred.size(), "source inner tables")) ||
        (rc = dev_upload(&s->d_off, s->off.data(), s->off.size(), "source offsets")) ||
        (rc = dev_upload(&s->d_amp_off, s->amp_off.data(), s->amp_off.size(), "source amplitude offsets")) ||
        (rc = dev_upload(&s->d_binom, s->builder.B.t.data(), s->builder.B.t.size(), "binomial table")) ||
        (rc = alloc_dev(&s->d_amp, (size_t)s->namp * 16, "common-group amplitudes")) ||
        (rc = alloc_dev((void **)&s->d_slots, nslots * G * 8, "source subset vectors")) ||
        (rc = alloc_dev((void **)&s->d_temp, ntemp * G * 8, "source butterfly scratch")) ||
        (rc = alloc_dev((void **)&s->d_part, (size_t)(SLOS_SRC_STATS_MAX_BLOCKS + nmax + 1) * 3 * 8,
                        "source statistics partials")) ||
        (rc = alloc_dev((void **)&s->d_res, (size_t)(nmax + 1) * 3 * 8, "source statistics"))) {
        s->free_device();
        delete s;
        return rc;
    }
    const double one[2] = {1.0, 0.0};  // the empty group: the vacuum's coefficient
    hipError_t he = hipMemcpy(s->d_amp, one, sizeof one, hipMemcpyHostToDevice);
    if (he != hipSuccess) {
        rc = hip_fail(he, "source set-up");
        s->free_device();
        delete s;
        return rc;
    }
    *out = s;
    return SLOS_OK;
}

void slos_source_destroy(slos_source_t s)
{
    if (!s) return;
    s->free_device();
    delete s;
}

int64_t slos_source_num_outputs(slos_source_t s) { return s ? (int64_t)s->G : -1; }

int slos_source_info(slos_source_t s, int64_t *offsets, double *emission)
{
    if (!s) return fail(SLOS_ERR_INVALID_ARG, "source plan is NULL");
    if (offsets)
        for (int k = 0; k <= s->nmax + 1; ++k) offsets[k] = (int64_t)s->off[k];
    if (emission) {
        emission[0] = s->p0;
        emission[1] = s->p1;
        emission[2] = s->p2;
    }
    return SLOS_OK;
}

int slos_source_probs(slos_source_t s, const void *U, double *probs, void *stream)
{
    if (!s) return fail(SLOS_ERR_INVALID_ARG, "source plan is NULL");
    if (!U || !probs) return fail(SLOS_ERR_INVALID_ARG, "U and probs must be device pointers");
    const uint64_t G = s->G;
    int e;
    SrcGroupParams gp{};
    gp.amp = (double2 *)s->d_amp;
    gp.amp_off = s->d_amp_off;
    gp.desc = s->d_desc;
    gp.pred = s->d_pred;
    gp.U = U;
    gp.m = s->m;
    for (int b = 0; b < s->n; ++b) gp.modes[b] = (uint8_t)s->modes[b];
    for (int a = 1; a <= std::min(s->n, s->nmax); ++a) {
        gp.subsets = s->d_sub + s->sub_off[a];
        gp.leaf_lo = s->leaves_upto[a - 1];
        gp.leaf_hi = s->leaves_upto[a];
        gp.off_out = s->off[a];
        gp.off_in = s->off[a - 1];
        if ((e = slos_launch_src_group(gp, (int)(s->sub_off[a + 1] - s->sub_off[a]), stream)))
            return hip_fail((hipError_t)e, "source group kernel");
    }
    SrcFillParams fp{};
    fp.slots = s->d_slots;
    fp.G = G;
    fp.amp = (const double2 *)s->d_amp;
    fp.amp_off = s->d_amp_off;
    fp.inv_tfac = s->d_inv_tfac;
    fp.desc = s->d_desc;
    fp.lowfac = s->d_lowfac;
    for (int k = 0; k <= s->nmax; ++k) fp.leaves_upto[k] = s->leaves_upto[k];
    for (int k = 0; k <= s->nmax + 1; ++k) fp.off[k] = s->off[k];
    fp.nmax = s->nmax;
    if ((e = slos_launch_src_fill(fp, 1 << s->n, stream))) return hip_fail((hipError_t)e, "source fill kernel");
    SrcPassParams pp{};
    pp.desc = s->d_desc;
    pp.nleaves = s->nleaves;
    pp.pred = s->d_pred;
    pp.U = U;
    pp.m = s->m;
    pp.nmax = s->nmax;
    for (int b = 0; b < s->n; ++b) {
        // pairs r: P0 = slot (2r) << b (source b not common), P1 = slot (2r+1) << b.
        // With c = popcount(r): P0 holds photon numbers [c, c + 2b], P1 [c + 1, c + 1 + 2b].
        const int npairs = 1 << (s->n - b - 1);
        const uint64_t st = (uint64_t(2) << b) * G;
        double *P0 = s->d_slots, *P1 = s->d_slots + (uint64_t(1) << b) * G, *Z = s->d_temp;
        const int cmax = s->n - b - 1;  // largest c of the step
        pp.col = s->modes[b];
        // Z = (1-x) p2 L P0 + x p2 P1 + (1-x) p1 P0, photon numbers [c, c + 2b + 1]
        pp.in = P0;
        pp.s_in = st;
        pp.in_lo = 0;
        pp.in_len = 2 * b;
        pp.a = P1;
        pp.s_a = st;
        pp.a_lo = 1;
        pp.a_len = 2 * b;
        pp.b = P0;
        pp.s_b = st;
        pp.b_lo = 0;
        pp.b_len = 2 * b;
        pp.y = Z;
        pp.s_y = G;
        pp.y_len = 2 * b + 1;
        pp.gamma = (1.0 - s->x) * s->p2;
        pp.alpha = s->x * s->p2;
        pp.beta = (1.0 - s->x) * s->p1;
        pp.nleaves = s->leaves_upto[std::min(s->nmax, cmax + pp.y_len)];
        if ((e = slos_launch_src_pass(pp, npairs, stream))) return hip_fail((hipError_t)e, "source pass kernel");
        // P0 <- L Z + p0 P0 + x p1 P1, photon numbers [c, c + 2b + 2]
        pp.in = Z;
        pp.s_in = G;
        pp.in_lo = 0;
        pp.in_len = 2 * b + 1;
        pp.a = P0;
        pp.s_a = st;
        pp.a_lo = 0;
        pp.a_len = 2 * b;
        pp.b = P1;
        pp.s_b = st;
        pp.b_lo = 1;
        pp.b_len = 2 * b;
        pp.y = P0;
        pp.s_y = st;
        pp.y_len = 2 * b + 2;
        pp.gamma = 1.0;
        pp.alpha = s->p0;
        pp.beta = s->x * s->p1;
        pp.nleaves = s->leaves_upto[std::min(s->nmax, cmax + pp.y_len)];
        if ((e = slos_launch_src_pass(pp, npairs, stream))) return hip_fail((hipError_t)e, "source pass kernel");
    }
    hipError_t he = hipMemcpyAsync(probs, s->d_slots, G * 8, hipMemcpyDeviceToDevice, (hipStream_t)stream);
    if (he != hipSuccess) return hip_fail(he, "source result copy");
    return SLOS_OK;
}

int slos_source_postselect(slos_source_t s, const double *probs, const int32_t *group_of_mode, int ngroups,
                           const int32_t *count_min, const int32_t *count_max, int min_modes, double *result,
                           void *stream)
{
    if (!s) return fail(SLOS_ERR_INVALID_ARG, "source plan is NULL");
    if (!probs || !result) return fail(SLOS_ERR_INVALID_ARG, "probs (device) and result (host) are required");
    if (ngroups < 0 || ngroups > SLOS_PS_MAX_GROUPS)
        return fail(SLOS_ERR_INVALID_ARG, "ngroups = %d outside [0, %d]", ngroups, SLOS_PS_MAX_GROUPS);
    if (ngroups > 0 && (!count_min || !count_max))
        return fail(SLOS_ERR_INVALID_ARG, "count_min and count_max are required");
    if (min_modes < 0) return fail(SLOS_ERR_INVALID_ARG, "min_modes = %d is negative", min_modes);
    SrcStatsParams sp{};
    for (int j = 0; j < 256; ++j) sp.group[j] = -1;
    if (group_of_mode)
        for (int j = 0; j < s->m; ++j) {
            const int g = group_of_mode[j];
            if (g < -1 || g >= ngroups)
                return fail(SLOS_ERR_INVALID_ARG, "group_of_mode[%d] = %d outside [-1, %d)", j, g, ngroups);
            sp.group[j] = (int8_t)g;
        }
    for (int g = 0; g < ngroups; ++g) {
        if (count_min[g] < 0 || count_max[g] < count_min[g] || count_max[g] > 255)
            return fail(SLOS_ERR_INVALID_ARG, "group %d: bounds [%d, %d] invalid", g, count_min[g], count_max[g]);
        sp.cmin[g] = (uint8_t)count_min[g];
        sp.cmax[g] = (uint8_t)count_max[g];
    }
    sp.P = probs;
    sp.off = s->d_off;
    sp.binom = s->d_binom;
    sp.bstride = s->builder.B.stride;
    sp.m = s->m;
    sp.nmax = s->nmax;
    sp.ngroups = ngroups;
    sp.min_modes = min_modes;
    sp.partials = s->d_part;
    sp.result = s->d_res;
    // fixed chunks of >= 1024 states (a multiple of 256), whole chunks per photon number
    uint64_t chunk = std::max<uint64_t>(1024, (s->G + SLOS_SRC_STATS_MAX_BLOCKS - 1) / SLOS_SRC_STATS_MAX_BLOCKS);
    chunk = (chunk + 255) / 256 * 256;
    sp.chunk = chunk;
    sp.blk_off[0] = 0;
    for (int k = 0; k <= s->nmax; ++k)
        sp.blk_off[k + 1] = sp.blk_off[k] + (uint32_t)((s->off[k + 1] - s->off[k] + chunk - 1) / chunk);
    int e = slos_launch_src_stats(sp, stream);
    if (e) return hip_fail((hipError_t)e, "source statistics kernel");
    hipError_t he = hipMemcpyAsync(result, s->d_res, (size_t)(s->nmax + 1) * 3 * 8, hipMemcpyDeviceToHost,
                                   (hipStream_t)stream);
    if (he == hipSuccess) he = hipStreamSynchronize((hipStream_t)stream);
    if (he != hipSuccess) return hip_fail(he, "source statistics copy");
    return SLOS_OK;
}

} // extern "C"
