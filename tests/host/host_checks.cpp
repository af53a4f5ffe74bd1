// Host-side checks of the planner (plan.cpp), built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py.  Everything here
// runs without a GPU: Fock-space arithmetic, host-only plans (leaf tilings,
// inner tables, descriptors) over a range of shapes, option validation and the
// error paths, and the batch and source planners up to their device check.
// Prints one line per failed check and exits non-zero if any failed.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "slos.h"

static int failures = 0;
#define CHECK(cond, ...)                                  \
    do {                                                  \
        if (!(cond)) {                                    \
            ++failures;                                   \
            std::printf("FAIL %s:%d: ", __FILE__, __LINE__); \
            std::printf(__VA_ARGS__);                     \
            std::printf(" [%s]\n", slos_last_error());    \
        }                                                 \
    } while (0)

static int64_t binom(int a, int b)
{
    if (b < 0 || a < b) return 0;
    int64_t v = 1;
    for (int i = 1; i <= b; ++i) v = v * (a - b + i) / i;
    return v;
}

// rank <-> state is a bijection onto [0, C(m+n-1, n)); ranks follow colex order
// (lexicographic on the occupations read from the last mode); and the states
// whose highest photon sits at c = d_n + n - 1 fill ranks [C(c, n), C(c+1, n)).
static void fock_bijection(int m, int n)
{
    int64_t M = 0;
    CHECK(slos_fock_count(m, n, &M) == SLOS_OK && M == binom(m + n - 1, n), "count m=%d n=%d", m, n);
    std::vector<int32_t> s(m), prev(m);
    for (int64_t r = 0; r < M; ++r) {
        CHECK(slos_fock_unrank(m, n, r, s.data()) == SLOS_OK, "unrank %lld", (long long)r);
        int sum = 0, top = -1;
        for (int j = 0; j < m; ++j) {
            sum += s[j];
            if (s[j] > 0) top = j;
        }
        CHECK(sum == n, "unrank %lld sums to %d", (long long)r, sum);
        int64_t back = -1;
        CHECK(slos_fock_rank(m, n, s.data(), &back) == SLOS_OK && back == r, "rank(unrank(%lld)) = %lld",
              (long long)r, (long long)back);
        if (n > 0) {
            const int c = top + n - 1;
            CHECK(binom(c, n) <= r && r < binom(c + 1, n), "m=%d n=%d rank %lld outside its top block", m, n,
                  (long long)r);
        }
        if (r > 0) {
            int j = m - 1;
            while (j >= 0 && s[j] == prev[j]) --j;
            CHECK(j >= 0 && s[j] > prev[j], "m=%d n=%d ranks %lld, %lld out of colex order", m, n,
                  (long long)r - 1, (long long)r);
        }
        prev = s;
    }
}

static void host_plan(int m, const std::vector<int32_t> &T, int flags, const slos_options_t *opts)
{
    int n = 0;
    for (int t : T) n += t;
    slos_plan_t p = nullptr;
    const int rc = slos_plan_ex(m, n, T.data(), flags | SLOS_HOST_ONLY, opts, &p);
    CHECK(rc == SLOS_OK && p, "host-only plan m=%d n=%d flags=%x", m, n, flags);
    if (!p) return;
    int64_t M = 0;
    slos_fock_count(m, n, &M);
    CHECK(slos_num_outputs(p) == M, "num_outputs m=%d n=%d", m, n);
    for (int k = 1; k <= n; ++k) {
        int64_t Nk = 0, nl = 0;
        CHECK(slos_plan_info(p, k, &Nk, &nl) == SLOS_OK, "info k=%d", k);
        int64_t want = 0;
        slos_fock_count(m, k, &want);
        CHECK(Nk == want, "layer %d has %lld states, want %lld", k, (long long)Nk, (long long)want);
        // the leaves tile the layer: every first rank in range, and the leaf
        // bases distinct (their sizes are checked by the Python host tests)
        std::vector<int64_t> bases;
        const int64_t step = nl > 4096 ? nl / 4096 : 1;
        for (int64_t i = 0; i < nl; i += step) {
            int64_t base = -1;
            int32_t q = -1, K = -1;
            std::vector<int32_t> hm(k + 1, -1);
            CHECK(slos_plan_leaf(p, k, i, &base, &q, &K, hm.data()) == SLOS_OK, "leaf %lld", (long long)i);
            CHECK(base >= 0 && base < Nk, "leaf %lld base %lld", (long long)i, (long long)base);
            CHECK(q >= 0 && q <= m && K >= 0 && K <= k, "leaf %lld q=%d K=%d", (long long)i, q, K);
            for (int h = 0; h < k - K; ++h) CHECK(hm[h] >= 0 && hm[h] < m, "leaf high mode %d", hm[h]);
        }
        int64_t base = 0;
        CHECK(slos_plan_leaf(p, k, nl, &base, nullptr, nullptr, nullptr) != SLOS_OK, "leaf past the end accepted");
    }
    CHECK(slos_plan_info(p, n + 1, nullptr, nullptr) != SLOS_OK || n == 0, "layer past n accepted");
    // normalisation factors of a spread of outputs (and two outside the set)
    {
        std::vector<int64_t> rk = {-1, M, 0, M - 1};
        for (int64_t r = 1; r < M - 1; r += 1 + M / 97) rk.push_back(r);
        std::vector<double> sc(rk.size(), -1.0);
        CHECK(slos_output_scales(p, rk.data(), (int64_t)rk.size(), sc.data()) == SLOS_OK, "output scales");
        CHECK(sc[0] == 0.0 && sc[1] == 0.0, "ranks outside the output set must get 0");
        for (size_t t = 2; t < rk.size(); ++t) CHECK(sc[t] > 0.0 && sc[t] < 1e30, "scale of rank %lld", (long long)rk[t]);
    }
    slos_plan_destroy(p);
}

int main()
{
    // Fock-space arithmetic
    for (int m = 1; m <= 14; ++m)
        for (int n = 0; n <= 7; ++n) fock_bijection(m, n);
    int64_t c = 0;
    CHECK(slos_fock_count(255, 32, &c) == SLOS_ERR_SIZE_OVERFLOW || c > 0, "count(255, 32)");
    CHECK(slos_fock_count(0, 3, &c) != SLOS_OK, "m = 0 accepted");
    CHECK(slos_fock_count(3, -1, &c) != SLOS_OK, "n < 0 accepted");
    int32_t bad[3] = {1, -1, 2};
    int64_t r = 0;
    CHECK(slos_fock_rank(3, 2, bad, &r) != SLOS_OK, "negative occupation accepted");
    CHECK(slos_fock_unrank(3, 2, 99, bad) != SLOS_OK, "rank past the end accepted");

    // host-only plans over a range of shapes, dtypes and options
    std::vector<int32_t> t6 = {1, 1, 1, 0, 0, 0}, t12(12, 0), t24(24, 0), tb = {2, 0, 3, 0, 1, 0, 2, 0, 0};
    for (int i = 0; i < 6; ++i) t12[i] = 1;
    for (int i = 0; i < 12; ++i) t24[i] = 1;
    std::vector<int32_t> t255(255, 0);
    t255[0] = t255[127] = t255[254] = 1;
    std::vector<int32_t> t32 = {10, 11, 11}, t1 = {4}, t0 = {0, 0, 0};
    for (int flags : {SLOS_C64, SLOS_C128, SLOS_C64 | SLOS_COMPENSATED, SLOS_C128 | SLOS_KEEP_LAYERS}) {
        host_plan(6, t6, flags, nullptr);
        host_plan(12, t12, flags, nullptr);
        host_plan(9, tb, flags, nullptr);
        host_plan(3, t32, flags, nullptr);
        host_plan(1, t1, flags, nullptr);
        host_plan(3, t0, flags, nullptr);
    }
    host_plan(24, t24, SLOS_C64 | SLOS_COMPENSATED, nullptr);
    host_plan(255, t255, SLOS_C128, nullptr);
    slos_options_t o{};
    o.leaf_max = 40;
    o.leaf_order = 3;
    host_plan(12, t12, SLOS_C64, &o);
    o = slos_options_t{};
    o.low_block_max = 6;
    o.leaf_max = 200;
    host_plan(9, tb, SLOS_C128, &o);
    o = slos_options_t{};
    o.wide_descriptors = 1;
    host_plan(12, t12, SLOS_C64, &o);

    // invalid arguments and options: error codes, never a crash
    slos_plan_t p = nullptr;
    CHECK(slos_plan_ex(6, 2, t6.data(), SLOS_C64 | SLOS_HOST_ONLY, nullptr, &p) != SLOS_OK, "wrong n accepted");
    CHECK(slos_plan_ex(6, 3, t6.data(), SLOS_C64 | SLOS_C128 | SLOS_HOST_ONLY, nullptr, &p) != SLOS_OK,
          "two dtypes accepted");
    CHECK(slos_plan_ex(6, 3, nullptr, SLOS_C64 | SLOS_HOST_ONLY, nullptr, &p) != SLOS_OK, "NULL state accepted");
    for (int field = 0; field < 6; ++field) {
        o = slos_options_t{};
        if (field == 0) o.leaf_max = 1 << 20;
        if (field == 1) o.block_threads = 96;
        if (field == 2) o.outputs_per_lane = 3;
        if (field == 3) o.leaf_order = 9;
        if (field == 4) o.low_block_max = -7;
        if (field == 5) o.ticket_leaves = 1 << 20;
        CHECK(slos_plan_ex(6, 3, t6.data(), SLOS_C64 | SLOS_HOST_ONLY, &o, &p) == SLOS_ERR_INVALID_ARG,
              "bad option %d accepted", field);
    }
    slos_plan_destroy(nullptr);
    CHECK(slos_num_outputs(nullptr) == -1, "NULL plan outputs");

    // the batch and source planners build their host tables, then need a device
    std::vector<int32_t> ms = {6, 12, 3, 9}, ins;
    ins.insert(ins.end(), t6.begin(), t6.end());
    ins.insert(ins.end(), t12.begin(), t12.end());
    ins.insert(ins.end(), t0.begin(), t0.end());
    ins.insert(ins.end(), tb.begin(), tb.end());
    slos_batch_t b = nullptr;
    const int brc = slos_batch_plan((int)ms.size(), ms.data(), ins.data(), SLOS_C64, nullptr, &b);
    CHECK(brc == SLOS_OK || brc == SLOS_ERR_NO_DEVICE, "batch plan: %d", brc);
    slos_batch_destroy(b);
    slos_source_params_t sp{0.9, 0.05, 0.92};
    slos_source_t s = nullptr;
    const int src = slos_source_plan(12, t12.data(), &sp, -1, nullptr, &s);
    CHECK(src == SLOS_OK || src == SLOS_ERR_NO_DEVICE, "source plan: %d", src);
    slos_source_destroy(s);

    std::printf("host checks: %d failure(s)\n", failures);
    return failures ? 1 : 0;
}
