"""CPU tests of the C ABI's host logic: exports, Fock ranking, leaf tiling, errors.

No GPU is touched: plans here use SLOS_HOST_ONLY, and device calls are only
checked for their argument validation.
"""
import ctypes
import itertools
import math
import os
import re

import numpy as np
import pytest

from paper_2204_00602_amd import slos

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "slos.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(slos_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    names = header_functions()
    assert "slos_amplitudes" in names and "slos_plan" in names
    L = slos.lib()
    for name in names:
        assert hasattr(L, name), name


@pytest.mark.parametrize("m,n", [(1, 0), (1, 7), (6, 3), (12, 6), (24, 12), (255, 3)])
def test_fock_count(m, n):
    assert slos.fock_count(m, n) == math.comb(m + n - 1, n)


def test_fock_count_overflow_detected():
    with pytest.raises(slos.SlosError) as e:
        slos.fock_count(255, 32)
    assert e.value.code == -2


def rev_lex_key(s):
    return tuple(reversed(list(s)))


@pytest.mark.parametrize("m,n", [(1, 4), (2, 3), (3, 3), (5, 4), (6, 3), (4, 6), (8, 2)])
def test_rank_unrank_bijection_and_colex_order(m, n):
    M = math.comb(m + n - 1, n)
    states = [slos.fock_unrank(m, n, r) for r in range(M)]
    assert all(s.sum() == n and s.min() >= 0 for s in states)
    assert len({s.tobytes() for s in states}) == M
    for r, s in enumerate(states):
        assert slos.fock_rank(s) == r
    # colex = lexicographic on the occupation vector read from the last mode
    keys = [rev_lex_key(s) for s in states]
    assert keys == sorted(keys)
    assert np.array_equal(states[0], np.eye(m, dtype=np.int32)[0] * n)


def test_rank_spot_checks_24_12():
    rng = np.random.default_rng(3)
    M = math.comb(35, 12)
    for r in list(rng.integers(0, M, 200)) + [0, M - 1]:
        s = slos.fock_unrank(24, 12, int(r))
        assert slos.fock_rank(s) == r
    top = np.zeros(24, np.int32)
    top[-1] = 12
    assert slos.fock_rank(top) == M - 1


def test_rank_rejects_bad_states():
    with pytest.raises(slos.SlosError):
        slos.fock_rank([1, -1, 2])
    with pytest.raises(slos.SlosError):
        slos.fock_unrank(3, 2, 6)  # only 6 states: ranks 0..5


@pytest.mark.parametrize("T", [[1, 1, 1, 0, 0, 0], [2, 0, 1, 0, 3], [0, 0, 4], [1] * 6 + [0] * 6])
def test_plan_rank_unrank_match_independent_enumeration(T):
    """slos_rank / slos_unrank of a plan: a bijection onto [0, M) that agrees
    with the Fock-space functions, checked on the oracle's own enumeration of
    the output states (recursive generation, no shared code)."""
    import oracle
    m, n = len(T), int(sum(T))
    p = slos.Plan(T, "c64", host_only=True)
    S = oracle.fock_states(m, n)
    ranks = [p.rank(s) for s in S]
    assert sorted(ranks) == list(range(math.comb(m + n - 1, n)))
    for s, r in zip(S, ranks):
        assert r == slos.fock_rank(s)
        assert np.array_equal(p.unrank(r), s)


def test_plan_rank_unrank_reject_bad_arguments():
    p = slos.Plan([1, 1, 0], "c64", host_only=True)
    with pytest.raises(slos.SlosError):
        p.rank([1, 1, 1])          # three photons, the plan has two
    with pytest.raises(slos.SlosError):
        p.rank([3, -1, 0])
    with pytest.raises(slos.SlosError):
        p.unrank(6)                # C(4, 2) = 6 outputs: ranks 0..5
    with pytest.raises(slos.SlosError):
        p.unrank(-1)
    L = slos.lib()
    r = ctypes.c_int64(0)
    st = (ctypes.c_int32 * 3)(1, 1, 0)
    assert L.slos_rank(None, st, ctypes.byref(r)) == -1
    assert L.slos_unrank(None, 0, st) == -1


@pytest.mark.parametrize("m,T,leaf_max", [
    (6, [1, 1, 1, 0, 0, 0], 4096), (6, [1, 1, 1, 0, 0, 0], 3), (12, [1] * 6 + [0] * 6, 64),
    (9, [2, 0, 1, 0, 0, 2, 0, 0, 1], 17), (3, [4, 0, 2], 1), (14, [1, 2, 0, 1, 0, 0, 2, 0, 1, 0, 0, 0, 0, 0], 256),
    (20, [1] * 5 + [0] * 15, 128),
])
@pytest.mark.parametrize("order", [0, 2])
def test_leaf_tiling_covers_each_layer_once(m, T, leaf_max, order):
    p = slos.Plan(T, "c64", host_only=True, options={"leaf_max": leaf_max, "leaf_order": order})
    n = int(sum(T))
    for k in range(1, n + 1):
        Nk, nl = p.layer_info(k)
        assert Nk == math.comb(m + k - 1, k)
        nxt = 0
        for base, q, K, hm in sorted(p.leaf(k, idx) for idx in range(nl)):
            size = math.comb(q + K - 1, K)
            assert base == nxt, (k, idx)
            assert size <= leaf_max or K == 0 or q == 1 or (q == m and size == Nk)
            assert len(hm) == k - K and all(h >= q for h in hm) and hm == sorted(hm, reverse=True)
            # first and last state of the leaf: same high part, low part spans F(q, K)
            first = slos.fock_unrank(m, k, base)
            last = slos.fock_unrank(m, k, base + size - 1)
            high = np.zeros(m, np.int32)
            for h in hm:
                high[h] += 1
            assert np.array_equal(first[q:], high[q:]) and np.array_equal(last[q:], high[q:])
            assert first[0] == K and last[q - 1] == K
            nxt = base + size
        assert nxt == Nk


def test_plan_argument_validation():
    bad = [
        ((0, 0, [], slos.SLOS_C64), -1),
        ((3, 2, [1, 0, 0], slos.SLOS_C64), -1),          # wrong photon count
        ((3, 1, [2, -1, 0], slos.SLOS_C64), -1),         # negative occupation
        ((3, 1, [1, 0, 0], slos.SLOS_C64 | slos.SLOS_C128), -4),
        ((3, 1, [1, 0, 0], 0), -4),
        ((3, 1, [1, 0, 0], slos.SLOS_C128 | slos.SLOS_COMPENSATED), -4),
        ((3, 1, [1, 0, 0], slos.SLOS_C64 | 0x8000), -1),
        ((3, 1, [1, 0, 0], slos.SLOS_C64 | slos.SLOS_COMP_FP64), -1),             # needs COMPENSATED
        ((3, 1, [1, 0, 0], slos.SLOS_C64 | slos.SLOS_COMPENSATED | slos.SLOS_COMP_FP64
          | slos.SLOS_COMP_KNUTH), -1),                                           # two modes at once
        ((256, 1, [1] + [0] * 255, slos.SLOS_C64), -1),
        ((2, 33, [33, 0], slos.SLOS_C64), -1),
    ]
    import ctypes
    L = slos.lib()
    for (m, n, T, flags), code in bad:
        arr = np.asarray(T if T else [0], dtype=np.int32)
        h = ctypes.c_void_p()
        rc = L.slos_plan(m, n, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), flags, ctypes.byref(h))
        assert rc == code, (m, n, T, flags, rc, L.slos_last_error())
        assert not h.value
        assert L.slos_last_error()


def test_plan_options_validation():
    for opts in ({"leaf_max": 70000}, {"block_threads": 96}, {"outputs_per_lane": 3},
                 {"grid_blocks": -1}, {"comp_from_layer": -2}, {"max_batch": 70000}, {"max_batch": -3}):
        with pytest.raises(slos.SlosError) as e:
            slos.Plan([1, 1, 0], "c64", host_only=True, options=opts)
        assert e.value.code == -1


def test_device_calls_reject_null_and_host_only_plans():
    L = slos.lib()
    assert L.slos_amplitudes(None, None, None, None, None) == -1
    assert L.slos_num_outputs(None) == -1
    L.slos_plan_destroy(None)
    p = slos.Plan([1, 1, 0], "c64", host_only=True)
    assert L.slos_probs(p._h, None, None, None, None) == -1
    assert p.num_outputs == 6


def test_algorithmic_bytes_formula():
    # m=24, n=12, c64: 13.35 GB (each layer read once and written once)
    b = slos.algorithmic_bytes(24, 12, 8)
    assert abs(b / 1e9 - 13.35) < 0.01
    assert slos.algorithmic_bytes(24, 12, 16) == 2 * b
    N = [math.comb(6 + k - 1, k) for k in range(4)]
    assert slos.algorithmic_bytes(6, 3, 16) == 16 * (sum(N[:3]) + sum(N[1:]))


def test_batch_plan_validation():
    import ctypes
    L = slos.lib()
    h = ctypes.c_void_p()
    i32p = ctypes.POINTER(ctypes.c_int32)
    ms = np.array([3, 2], np.int32)
    bad_inputs = [np.array([1, -1, 0, 1, 0], np.int32), np.array([17, 0, 0, 0, 0], np.int32)]
    for inp in bad_inputs:
        rc = L.slos_batch_plan(2, ms.ctypes.data_as(i32p), inp.ctypes.data_as(i32p), slos.SLOS_C64, None,
                               ctypes.byref(h))
        assert rc == -1 and not h.value
    ok = np.array([1, 0, 1, 1, 1], np.int32)
    assert L.slos_batch_plan(0, ms.ctypes.data_as(i32p), ok.ctypes.data_as(i32p), slos.SLOS_C64, None,
                             ctypes.byref(h)) == -1
    assert L.slos_batch_plan(2, ms.ctypes.data_as(i32p), ok.ctypes.data_as(i32p), 0, None, ctypes.byref(h)) == -4
    # option checks come before any device work: a low-block cap below -1, or a
    # leaf size whose low blocks overflow a workgroup's LDS, is refused
    for opts in ({"low_block_max": -2}, {"leaf_max": 0x10001}, {"outputs_per_lane": 3}):
        o = slos.Options()
        for k, v in opts.items():
            setattr(o, k, v)
        rc = L.slos_batch_plan(2, ms.ctypes.data_as(i32p), ok.ctypes.data_as(i32p), slos.SLOS_C64,
                               ctypes.byref(o), ctypes.byref(h))
        assert rc == -1 and not h.value, (opts, rc)
    L.slos_batch_destroy(None)


def test_sampling_calls_validate_arguments():
    L = slos.lib()
    assert L.slos_cdf(None, None, None) == -1
    assert L.slos_marginals(None, None, None, None) == -1
    assert L.slos_sample(None, None, None, 1, None, None) == -1
    p = slos.Plan([1, 1, 0], "c64", host_only=True)
    assert L.slos_cdf(p._h, None, None) == -1


def test_postselect_validates_arguments():
    import ctypes
    L = slos.lib()
    i32p = ctypes.POINTER(ctypes.c_int32)
    assert L.slos_postselect(None, None, None, 0, None, None, None, None, None, 0, None, None) == -1
    p = slos.Plan([1, 1, 0], "c64", host_only=True)
    assert L.slos_postselect(p._h, None, None, 0, None, None, None, None, None, 0, None, None) == -1


def test_many_calls_validate_arguments():
    L = slos.lib()
    assert L.slos_amplitudes_many(None, 1, None, None, None, None) == -1
    assert L.slos_backward_many(None, 1, None, None, None, None) == -1
    p = slos.Plan([1, 1, 0], "c64", host_only=True, options={"max_batch": 4})
    assert L.slos_probs_many(p._h, 2, None, None, None, None) == -1


@pytest.mark.parametrize("T", [[1, 1, 1, 0, 0, 0], [2, 0, 1, 0], [1] * 6 + [0] * 6, [3, 0, 0]])
def test_output_scales_are_the_normalisation(T):
    # c_S = sqrt(prod_j s_j!) / sqrt(prod_i t_i!): a(S) = perm(U_{S,T}) / sqrt(prod s! prod t!)
    # (Eq. eqperm) while the recurrence's A_n[S] = perm(U_{S,T}) / prod_j s_j!
    p = slos.Plan(T, "c64", host_only=True, options={"leaf_max": 64})
    M = p.num_outputs
    rng = np.random.default_rng(7)
    ranks = np.unique(np.concatenate([[0, M - 1], rng.integers(0, M, size=min(M, 300))])).astype(np.int64)
    sc = p.output_scales(ranks)
    tfac = math.prod(math.factorial(t) for t in T)
    for r, c in zip(ranks, sc):
        s = p.unrank(int(r))
        sfac = math.prod(math.factorial(v) for v in s)
        assert c == pytest.approx(math.sqrt(sfac) / math.sqrt(tfac), rel=4e-16), (r, s)


def test_output_scales_and_fused_loss_validate_arguments():
    L = slos.lib()
    p = slos.Plan([1, 1, 0], "c64", host_only=True, options={"max_batch": 4})
    # ranks outside [0, M) get 0; a negative count or missing arrays are errors
    sc = p.output_scales(np.array([-1, 0, 6, 5], dtype=np.int64))
    assert sc[0] == 0.0 and sc[2] == 0.0 and sc[1] > 0.0 and sc[3] > 0.0
    assert L.slos_output_scales(p._h, None, -1, None) == -1
    assert L.slos_output_scales(p._h, None, 3, None) == -1
    assert L.slos_output_scales(None, None, 0, None) == -1
    assert L.slos_sq_loss_backward_many(None, 1, None, None, None, None, 0, None, None, None, None) == -1
    # device call on a host-only plan
    assert L.slos_sq_loss_backward_many(p._h, 1, None, None, None, None, 0, None, None, None, None) == -1


def test_select_validates_arguments():
    L = slos.lib()
    assert L.slos_select(None, None, None, 1, None, None) == -1
    p = slos.Plan([1, 1, 0], "c64", host_only=True)
    assert L.slos_select(p._h, None, None, 1, None, None) == -1


@pytest.mark.parametrize("beta,g2,V,nmax,state", [
    (0.0, 0.0, 1.0, -1, [1, 1, 0]),        # no emission
    (1.2, 0.0, 1.0, -1, [1, 1, 0]),
    (1.0, -0.1, 1.0, -1, [1, 1, 0]),
    (1.0, 0.6, 1.0, -1, [1, 1, 0]),        # beta * g2 above 1/2
    (1.0, 0.0, 1.5, -1, [1, 1, 0]),
    (1.0, 0.1, 1.0, 17, [1, 1, 0]),        # nmax above 16
    (1.0, 0.1, 1.0, 5, [1, 1, 0]),         # nmax above 2n
    (1.0, 0.1, 1.0, -1, [9, 0, 0]),        # 2n = 18 photons by default
    (1.0, 0.0, 1.0, -1, [13, 0, 0]),       # more than 12 sources
    (1.0, 0.0, 1.0, -1, [1, -1, 0]),
])
def test_source_plan_validates_arguments(beta, g2, V, nmax, state):
    import ctypes
    L = slos.lib()
    st = np.ascontiguousarray(np.asarray(state, np.int32))
    sp = slos.SourceParams(beta, g2, V)
    h = ctypes.c_void_p()
    rc = L.slos_source_plan(len(state), st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(sp),
                            nmax, None, ctypes.byref(h))
    assert rc == -1 and not h.value
    assert b"outside" in L.slos_last_error() or b"exceeds" in L.slos_last_error() or \
        b"sources" in L.slos_last_error() or b"above" in L.slos_last_error() or b"negative" in L.slos_last_error()


def test_source_calls_validate_arguments():
    L = slos.lib()
    assert L.slos_source_plan(3, None, None, -1, None, None) == -1
    assert L.slos_source_probs(None, None, None, None) == -1
    assert L.slos_source_postselect(None, None, None, 0, None, None, 0, None, None) == -1
    assert L.slos_source_info(None, None, None) == -1
    assert L.slos_source_num_outputs(None) == -1
    L.slos_source_destroy(None)


@pytest.mark.parametrize("cap", [8, 35, 120])
def test_low_block_cap_splits_leaves(cap):
    """Every leaf's low block (same high part, K - 1 low photons) stays within
    low_block_max, and the leaves still tile each layer exactly."""
    m, T = 9, [1, 1, 1, 1, 0, 0, 0, 0, 1]
    p = slos.Plan(T, "c64", host_only=True, options={"leaf_max": 4096, "low_block_max": cap})
    for k in range(1, 6):
        Nk, nl = p.layer_info(k)
        nxt = 0
        for base, q, K, hm in sorted(p.leaf(k, idx) for idx in range(nl)):
            low = math.comb(q + K - 2, K - 1) if K > 0 else 0
            assert low <= cap or q == 1, (k, q, K, low)
            assert base == nxt
            nxt = base + math.comb(q + K - 1, K)
        assert nxt == Nk


@pytest.mark.parametrize("dt,cap", [("c64", 3072), ("c128", 2560)])
def test_default_low_block_cap(dt, cap):
    """With default options the low blocks stay within the documented cap
    (3072 complex64 states = 24 KiB, six workgroups per CU; 2560 complex128
    states = 40 KiB), and the cap is reached, so it is the one in force."""
    T = [1] * 10 + [0] * 14  # last layer 92.6M states: leaves of the full 16384/8192 size
    p = slos.Plan(T, dt, host_only=True)
    Nk, nl = p.layer_info(10)
    biggest = 0
    for idx in range(nl):
        base, q, K, hm = p.leaf(10, idx)
        low = math.comb(q + K - 2, K - 1) if K > 0 else 0
        assert low <= cap or q == 1, (q, K, low)
        biggest = max(biggest, low)
    assert biggest > cap * 3 // 4, biggest
    p.close()


def test_leaf_order_and_cap_validation():
    with pytest.raises(slos.SlosError):
        slos.Plan([1, 1, 0], "c64", host_only=True, options={"leaf_order": 5})
    with pytest.raises(slos.SlosError):
        slos.Plan([1, 1, 0], "c64", host_only=True, options={"low_block_max": -2})
