"""GPU parity of post-selection over mode groups (heralds, post-selection
functions, Analyzer tables) against the oracle."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2204_00602_amd import inputs, slos

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    slos.lib()


def _probs(T, U, dtype):
    p = slos.Plan(T, dtype)
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    P = p.probs(torch.from_numpy(np.ascontiguousarray(U)).to(tdt).cuda())
    torch.cuda.synchronize()
    return p, P


def _cnot(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "ralph_cnot.json")))
    U = np.zeros((6, 6), np.complex128)
    for j, row in enumerate(g["unitary"]):
        for i, ((a, r), (b, s)) in enumerate(row):
            U[j, i] = (a * math.sqrt(r) + 1j * b * math.sqrt(s)) / 3.0
    return g, U


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("heralded", [False, True])
def test_cnot_performance_and_truth_table(golden_dir, dtype, heralded):
    g, U = _cnot(golden_dir)
    names = sorted(g["logical_states"])
    states = [np.array(g["logical_states"][k], np.int32) for k in names]
    ranks = [slos.fock_rank(s) for s in states]
    if heralded:
        gm, lo, hi = [2, 0, 0, 1, 1, 3], [1, 1, 0, 0], [1, 1, 0, 0]
    else:
        gm, lo, hi = [-1, 0, 0, 1, 1, -1], [1, 1], [1, 1]
    tol = 1e-12 if dtype == "c128" else 1e-6
    S = oracle.colex_sorted(oracle.fock_states(6, 2))
    keep_ref, _ = oracle.postselect(np.ones(len(S)), S, gm, lo, hi)
    fid = []
    for a, T in enumerate(states):
        p, P = _probs(T, U, dtype)
        kept, masked, table = p.postselect(P, gm, lo, hi, masked=True, ranks=ranks)
        assert abs(float(kept.item()) - 1.0 / 9.0) <= tol
        want = np.zeros(4)
        want[names.index(g["expected_map"][names[a]])] = 1.0
        assert np.allclose(table.cpu().numpy(), want, atol=10 * tol)
        fid.append(table.cpu().numpy()[names.index(g["expected_map"][names[a]])])
        Pn = P.cpu().numpy()
        assert np.array_equal(masked.cpu().numpy(), np.where(keep_ref, Pn, 0))
    assert abs(np.mean(fid) - 1.0) <= 10 * tol


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_config2_groups_match_oracle(dtype):
    m, n = 12, 6
    T, U = inputs.first_modes_input(m, n), inputs.haar_unitary(m, 2)
    p, P = _probs(T, U, dtype)
    S = oracle.colex_sorted(oracle.fock_states(m, n))
    Pref = oracle.probabilities(U, T, S)
    cases = [
        ([0, 0, 0, -1, -1, 1, -1, 2, 2, 2, 2, 2], [1, 0, 2], [2, 0, 6]),
        ([0] * 6 + [1] * 6, [3, 3], [3, 3]),
        ([-1] * m, [], []),
        ([0] + [-1] * 11, [7], [9]),   # more photons than exist: nothing kept
        ([i % 4 for i in range(m)], [1, 1, 1, 1], [2, 2, 2, 2]),
        # more than 4 groups: the 16-count table entries
        ([i % 5 for i in range(m)], [0, 1, 0, 1, 0], [2, 2, 1, 3, 2]),
        ([i % 6 for i in range(m)], [1] * 6, [1] * 6),
        (list(range(m)), [0] * m, [1] * m),                             # no bunching
    ]
    Pn = P.cpu().numpy().astype(np.float64)
    for gm, lo, hi in cases:
        kept, masked, table = p.postselect(P, gm, lo, hi, masked=True, ranks=[0, 5, 777, 12375])
        keep, tot_ref = oracle.postselect(Pref, S, gm, lo, hi)
        _, tot_same = oracle.postselect(Pn, S, gm, lo, hi)
        k = float(kept.item())
        assert abs(k - tot_same) <= 1e-12 * max(1.0, tot_same)
        assert abs(k - tot_ref) <= (1e-12 if dtype == "c128" else 2e-6)
        assert np.array_equal(masked.cpu().numpy(), np.where(keep, P.cpu().numpy(), 0))
        tb = table.cpu().numpy()
        for i, r in enumerate([0, 5, 777, 12375]):
            want = Pn[r] / k if keep[r] else 0.0
            assert tb[i] == pytest.approx(want, rel=1e-12, abs=1e-300), (gm, r)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_many_leaves_match_oracle(dtype):
    """m=16, n=8 (490,314 outputs): post-selection splits the last layer into
    many leaves of its own (up to 32768 states each) with several inner shapes,
    unlike config 2, which is a single leaf."""
    m, n = 16, 8
    T, U = inputs.first_modes_input(m, n), inputs.haar_unitary(m, 11)
    print(f"[postselect] m={m} n={n} {dtype}", flush=True)
    p, P = _probs(T, U, dtype)
    S = oracle.colex_sorted(oracle.fock_states(m, n))
    Pn = P.cpu().numpy().astype(np.float64)
    Pref = oracle.probabilities(U, T, S) if dtype == "c128" else None
    cases = [
        ([0, 0, 1, 1] + [-1] * 10 + [2, 2], [1, 0, 0], [1, 1, 0]),
        ([i % 3 for i in range(m)], [2, 2, 2], [3, 3, 3]),
        ([i % 5 for i in range(m)], [0, 1, 0, 1, 0], [3, 3, 2, 3, 3]),   # 16-count entries
        ([-1] * 8 + [0] * 8, [0], [0]),
    ]
    for gm, lo, hi in cases:
        kept, masked, _ = p.postselect(P, gm, lo, hi, masked=True)
        keep, tot_same = oracle.postselect(Pn, S, gm, lo, hi)
        k = float(kept.item())
        assert abs(k - tot_same) <= 1e-12 * max(1.0, tot_same), (gm, k, tot_same)
        assert np.array_equal(masked.cpu().numpy(), np.where(keep, P.cpu().numpy(), 0)), gm
        if Pref is not None:
            _, tot_ref = oracle.postselect(Pref, S, gm, lo, hi)
            assert abs(k - tot_ref) <= 1e-12, (gm, k, tot_ref)
    p.close()


def test_config3_groups_against_marginals_and_partition():
    m, n = 24, 12
    T, U = inputs.first_modes_input(m, n), inputs.haar_unitary(m, 3)
    p, P = _probs(T, U, "c64")
    p.cdf(P)
    pk = p.marginals(P).cpu().numpy()
    for K in (3, 8, 12, 18, 23):
        gm = [-1] * K + [0] * (m - K)
        kept, _, _ = p.postselect(P, gm, [0], [0])
        assert abs(float(kept.item()) - pk[K - 1]) <= 1e-12
    tot = 0.0
    for c in range(n + 1):
        kept, _, _ = p.postselect(P, [0] + [-1] * (m - 1), [c], [c])
        tot += float(kept.item())
    assert abs(tot - pk[-1]) <= 1e-9
    # masked output spot-checked with the host occupation of sampled ranks
    gm = [0, 0, 1, 1, 2, 2] + [-1] * 18
    lo, hi = [1, 0, 0], [1, 1, 2]
    kept, masked, _ = p.postselect(P, gm, lo, hi, masked=True)
    rk = np.random.default_rng(5).integers(0, p.num_outputs, 4000)
    mv = masked[torch.from_numpy(rk).cuda()].cpu().numpy()
    pv = P[torch.from_numpy(rk).cuda()].cpu().numpy()
    for r, a, b in zip(rk, mv, pv):
        s = slos.fock_unrank(m, n, int(r))
        ok = s[0] + s[1] == 1 and s[2] + s[3] <= 1 and s[4] + s[5] <= 2
        assert a == (b if ok else 0.0)
    assert abs(float(kept.item()) - float(masked.double().sum().item())) <= 1e-9
    del masked, P
    torch.cuda.empty_cache()


def test_single_output_plans_and_empty_groups():
    p, P = _probs([0, 0, 0], np.eye(3), "c128")
    kept, _, table = p.postselect(P, [0, 0, -1], [0], [0], ranks=[0])
    assert float(kept.item()) == pytest.approx(1.0) and table.cpu().tolist() == [1.0]
    kept, _, _ = p.postselect(P, [0, 0, -1], [1], [2])
    assert float(kept.item()) == 0.0
    p, P = _probs([3], np.array([[0.6 + 0.8j]]), "c64")
    kept, _, _ = p.postselect(P, [0], [3], [3])
    assert float(kept.item()) == pytest.approx(1.0, abs=1e-6)
