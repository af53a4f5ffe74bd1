"""GPU invariants that need no oracle, at full size.

* The Fourier suppression law over all 834,451,800 outputs of m = 24, n = 12
  (one photon in every other mode of the 24-mode Fourier interferometer): a(S)
  vanishes unless sum_j j s_j = 0 (mod 12), for the headline variant
  (complex64, compensated) and for complex128.  Every output's class is found
  by unranking its colex rank on the device with the binomial table (the test's
  own arithmetic, not the library's).
* Haar statistics: over 1,000 seeded Haar unitaries at m = 6, n = 3 the mean of
  P(S) is 1/M for every output S, and the mean of P(K) (the probability that
  modes K+1..m are empty) follows Eq. eqhaarpk.
"""
import math

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


def _weight_mod(m, n, lo, hi):
    """sum_j j s_j mod n for the outputs of colex ranks lo..hi-1 (device int64)."""
    rem = torch.arange(lo, hi, dtype=torch.int64, device="cuda")
    q = torch.zeros_like(rem)
    for r in range(n, 0, -1):
        col = torch.tensor([math.comb(c, r) for c in range(m + n - 1)], dtype=torch.int64, device="cuda")
        c = torch.searchsorted(col, rem, right=True) - 1   # the largest c with C(c, r) <= rank
        q += c - (r - 1)                                    # the mode of the r-th photon
        rem -= col[c]
        del c
    assert int(rem.abs().max()) == 0
    return q % n


@pytest.mark.parametrize("dtype,comp", [("c64", True), ("c128", False)])
def test_fourier_suppression_all_outputs_m24_n12(dtype, comp):
    m, n = 24, 12
    F = inputs.fourier_unitary(m)
    T = inputs.periodic_input(m, n)
    print(f"[invariant] Fourier m=24 n=12 {dtype} comp={comp}: all outputs", flush=True)
    p = slos.Plan(T, dtype, compensated=comp)
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    s = torch.zeros(1, dtype=torch.float64, device="cuda")
    out = p.amplitudes(torch.from_numpy(F).to(tdt).cuda(), sum_p=s)
    torch.cuda.synchronize()
    M = p.num_outputs
    worst, allowed_mass, allowed = 0.0, 0.0, 0
    step = 1 << 27
    for lo in range(0, M, step):
        hi = min(M, lo + step)
        q = _weight_mod(m, n, lo, hi)
        P = out[lo:hi].abs().to(torch.float64) ** 2
        zero = q != 0
        if bool(zero.any()):
            worst = max(worst, float(P[zero].max()))
        allowed_mass += float(P[~zero].sum())
        allowed += int((~zero).sum())
        del q, P, zero
    print(f"  allowed outputs {allowed} of {M}, their total P {allowed_mass:.15f}, "
          f"largest suppressed P {worst:.3e}", flush=True)
    # c128: suppressed |a| at rounding level; c64: far below the 1e-5 / M bar
    assert worst <= (1e-26 if dtype == "c128" else 1e-5 / M)
    assert abs(allowed_mass - 1.0) <= (1e-12 if dtype == "c128" else 1e-6)
    assert abs(float(s.item()) - 1.0) <= (1e-12 if dtype == "c128" else 1e-6)
    del out
    p.close()
    torch.cuda.empty_cache()


def test_haar_statistics_m6_n3():
    m, n, N = 6, 3, 1000
    T = [1, 1, 1, 0, 0, 0]
    plan = slos.Plan(T, "c128", options={"max_batch": N})
    U = torch.stack([torch.from_numpy(inputs.haar_unitary(m, 7000 + b)) for b in range(N)]).cuda()
    P = (plan.amplitudes_many(U.contiguous()).abs() ** 2).cpu().numpy()
    M = P.shape[1]
    mean, std = P.mean(axis=0), P.std(axis=0, ddof=1)
    z = np.abs(mean - 1.0 / M) / (std / math.sqrt(N))
    print(f"[invariant] Haar m=6 n=3: max z of mean P(S) vs 1/M over {M} outputs: {z.max():.2f}", flush=True)
    assert z.max() < 5.0
    # P(K): the outputs with modes K..m-1 empty are the first C(K+n-1, n) colex ranks
    for K in range(1, m + 1):
        pk = P[:, : math.comb(K + n - 1, n)].sum(axis=1)
        zk = abs(pk.mean() - oracle.haar_pk_mean(K, m, n)) / (max(pk.std(ddof=1), 1e-300) / math.sqrt(N))
        assert K == m or zk < 5.0, (K, zk)
    plan.close()
