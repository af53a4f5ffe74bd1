"""A forward pass captured into a HIP graph (slos_plan_capture / replay).

Every replay is checked against the eager pass on the same buffers, with other
eager work on the same plan (another U) between replays, so a graph node that
kept state from an earlier launch would show.  Capture itself must not run
anything, and the replayed amplitudes of a small case match the oracle.
"""
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


def _dev(U, dt):
    return torch.from_numpy(np.ascontiguousarray(U)).to(torch.complex64 if dt == "c64" else torch.complex128).cuda()


def _fwd(plan, U, probs, sum_p):
    return plan.probs(U, sum_p=sum_p) if probs else plan.amplitudes(U, sum_p=sum_p)


@pytest.mark.parametrize("dt,comp,probs", [("c64", True, False), ("c64", False, True), ("c128", False, False),
                                           ("c128", False, True)])
def test_replays_match_eager(dt, comp, probs):
    m, n = 12, 6
    T = inputs.first_modes_input(m, n)
    print(f"[graph] m={m} n={n} {dt} comp={comp} probs={probs}", flush=True)
    plan = slos.Plan(T, dt, compensated=comp)
    U1, U2 = _dev(inputs.haar_unitary(m, 2), dt), _dev(inputs.haar_unitary(m, 9), dt)
    s1 = torch.zeros(1, dtype=torch.float64, device="cuda")
    s2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    ref1 = _fwd(plan, U1, probs, s1).clone()
    ref2 = _fwd(plan, U2, probs, s2).clone()
    torch.cuda.synchronize()
    out = torch.zeros_like(ref1)
    sp = torch.zeros(1, dtype=torch.float64, device="cuda")
    plan.capture(U1, out, sp, probs=probs)
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0 and float(sp.item()) == 0.0  # capture ran nothing
    for rep in range(4):
        plan.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref1), rep
        assert float(sp.item()) == float(s1.item()), rep
        other = _fwd(plan, U2, probs, s2)  # eager work on the same plan between replays
        torch.cuda.synchronize()
        assert torch.equal(other, ref2), rep
        out.zero_()
        sp.zero_()
    plan.close()


def test_replay_batch_of_unitaries_and_oracle():
    m, T = 6, [1, 1, 1, 0, 0, 0]
    plan = slos.Plan(T, "c128", options={"max_batch": 3})
    Us = [inputs.haar_unitary(m, 20 + b) for b in range(3)]
    U = torch.stack([_dev(u, "c128") for u in Us]).contiguous()
    ref = plan.amplitudes_many(U).clone()
    out = torch.zeros_like(ref)
    sp = torch.zeros(3, dtype=torch.float64, device="cuda")
    plan.capture(U, out, sp)
    S = oracle.fock_states(m, 3)
    idx = torch.tensor([slos.fock_rank(s) for s in S], device="cuda")
    for rep in range(3):
        plan.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), rep
        for b in range(3):
            a = out[b][idx].cpu().numpy()
            assert np.abs(a - oracle.amplitudes(Us[b], T, S)).max() < 1e-13
        assert torch.allclose(sp, torch.ones_like(sp), atol=1e-13, rtol=0)
        out.zero_()
    plan.close()


def test_capture_rules():
    plan = slos.Plan([1, 1, 0, 0], "c64")
    U = _dev(inputs.haar_unitary(4, 1), "c64")
    out = torch.zeros(plan.num_outputs, dtype=torch.complex64, device="cuda")
    with pytest.raises(slos.SlosError):
        plan.replay()  # nothing captured yet
    plan.set_timing(True)
    with pytest.raises(slos.SlosError):
        plan.capture(U, out)
    plan.set_timing(False)
    with pytest.raises(ValueError):
        plan.capture(U, torch.zeros(plan.num_outputs, dtype=torch.float32, device="cuda"))  # amplitudes need complex
    plan.capture(U, out)
    plan.replay()
    torch.cuda.synchronize()
    assert torch.equal(out, plan.amplitudes(U))
    plan.close()
