"""One plan, many unitaries: the batched forward and adjoint against the
single-unitary calls (bit for bit) and the oracle."""
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


def _cdt(dtype):
    return torch.complex64 if dtype == "c64" else torch.complex128


@pytest.mark.parametrize("dtype,comp,keep", [("c128", False, False), ("c64", False, False), ("c64", True, False),
                                             ("c64", False, True), ("c128", False, True)])
def test_many_forward_equals_single_calls(dtype, comp, keep):
    m, n, B = 12, 6, 5
    T = inputs.first_modes_input(m, n)
    Us = torch.stack([torch.from_numpy(inputs.haar_unitary(m, 40 + b)) for b in range(B)]).to(_cdt(dtype)).cuda()
    pm = slos.Plan(T, dtype, compensated=comp, keep_layers=keep, options={"max_batch": 8})
    ps = slos.Plan(T, dtype, compensated=comp, keep_layers=keep)
    s = torch.zeros(B, dtype=torch.float64, device="cuda")
    out = pm.amplitudes_many(Us.contiguous(), sum_p=s)
    torch.cuda.synchronize()
    for b in range(B):
        s1 = torch.zeros(1, dtype=torch.float64, device="cuda")
        ref = ps.amplitudes(Us[b].contiguous(), sum_p=s1)
        assert torch.equal(out[b].view(torch.float32 if dtype == "c64" else torch.float64),
                           ref.view(torch.float32 if dtype == "c64" else torch.float64)), b
        assert float(s[b]) == float(s1[0])
    # a smaller batch through the same plan
    out2 = pm.amplitudes_many(Us[:2].contiguous())
    assert torch.equal(out2[1], out[1])


def test_many_probs_and_oracle():
    m, n, B = 6, 3, 3
    T = np.array([1, 1, 1, 0, 0, 0])
    Ush = [inputs.haar_unitary(m, 70 + b) for b in range(B)]
    p = slos.Plan(T, "c128", options={"max_batch": B})
    out = p.amplitudes_many(torch.from_numpy(np.stack(Ush)).cuda())
    S = oracle.fock_states(m, n)
    idx = torch.tensor([slos.fock_rank(x) for x in S], device="cuda")
    for b in range(B):
        ref = oracle.amplitudes(Ush[b], T, S)
        a = out[b][idx].cpu().numpy()
        assert np.abs(a - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_many_backward_equals_single_calls(dtype):
    m, n, B = 12, 6, 4
    T = inputs.first_modes_input(m, n)
    rng = np.random.default_rng(9)
    Us = torch.stack([torch.from_numpy(inputs.haar_unitary(m, 50 + b)) for b in range(B)]).to(_cdt(dtype)).cuda()
    M = slos.fock_count(m, n)
    ga = torch.from_numpy(rng.standard_normal((B, M)) + 1j * rng.standard_normal((B, M))).to(_cdt(dtype)).cuda()
    pm = slos.Plan(T, dtype, keep_layers=True, options={"max_batch": B})
    pm.amplitudes_many(Us.contiguous())
    G = pm.backward_many(Us.contiguous(), ga)
    torch.cuda.synchronize()
    ps = slos.Plan(T, dtype, keep_layers=True)
    for b in range(B):
        ps.amplitudes(Us[b].contiguous())
        g1 = ps.backward(Us[b].contiguous(), ga[b].contiguous())
        assert torch.equal(G[b], g1), b


def test_many_autograd_mesh_gradient_matches_oracle():
    """Config 5 shape (m=12, n=6, 200 targets) for 3 phase sets through the batched path."""
    from paper_2204_00602_amd import autograd as ag
    m, n, B = 12, 6, 3
    k = slos.mesh_mzi_count(m)
    phases = inputs.mesh_phases(B, k, 5)
    teacher = inputs.mesh_phases(B, k, 55)
    targets = inputs.uniform_fock_states(m, n, 200, 505)
    T = inputs.first_modes_input(m, n)
    p_t = np.stack([oracle.probabilities(oracle.clements_unitary(m, teacher[b]), T, targets) for b in range(B)])
    plan = slos.Plan(T, "c128", keep_layers=True, options={"max_batch": B})
    ph = torch.from_numpy(phases).cuda().requires_grad_(True)
    U = ag.mesh(ph, m, "c128")
    a = ag.amplitudes_many(plan, U.contiguous())
    idx = torch.tensor([slos.fock_rank(s) for s in targets], device="cuda")
    P = a[:, idx].abs() ** 2
    loss = ((P - torch.from_numpy(p_t).cuda()) ** 2).sum()
    loss.backward()
    g = ph.grad.cpu().numpy()
    for b in range(B):
        gm = oracle.mesh_grad_phases(phases[b], m, T, targets, p_t[b])
        assert np.abs(g[b] - gm).max() <= 1e-9 * np.abs(gm).max()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_sq_loss_grad_matches_plain_torch(dtype):
    """slos_sq_loss_grad_many against the same loss and gradient written out in
    torch (FP64 P, 4 (P - P_t) a at the targets, zeros elsewhere), for a batch;
    no targets gives zeros and zero loss; a rank outside the outputs is skipped."""
    m, n, B = 8, 4, 3
    T = inputs.first_modes_input(m, n)
    plan = slos.Plan(T, dtype, options={"max_batch": B})
    Us = torch.stack([torch.from_numpy(inputs.haar_unitary(m, 60 + b)) for b in range(B)]).to(_cdt(dtype)).cuda()
    a = plan.amplitudes_many(Us.contiguous())
    M = plan.num_outputs
    ranks = torch.tensor(np.random.default_rng(61).choice(M, 40, replace=False), dtype=torch.int64, device="cuda")
    pt = torch.from_numpy(np.random.default_rng(62).random((B, 40)) * 0.02).cuda()
    g, loss = plan.sq_loss_grad_many(a, ranks, pt)
    torch.cuda.synchronize()
    sel = a[:, ranks]
    d = sel.real.double() ** 2 + sel.imag.double() ** 2 - pt
    want = torch.zeros_like(a)
    want[:, ranks] = (4.0 * d).to(sel.real.dtype) * sel
    if dtype == "c64":
        # FP64 products of FP32 values are exact, so P and the gradient agree bit for bit
        assert torch.equal(g, want)
    else:
        # the kernel may fuse P = x^2 + y^2 into one FMA: a few FP64 roundings per term
        assert torch.equal(g == 0, want == 0)
        assert ((g - want).abs() <= 8 * 2.0 ** -52 * (4.0 * (d.abs() + pt) * sel.abs()).max()).all()
    ref_loss = (d ** 2).sum(1).cpu().numpy()
    assert np.allclose(loss.cpu().numpy(), ref_loss, rtol=1e-13, atol=0)
    # no targets: all zeros, zero loss (the output buffer held garbage before)
    g0 = torch.full_like(a, 7.0)
    _, l0 = plan.sq_loss_grad_many(a, ranks[:0], pt[:, :0], grad_a=g0)
    assert torch.count_nonzero(g0).item() == 0 and float(l0.abs().max()) == 0.0
    # a rank past the last output is skipped; the others are unchanged
    bad = torch.cat([ranks[:5], torch.tensor([M + 3], device="cuda")])
    g1, l1 = plan.sq_loss_grad_many(a, bad, pt[:, :6].contiguous())
    assert torch.equal(g1[:, ranks[:5]], g[:, ranks[:5]])
    assert torch.count_nonzero(g1).item() == torch.count_nonzero(g[:, ranks[:5]]).item()
    d5 = d[:, :5]
    assert np.allclose(l1.cpu().numpy(), (d5 ** 2).sum(1).cpu().numpy(), rtol=1e-13, atol=0)


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-9), ("c64", 1e-4)])
def test_config5_graph_step_replays_match_eager_and_oracle(dtype, tol):
    """The config-5 gradient step (m=12, n=6, 200 targets) recorded into one
    HIP graph: several replays, each on new phases with eager work and
    synchronisation in between, equal the eager step bit for bit; the gradient
    matches the oracle's minor-permanent mesh gradient and the autograd path."""
    from paper_2204_00602_amd import autograd as ag
    m, n, B = 12, 6, 4
    k = slos.mesh_mzi_count(m)
    T = inputs.first_modes_input(m, n)
    targets = inputs.uniform_fock_states(m, n, 200, 505)
    teacher = inputs.mesh_phases(B, k, 55)
    p_t = np.stack([oracle.probabilities(oracle.clements_unitary(m, teacher[b]), T, targets) for b in range(B)])
    idx = torch.tensor([slos.fock_rank(s) for s in targets], device="cuda")
    plan = slos.Plan(T, dtype, keep_layers=True, options={"max_batch": B})
    step = ag.MeshLossGradient(plan, m, B, idx, torch.from_numpy(p_t).cuda(), dtype).capture()
    other = slos.Plan(inputs.first_modes_input(8, 4), "c64")
    U8 = torch.from_numpy(inputs.haar_unitary(8, 1)).to(torch.complex64).cuda()
    for rep in range(3):
        phases = inputs.mesh_phases(B, k, 5 + rep)
        ph = torch.from_numpy(phases).cuda()
        eager = step.eager(ph).clone()
        eager_loss = step.loss()
        torch.cuda.synchronize()
        other.amplitudes(U8)                      # unrelated eager work between replays
        torch.cuda.synchronize()
        got = step.replay(ph).clone()
        torch.cuda.synchronize()
        assert torch.equal(got, eager), rep
        assert step.loss() == eager_loss
        g = got.cpu().numpy()
        for b in (0, B - 1):
            gm = oracle.mesh_grad_phases(phases[b], m, T, targets, p_t[b])
            assert np.abs(g[b] - gm).max() <= tol * np.abs(gm).max(), (rep, b)
    # the same gradient through torch.autograd (one plan, batched)
    ph = torch.from_numpy(phases).cuda().requires_grad_(True)
    plan2 = slos.Plan(T, dtype, keep_layers=True, options={"max_batch": B})
    a = ag.amplitudes_many(plan2, ag.mesh(ph, m, dtype).contiguous())
    loss = ((a[:, idx].abs().double() ** 2 - torch.from_numpy(p_t).cuda()) ** 2).sum()
    loss.backward()
    ga = ph.grad
    assert (ga - got).abs().max().item() <= tol * ga.abs().max().item()


def test_many_edge_cases():
    p = slos.Plan([0, 0, 0], "c128", options={"max_batch": 3})
    out = p.amplitudes_many(torch.eye(3, dtype=torch.complex128, device="cuda").repeat(3, 1, 1).contiguous())
    assert out.cpu().numpy().ravel().tolist() == [1, 1, 1]
    p = slos.Plan([1, 1, 0], "c64", options={"max_batch": 2})
    with pytest.raises(ValueError):
        p.amplitudes_many(torch.eye(3, dtype=torch.complex64, device="cuda").repeat(3, 1, 1).contiguous())
