"""GPU test of slos_amplitudes_noalloc, the entry point that allocates nothing.

It is called through the C ABI and compared with slos_amplitudes on the same
plan and unitary: the amplitudes bit for bit and the FP64 sum of P exactly
(same kernels, each output one thread's fixed-order sum, the sum a
fixed-order reduction).  Two calls in a row share the static scratch area, the
second on a smaller plan, so a stale area would show.
"""
import ctypes
import math

import numpy as np
import pytest

from paper_2204_00602_amd import inputs, slos

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    slos.lib()


def _cdt(dtype):
    return torch.complex64 if dtype == "c64" else torch.complex128


def _noalloc(plan, Ud, dtype):
    L = slos.lib()
    out = torch.empty(plan.num_outputs, dtype=_cdt(dtype), device="cuda")
    s = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    rc = L.slos_amplitudes_noalloc(plan._h, ctypes.c_void_p(Ud.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(st))
    assert rc == 0, slos.lib().slos_last_error().decode()
    return out, s


def _reference(plan, Ud, dtype):
    s = torch.zeros(1, dtype=torch.float64, device="cuda")
    out = plan.amplitudes(Ud, sum_p=s)
    return out, s


@pytest.mark.parametrize("first,second", [
    ((12, [1] * 6 + [0] * 6, "c64", True), (8, [1, 0, 2, 0, 1, 0, 0, 0], "c128", False)),
    ((16, [1] * 8 + [0] * 8, "c128", False), (6, [1, 1, 1, 0, 0, 0], "c64", False)),
])
def test_noalloc_matches_slos_amplitudes_on_two_calls(first, second):
    for step, (m, T, dtype, comp) in enumerate((first, second)):
        print(f"[noalloc] call {step}: m={m} T={T} {dtype} comp={comp}", flush=True)
        T = np.array(T, np.int32)
        plan = slos.Plan(T, dtype, compensated=comp)
        U = inputs.haar_unitary(m, 700 + 10 * step + m)
        Ud = torch.from_numpy(U).to(_cdt(dtype)).to("cuda")
        got, s_got = _noalloc(plan, Ud, dtype)
        ref, s_ref = _reference(plan, Ud, dtype)
        torch.cuda.synchronize()
        fl = torch.float32 if dtype == "c64" else torch.float64
        assert torch.equal(got.view(fl), ref.view(fl)), (m, dtype)
        assert float(s_got.item()) == float(s_ref.item())
        tol = 1e-6 if dtype == "c64" else 1e-12
        assert abs(float(s_got.item()) - 1.0) <= tol
        plan.close()


def test_noalloc_rejects_plans_beyond_the_static_area():
    L = slos.lib()
    U = torch.eye(20, dtype=torch.complex64, device="cuda")
    big = slos.Plan([1] * 10 + [0] * 10, "c64")          # layers 8 and 9 alone need ~73 MB
    # full-size buffers, so that the call would stay in bounds even if it ran
    out = torch.empty(big.num_outputs, dtype=torch.complex64, device="cuda")
    rc = L.slos_amplitudes_noalloc(big._h, ctypes.c_void_p(U.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                   None, None)
    assert rc == -2 and b"static area" in L.slos_last_error()
    big.close()
    kept = slos.Plan([1, 1, 0, 0], "c64", keep_layers=True)
    U4 = torch.eye(4, dtype=torch.complex64, device="cuda")
    out = torch.empty(kept.num_outputs, dtype=torch.complex64, device="cuda")
    rc = L.slos_amplitudes_noalloc(kept._h, ctypes.c_void_p(U4.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                   None, None)
    assert rc == -1
    kept.close()
    assert (math.comb(28, 9) + math.comb(27, 8)) * 8 > (32 << 20)
