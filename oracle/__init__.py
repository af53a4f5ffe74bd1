"""Plain, slow CPU oracle for the SLOS strong-simulation hot path.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline of bench.py, never by the library.  It shares no code with the HIP
path (it does not import the package, and the package does not import it).

What each function follows (paper = arXiv 2204.00602):
  * amplitudes / probabilities: Section 4.2.1, Eq. eqperm -- a(S) is the
    permanent of U_{T,S} over sqrt(prod s! prod t!), P(S) = |a(S)|^2;
    the permanent itself is computed by the C library (definition, Ryser,
    Glynn; Section 3.2.3 names the latter two).
  * fock_states: the output set S_{m,n} of Section 4.2.1 (all m-tuples of
    non-negative integers summing to n), enumerated by plain recursion.
  * partial_certificate: Eq. eqpk.  haar_pk_mean: Eq. eqhaarpk.
  * beam_splitter_rx: Eq. eq:bs; phase_shifter: the scalar e^{i phi} of
    Section 2; mzi: the BS, PS(phi_a) on mode 0, BS, PS(phi_b) on mode 1
    composition of the Appendix B.2 boson-sampling code.
  * clements_unitary: a rectangular ("square", Section 2) mesh of MZIs; the
    column layout is this project's reading (the paper only cites the mesh).
  * grad_U: d Perm(A)/d A[r][c] is the permanent of the (r, c) minor.
  * slos_recurrence: the paper's own method (Section 3.2.3, SLOS back-end),
    the layered photon-addition recurrence in plain FP64 C with OpenMP: the
    CPU baseline of the method, and a second route to Eq. eqperm's numbers
    that the pins compare with the permanent definition.
  * source_emission / source_events / source_distribution /
    source_performance: the imperfect-source mixture of Section 3.2.4 (emission
    probability, pair emission through g2, indistinguishability), each event's
    output law the convolution of its independent groups, summed over every
    emission event; the readings are stated beside the functions and pinned by
    the CNOT figures printed in Appendix A.4 (Fig. slos_output2).
Parity status: every function here is pinned by tests/test_oracle_pins.py
(closed forms, brute force, the paper's worked examples); none is unpinned.
"""
from __future__ import annotations

import ctypes
import math
import os
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

RYSER, GLYNN, BRUTE = 0, 1, 2
_METHODS = {"ryser": RYSER, "glynn": GLYNN, "brute": BRUTE}


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    lib.oracle_perm.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp]
    lib.oracle_perm.restype = ctypes.c_int
    lib.oracle_amplitudes.argtypes = [ctypes.c_int, ctypes.c_int, dp, ip, ctypes.c_int64,
                                      ip, ctypes.c_int, ctypes.c_int, dp]
    lib.oracle_amplitudes.restype = ctypes.c_int
    lib.oracle_grad_U.argtypes = [ctypes.c_int, ctypes.c_int, dp, ip, ctypes.c_int64,
                                  ip, dp, ctypes.c_int, dp]
    lib.oracle_grad_U.restype = ctypes.c_int
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    for name in ("oracle_slos_all", "oracle_slos_all_ext"):
        getattr(lib, name).argtypes = [ctypes.c_int, dp, ip, dp, dp, ctypes.c_int]
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def num_threads() -> int:
    """Threads the oracle's OpenMP loops use on this host."""
    return int(_load().oracle_num_threads())


def perm(A, method: str = "ryser") -> complex:
    """Permanent of a square complex matrix (brute force = the definition)."""
    A = np.ascontiguousarray(np.asarray(A, dtype=np.complex128))
    n = A.shape[0]
    assert A.shape == (n, n)
    out = np.zeros(2, dtype=np.float64)
    rc = _load().oracle_perm(n, _dptr(A.view(np.float64)), _METHODS[method], _dptr(out))
    if rc != 0:
        raise ValueError(f"oracle_perm failed ({rc}) for n={n}, method={method}")
    return complex(out[0], out[1])


def fock_states(m: int, n: int) -> np.ndarray:
    """All m-tuples of non-negative ints summing to n (the set S_{m,n}).

    Plain recursion, first mode varying slowest; the order carries no meaning.
    """
    out = []

    def rec(prefix, left, modes_left):
        if modes_left == 1:
            out.append(prefix + [left])
            return
        for v in range(left, -1, -1):
            rec(prefix + [v], left - v, modes_left - 1)

    if m == 0:
        return np.zeros((1 if n == 0 else 0, 0), dtype=np.int32)
    rec([], n, m)
    return np.asarray(out, dtype=np.int32).reshape(-1, m)


def amplitudes(U, T, states, method: str = "ryser", threads: int = 0) -> np.ndarray:
    """a(S) = Perm(U_{T,S}) / sqrt(prod s! prod t!) for each row S of `states`.

    U[j, i] is the amplitude from input mode i to output mode j (Eq. eqperm:
    rows of U_{T,S} are rows of U repeated s_j times, columns are columns of U
    repeated t_i times).
    """
    U = np.ascontiguousarray(np.asarray(U, dtype=np.complex128))
    m = U.shape[0]
    assert U.shape == (m, m)
    T = np.ascontiguousarray(np.asarray(T, dtype=np.int32).reshape(m))
    S = np.ascontiguousarray(np.asarray(states, dtype=np.int32).reshape(-1, m))
    n = int(T.sum())
    out = np.zeros(2 * S.shape[0], dtype=np.float64)
    rc = _load().oracle_amplitudes(m, n, _dptr(U.view(np.float64)), _iptr(T), S.shape[0],
                                   _iptr(S), _METHODS[method], int(threads), _dptr(out))
    if rc != 0:
        raise ValueError(f"oracle_amplitudes failed ({rc})")
    return out.view(np.complex128)


def slos_recurrence(U, T, threads: int = 0, extended: bool = False):
    """Every amplitude by the paper's own method, written plainly for the CPU
    (Section 3.2.3, SLOS back-end: photons added one at a time, A_k[t] = sum_j
    U[j, i_k] A_{k-1}[t - e_j], then the sqrt(prod s! / prod t!) factor), in FP64
    with OpenMP over states (extended=True: the layers and sums in long double).
    Returns (a, sum_P) with a[r] the amplitude of the r-th output in colex order
    (see colex_sorted).  A baseline and a second route to Eq. eqperm's numbers;
    the reference where permanents are out of reach (n = 32).
    """
    U = np.ascontiguousarray(np.asarray(U, dtype=np.complex128))
    T = np.ascontiguousarray(np.asarray(T, dtype=np.int32))
    m = T.size
    if U.shape != (m, m):
        raise ValueError("U must be m x m")
    n = int(T.sum())
    out = np.empty(fock_count(m, n), dtype=np.complex128)
    s = ctypes.c_double(0.0)
    fn = _load().oracle_slos_all_ext if extended else _load().oracle_slos_all
    rc = fn(m, _dptr(U.view(np.float64)), _iptr(T), _dptr(out.view(np.float64)), ctypes.byref(s), int(threads))
    if rc != 0:
        raise ValueError(f"oracle_slos_all failed ({rc})")
    return out, s.value


def probabilities(U, T, states, method: str = "ryser", threads: int = 0) -> np.ndarray:
    """P(S) = |a(S)|^2 (Eq. eqperm)."""
    a = amplitudes(U, T, states, method, threads)
    return a.real ** 2 + a.imag ** 2


def partial_certificate(probs, states, K: int) -> float:
    """P(K): total probability that modes K+1..m (1-based) are empty (Eq. eqpk)."""
    states = np.asarray(states)
    mask = np.all(states[:, K:] == 0, axis=1)
    return float(np.sum(np.asarray(probs)[mask]))


def colex_sorted(states) -> np.ndarray:
    """The rows of `states` in colex order: lexicographic on the occupation
    vector read from the last mode (the output order of the strong simulation)."""
    states = np.asarray(states)
    return states[np.lexsort(states.T)]


def inverse_cdf_sample(probs, r) -> np.ndarray:
    """Weak simulation from the strong one (the sampler the paper builds on
    SLOS, Section 3.2): for each uniform r in [0, 1), the index of the first
    output, in the given order, whose cumulative probability exceeds
    r * sum(P).  Cumulative sums in extended precision."""
    c = np.cumsum(np.asarray(probs, dtype=np.longdouble))
    t = np.asarray(r, dtype=np.longdouble) * c[-1]
    idx = np.searchsorted(c, t, side="right")
    return np.minimum(idx, len(c) - 1).astype(np.int64)


def postselect(probs, states, group_of_mode, count_min, count_max):
    """Post-selection over mode groups (heralds and post-selection functions of
    a Processor, Section 3.2.7 and Appendix Processor): state S is kept iff for
    every group g, count_min[g] <= sum of s_j over the modes j of group g <=
    count_max[g] (group -1: unconstrained mode).  Returns (kept mask, sum of P
    over the kept states)."""
    states = np.asarray(states)
    gm = np.asarray(group_of_mode)
    keep = np.ones(states.shape[0], dtype=bool)
    for g in range(len(count_min)):
        c = states[:, gm == g].sum(axis=1)
        keep &= (c >= count_min[g]) & (c <= count_max[g])
    return keep, float(np.sum(np.asarray(probs, dtype=np.float64)[keep]))


def analyze(U, inputs, outputs, expected, group_of_mode, count_min, count_max):
    """Analyzer quantities for logical input/output states: per input, the
    post-selected probability perf(in) and the table P(out | in) / perf(in)
    over the listed outputs; performance = mean perf(in), fidelity = mean of
    the table entry of each input's expected output.  Returns (table,
    performance, fidelity)."""
    m = len(group_of_mode)
    n = int(np.sum(inputs[0]))
    S = fock_states(m, n)
    table = np.zeros((len(inputs), len(outputs)))
    perfs, fids = [], []
    for a, T in enumerate(inputs):
        P = probabilities(U, T, S)
        _, perf = postselect(P, S, group_of_mode, count_min, count_max)
        Po = probabilities(U, T, np.asarray(outputs))
        table[a] = Po / perf
        perfs.append(perf)
        fids.append(table[a, expected[a]])
    return table, float(np.mean(perfs)), float(np.mean(fids))


def haar_pk_mean(K: int, m: int, n: int) -> float:
    """Haar average of P(K): K(K+1)..(K+n-1) / (m(m+1)..(m+n-1)) (Eq. eqhaarpk)."""
    num = 1.0
    den = 1.0
    for r in range(n):
        num *= K + r
        den *= m + r
    return num / den


def beam_splitter_rx(theta: float) -> np.ndarray:
    """Eq. eq:bs: [[cos(theta/2), i sin(theta/2)], [i sin(theta/2), cos(theta/2)]]."""
    c = math.cos(theta / 2.0)
    s = math.sin(theta / 2.0)
    return np.array([[c, 1j * s], [1j * s, c]], dtype=np.complex128)


def phase_shifter(phi: float) -> complex:
    """Section 2: a phase shifter acts on one mode as the scalar e^{i phi}."""
    return complex(math.cos(phi), math.sin(phi))


def mzi(phi_a: float, phi_b: float) -> np.ndarray:
    """BS, then PS(phi_a) on mode 0, then BS, then PS(phi_b) on mode 1.

    Components later in the circuit multiply on the left; BS is Eq. eq:bs at
    theta = pi/2 (a 50:50 splitter).
    """
    bs = beam_splitter_rx(math.pi / 2.0)
    ps0 = np.diag([phase_shifter(phi_a), 1.0]).astype(np.complex128)
    ps1 = np.diag([1.0, phase_shifter(phi_b)]).astype(np.complex128)
    return ps1 @ bs @ ps0 @ bs


def clements_layout(m: int):
    """MZI positions (column, top mode p) of the rectangular mesh, in order.

    Column c (0..m-1) holds MZIs on modes (p, p+1) with p = c mod 2, c mod 2 + 2, ...
    and p + 1 < m: m(m-1)/2 MZIs in total.
    """
    return [(c, p) for c in range(m) for p in range(c % 2, m - 1, 2)]


def clements_unitary(m: int, phases) -> np.ndarray:
    """U of the mesh: phases[2k], phases[2k+1] = (phi_a, phi_b) of MZI k.

    Each MZI is embedded on its mode pair and applied in layout order, so the
    first MZI is the right-most factor.
    """
    layout = clements_layout(m)
    phases = np.asarray(phases, dtype=np.float64).reshape(-1)
    assert phases.size == 2 * len(layout)
    U = np.eye(m, dtype=np.complex128)
    for k, (_, p) in enumerate(layout):
        B = mzi(phases[2 * k], phases[2 * k + 1])
        E = np.eye(m, dtype=np.complex128)
        E[p:p + 2, p:p + 2] = B
        U = E @ U
    return U


def grad_U(U, T, states, w, threads: int = 0) -> np.ndarray:
    """G[j, i] = sum_S w_S * conj(d a(S)/d U[j, i]) via minor permanents.

    With w_S the PyTorch-convention gradient of a real loss with respect to
    a(S), G is the PyTorch-convention gradient with respect to U.
    """
    U = np.ascontiguousarray(np.asarray(U, dtype=np.complex128))
    m = U.shape[0]
    T = np.ascontiguousarray(np.asarray(T, dtype=np.int32).reshape(m))
    S = np.ascontiguousarray(np.asarray(states, dtype=np.int32).reshape(-1, m))
    w = np.ascontiguousarray(np.asarray(w, dtype=np.complex128).reshape(-1))
    assert w.shape[0] == S.shape[0]
    n = int(T.sum())
    G = np.zeros(2 * m * m, dtype=np.float64)
    rc = _load().oracle_grad_U(m, n, _dptr(U.view(np.float64)), _iptr(T), S.shape[0],
                               _iptr(S), _dptr(w.view(np.float64)), int(threads), _dptr(G))
    if rc != 0:
        raise ValueError(f"oracle_grad_U failed ({rc})")
    return G.view(np.complex128).reshape(m, m)


def mesh_loss(phases, m, T, targets, p_target) -> float:
    """L = sum_S (P(S) - P_target(S))^2 over the target outputs, one phase set."""
    U = clements_unitary(m, phases)
    P = probabilities(U, T, targets)
    return float(np.sum((P - np.asarray(p_target)) ** 2))


def mesh_grad_phases(phases, m, T, targets, p_target) -> np.ndarray:
    """dL/dphases through the minor-permanent gradient and the mesh Jacobian."""
    phases = np.asarray(phases, dtype=np.float64).reshape(-1)
    U = clements_unitary(m, phases)
    a = amplitudes(U, T, targets)
    P = a.real ** 2 + a.imag ** 2
    dLdP = 2.0 * (P - np.asarray(p_target))
    w = 2.0 * a * dLdP                    # PyTorch convention for d/d conj(a)
    G = grad_U(U, T, targets, w)
    return mesh_vjp(phases, m, G)


def mesh_vjp(phases, m, G) -> np.ndarray:
    """dL/dphi = Re sum_{j,i} conj(G[j,i]) dU[j,i]/dphi for every mesh phase,
    with dU/dphi from the closed form of each MZI factor
    (d/dphi e^{i phi} = i e^{i phi}) and G = dL/dRe U + i dL/dIm U."""
    phases = np.asarray(phases, dtype=np.float64).reshape(-1)
    G = np.asarray(G, dtype=np.complex128)
    layout = clements_layout(m)
    factors = []
    for k, (_, p) in enumerate(layout):
        E = np.eye(m, dtype=np.complex128)
        E[p:p + 2, p:p + 2] = mzi(phases[2 * k], phases[2 * k + 1])
        factors.append(E)
    # prefix/suffix products: U = F_{K-1} ... F_0
    K = len(factors)
    right = [np.eye(m, dtype=np.complex128)]          # right[k] = F_{k-1}..F_0
    for k in range(K):
        right.append(factors[k] @ right[-1])
    left = [np.eye(m, dtype=np.complex128)] * (K + 1)  # left[k] = F_{K-1}..F_{k+1}
    acc = np.eye(m, dtype=np.complex128)
    for k in range(K - 1, -1, -1):
        left[k] = acc
        acc = acc @ factors[k]
    grad = np.zeros(2 * K)
    bs = beam_splitter_rx(math.pi / 2.0)
    for k, (_, p) in enumerate(layout):
        pa, pb = phases[2 * k], phases[2 * k + 1]
        ps0 = np.diag([phase_shifter(pa), 1.0])
        ps1 = np.diag([1.0, phase_shifter(pb)])
        dps0 = np.diag([1j * phase_shifter(pa), 0.0])
        dps1 = np.diag([0.0, 1j * phase_shifter(pb)])
        for which, dB in ((0, ps1 @ bs @ dps0 @ bs), (1, dps1 @ bs @ ps0 @ bs)):
            dE = np.zeros((m, m), dtype=np.complex128)
            dE[p:p + 2, p:p + 2] = dB
            dU = left[k] @ dE @ right[k]
            grad[2 * k + which] = float(np.real(np.sum(np.conj(G) * dU)))
    return grad


def mesh_grad_phases_fd(phases, m, T, targets, p_target, h: float = 1e-6) -> np.ndarray:
    """Central finite differences of mesh_loss in FP64."""
    phases = np.asarray(phases, dtype=np.float64).reshape(-1).copy()
    g = np.zeros_like(phases)
    for k in range(phases.size):
        old = phases[k]
        phases[k] = old + h
        lp = mesh_loss(phases, m, T, targets, p_target)
        phases[k] = old - h
        lm = mesh_loss(phases, m, T, targets, p_target)
        phases[k] = old
        g[k] = (lp - lm) / (2.0 * h)
    return g


def fock_count(m: int, n: int) -> int:
    """|S_{m,n}| = C(m+n-1, n) (Section 4.2.2)."""
    return math.comb(m + n - 1, n)


def derangements(n: int) -> int:
    """!n by the recurrence !n = (n-1)(!(n-1) + !(n-2)), used as a permanent pin."""
    if n == 0:
        return 1
    a, b = 1, 0  # !0, !1
    for k in range(2, n + 1):
        a, b = b, (k - 1) * (a + b)
    return b


def fibonacci(n: int) -> int:
    f0, f1 = 0, 1
    for _ in range(n):
        f0, f1 = f1, f0 + f1
    return f0


__all__ = [
    "perm", "fock_states", "amplitudes", "probabilities", "partial_certificate",
    "haar_pk_mean", "beam_splitter_rx", "phase_shifter", "mzi", "clements_layout",
    "clements_unitary", "grad_U", "mesh_loss", "mesh_grad_phases", "mesh_grad_phases_fd", "mesh_vjp",
    "fock_count", "derangements", "fibonacci", "num_threads",
]


# ---------------------------------------------------------------------------
# Imperfect sources (Section 3.2.4: the source model tunes emission
# probability, multi-photon emission and indistinguishability; Appendix A.4
# prints the performance of the Ralph CNOT under such sources).
#
# Readings (the paper names the parameters and prints their effect on one
# gate, but gives no formulas):
#   * every photon of the input T comes from a source of its own;
#   * a source emits nothing, one photon or two, with P(>= 1) = beta (the
#     emission probability) and g2 = 2 p2 / (p1 + 2 p2)^2 (the second-order
#     autocorrelation of the emitted light, "multiphoton_component");
#   * the first photon of an emission shares the common wavepacket with
#     probability sqrt(V), else it is distinguishable from every other photon,
#     so two emitted photons interfere with probability V (the HOM visibility);
#   * the second photon of a two-photon emission is distinguishable from every
#     other photon.
# Photons of different wavepackets do not interfere: the output distribution
# of one emission event is the convolution of the distributions of its groups
# of indistinguishable photons (each group's by Eq. eqperm).
# ---------------------------------------------------------------------------

def source_emission(beta: float, g2: float):
    """(p0, p1, p2) of one source: p1 + p2 = beta and 2 p2 / (p1 + 2 p2)^2 = g2.

    Solving the second for p2 with p1 = beta - p2 gives the quadratic
    g2 p2^2 - (1 - beta g2) p2 + beta^2 g2 / 2 = 0, whose smaller root is taken
    (the one that vanishes with g2)."""
    if g2 == 0.0:
        p2 = 0.0
    else:
        p2 = (1.0 - beta * g2 - math.sqrt(1.0 - 2.0 * beta * g2)) / g2
    return 1.0 - beta, beta - p2, p2


def _states_index(m: int, n: int):
    S = fock_states(m, n)
    return S, {tuple(int(v) for v in s): i for i, s in enumerate(S)}


def source_events(T, beta: float, g2: float, V: float):
    """All emission events of the sources behind input T, with their weights.

    Each event is (weight, main, dist): `main` is the occupation vector of the
    photons in the common wavepacket and `dist` the input modes of the
    distinguishable photons.  Per source, in this order: nothing; one photon,
    common; one photon, distinguishable; two photons, the first common; two
    photons, the first distinguishable (the second is always distinguishable).
    """
    T = [int(v) for v in T]
    m = len(T)
    modes = [i for i in range(m) for _ in range(T[i])]
    p0, p1, p2 = source_emission(beta, g2)
    x = math.sqrt(V)
    outcomes = [(p0, 0, 0), (p1 * x, 1, 0), (p1 * (1 - x), 0, 1), (p2 * x, 1, 1), (p2 * (1 - x), 0, 2)]
    events = []

    def rec(s, w, main, dist):
        if s == len(modes):
            events.append((w, tuple(main), tuple(dist)))
            return
        for ws, in_main, ndist in outcomes:
            if ws == 0.0:
                continue
            main2 = list(main)
            main2[modes[s]] += in_main
            rec(s + 1, w * ws, main2, dist + [modes[s]] * ndist)

    rec(0, 1.0, [0] * m, [])
    return events


def source_distribution(U, T, beta: float, g2: float, V: float, nmax: int):
    """Output distribution of the imperfect-source mixture, photon numbers
    0..nmax: a list whose entry N is (states, probs) over S_{m,N} (fock_states
    order).  Sum over the emission events of weight x the convolution of the
    common group's P (Eq. eqperm, by permanents) with one |U[:, i]|^2 per
    distinguishable photon; counts above nmax are dropped."""
    U = np.asarray(U, dtype=np.complex128)
    m = U.shape[0]
    Q = np.abs(U) ** 2
    idx = [_states_index(m, N) for N in range(nmax + 1)]
    out = [np.zeros(len(idx[N][0])) for N in range(nmax + 1)]
    main_cache = {}
    for w, main, dist in source_events(T, beta, g2, V):
        nm = sum(main)
        if nm > nmax:
            continue
        if main not in main_cache:
            main_cache[main] = probabilities(U, np.asarray(main), idx[nm][0])
        cur = {tuple(int(v) for v in s): p for s, p in zip(idx[nm][0], main_cache[main])}
        for i in dist:
            if sum(next(iter(cur))) + 1 > nmax:
                cur = None
                break
            nxt = {}
            for s, p in cur.items():
                for j in range(m):
                    if Q[j, i] == 0.0:
                        continue
                    t = list(s)
                    t[j] += 1
                    t = tuple(t)
                    nxt[t] = nxt.get(t, 0.0) + p * Q[j, i]
            cur = nxt
        if cur is None:
            continue
        N = nm + len(dist)
        for s, p in cur.items():
            out[N][idx[N][1][s]] += w * p
    return [(idx[N][0], out[N]) for N in range(nmax + 1)]


def source_performance(dist, group_of_mode, count_min, count_max, min_modes: int):
    """Processor figures over a graded distribution (list of (states, probs)):
    physical = total probability of the outputs with at least `min_modes`
    occupied modes; kept = the part of it whose mode groups hold between
    count_min[g] and count_max[g] photons.  The gate performance is kept /
    physical."""
    g = np.asarray(group_of_mode)
    phys = kept = 0.0
    for states, probs in dist:
        if len(states) == 0:
            continue
        occ = (states > 0).sum(axis=1) >= min_modes
        ok = occ.copy()
        for k in range(len(count_min)):
            c = states[:, g == k].sum(axis=1)
            ok &= (c >= count_min[k]) & (c <= count_max[k])
        phys += float(np.sum(probs[occ]))
        kept += float(np.sum(probs[ok]))
    return phys, kept


def source_probability(U, T, beta: float, g2: float, V: float, S) -> float:
    """P(S) of the imperfect-source mixture for one output S, by the event sum:
    sum over emission events of weight x sum over the splits S = S' + R of the
    common group's P(S') (Eq. eqperm) times the law of the distinguishable
    photons, Perm(|U|^2 restricted to rows R and their input columns) / prod R!
    (independent particles).  Independent of source_distribution's convolutions."""
    U = np.asarray(U, dtype=np.complex128)
    m = U.shape[0]
    Q = (np.abs(U) ** 2).astype(np.complex128)
    S = [int(v) for v in S]
    N = sum(S)
    pm_cache, qd_cache = {}, {}

    def subs(k):
        out = []

        def rec(j, left, cur):
            if j == m:
                if left == 0:
                    out.append(tuple(cur))
                return
            for v in range(min(S[j], left) + 1):
                rec(j + 1, left - v, cur + [v])

        rec(0, k, [])
        return out

    total = 0.0
    for w, main, dist in source_events(T, beta, g2, V):
        nm = sum(main)
        if nm + len(dist) != N:
            continue
        for Sp in subs(nm):
            key = (main, Sp)
            if key not in pm_cache:
                pm_cache[key] = float(probabilities(U, np.asarray(main), np.asarray([Sp]))[0])
            pm = pm_cache[key]
            if pm == 0.0:
                continue
            R = tuple(s - sp for s, sp in zip(S, Sp))
            dkey = (tuple(sorted(dist)), R)
            if dkey not in qd_cache:
                rows = [j for j in range(m) for _ in range(R[j])]
                sub = Q[np.ix_(rows, list(dkey[0]))] if rows else np.zeros((0, 0), np.complex128)
                fac = float(np.prod([math.factorial(r) for r in R]))
                qd_cache[dkey] = perm(sub).real / fac
            total += w * pm * qd_cache[dkey]
    return total
