"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these compares the oracle with itself: each checks a closed form, an
invariant, an identity stated in the paper, a library routine, or finite
differences, chosen so that a dropped term, a wrong sign, a wrong index or a
transposed operand in the oracle fails at least one of them.
"""
import numpy as np
import pytest
import scipy.interpolate as si
import scipy.linalg as sla

import oracle
from workloads import (System, basis_density_matrices, ensemble_state, gate_initial_states, observable_nm,
                       random_alpha, random_pure_states, random_system)


def mk(nlev, *, det=None, sk=None, ck=None, T1=None, T2=None, Ns=5, car=None, T=4.0, NT=40):
    Q = len(nlev)
    return System(nlev=tuple(nlev),
                  detuning=np.zeros(Q) if det is None else np.asarray(det, float),
                  selfkerr=np.zeros(Q) if sk is None else np.asarray(sk, float),
                  crosskerr=np.zeros((Q, Q)) if ck is None else np.asarray(ck, float),
                  T1=np.full(Q, np.inf) if T1 is None else np.asarray(T1, float),
                  T2=np.full(Q, np.inf) if T2 is None else np.asarray(T2, float),
                  Ns=Ns, carriers=np.zeros((Q, 1)) if car is None else np.asarray(car, float),
                  T=float(T), NT=int(NT))


def proj(N, k):
    r = np.zeros((N, N), complex)
    r[k, k] = 1
    return r


# ------------------------------------------------------------ operators

def test_lowering_and_subsystem_order():
    # a|k> = sqrt(k)|k-1>; subsystem 0 is the most significant digit.
    a = oracle.lowering(4)
    for k in range(1, 4):
        e = np.zeros(4)
        e[k] = 1
        out = a @ e
        assert out[k - 1] == pytest.approx(np.sqrt(k)) and np.count_nonzero(out) == 1
    nlev = (2, 3)
    a0 = oracle.embed(oracle.lowering(2), 0, nlev)
    a1 = oracle.embed(oracle.lowering(3), 1, nlev)
    # |1,2> has index 1*3 + 2 = 5; a0|1,2> = |0,2> (index 2), a1|1,2> = sqrt2 |1,1> (index 4)
    e = np.zeros(6)
    e[5] = 1
    assert np.allclose(a0 @ e, np.eye(6)[2])
    assert np.allclose(a1 @ e, np.sqrt(2) * np.eye(6)[4])


def test_system_energies_by_hand():
    # H_sys of Sec. II is diagonal with cross-Kerr only; expand it by hand
    # for |n0, n1> = |2, 3> in a 3x4 system.
    s = mk((3, 4), det=[0.1, -0.2], sk=[0.3, 0.25], ck=[[0, 0.05], [0, 0]])
    H = oracle.system_hamiltonian(s)
    assert np.allclose(H, np.diag(np.diag(H)))
    n0, n1 = 2, 3
    E = 0.1 * n0 - 0.3 / 2 * n0 * (n0 - 1) + (-0.2) * n1 - 0.25 / 2 * n1 * (n1 - 1) - 0.05 * n0 * n1
    assert H[n0 * 4 + n1, n0 * 4 + n1] == pytest.approx(2 * np.pi * E, rel=1e-15)
    Hs = oracle.system_hamiltonian(s, sparse=True).toarray()
    assert np.allclose(Hs, H, atol=1e-15)


def test_bspline_partition_of_unity_and_scipy_basis():
    s = mk((2,), Ns=9, T=7.0)
    t = np.linspace(0.0, 7.0, 1001)
    tot = sum(oracle.spline_basis(s, k, t) for k in range(s.Ns))
    assert np.max(np.abs(tot - 1.0)) < 1e-14
    dtau = s.T / (s.Ns - 2)
    for k in range(s.Ns):
        c = (k - 0.5) * dtau
        knots = c + dtau * np.array([-1.5, -0.5, 0.5, 1.5])
        ref = si.BSpline.basis_element(knots, extrapolate=False)(t)
        ref = np.nan_to_num(ref)
        assert np.max(np.abs(ref - oracle.spline_basis(s, k, t))) < 1e-14


def test_controls_constant_alpha_is_constant_drive():
    s = mk((2,), Ns=6, T=3.0, car=[[0.0, 0.02]])
    alpha = np.zeros((1, 6, 2, 2))
    alpha[0, :, 0, 0] = 0.004
    alpha[0, :, 0, 1] = -0.003
    for t in np.linspace(0, 3.0, 17):
        d = oracle.controls(s, alpha, t)
        assert d[0] == pytest.approx(2 * np.pi * (0.004 - 0.003j), rel=1e-14)
    # a single carrier at Omega contributes alpha * exp(i 2 pi Omega t)
    alpha2 = np.zeros((1, 6, 2, 2))
    alpha2[0, :, 1, 0] = 0.001
    t = 1.3
    assert oracle.controls(s, alpha2, t)[0] == pytest.approx(
        2 * np.pi * 0.001 * np.exp(1j * 2 * np.pi * 0.02 * t), rel=1e-14)


# ------------------------------------------------------------ dynamics pins

def test_t1_decay_discrete_closed_form_and_continuum():
    T1 = 7.0
    for n in (2, 3):
        s = mk((n,), T1=[T1], det=[0.11], T=5.0, NT=50)
        alpha = np.zeros((1, s.Ns, 1, 2))
        rhoT, st = oracle.imr_forward(s, alpha, proj(n, 1)[None], keep_states=True)
        h = s.dt / 2
        R = (1 - h / T1) / (1 + h / T1)
        for j, r in enumerate(st):
            assert r[0, 1, 1].real == pytest.approx(R ** j, abs=1e-14)
            assert r[0, 0, 0].real == pytest.approx(1 - R ** j, abs=1e-14)
    # continuum e^{-t/T1}: second order in dt
    errs = []
    for NT in (20, 40):
        s = mk((2,), T1=[T1], T=5.0, NT=NT)
        r = oracle.imr_forward(s, np.zeros((1, s.Ns, 1, 2)), proj(2, 1)[None])
        errs.append(abs(r[0, 1, 1].real - np.exp(-5.0 / T1)))
    assert 3.6 < errs[0] / errs[1] < 4.4


def test_dephasing_rate_and_detuning_phase():
    # rho01 obeys d/dt rho01 = (i 2 pi delta - 1/(2 T1) - 1/(2 T2)) rho01 for
    # L2 = a^+a / sqrt(T2) (the paper's dephasing operator) and a 2-level system.
    T1, T2, dl = 9.0, 5.0, 0.07
    s = mk((2,), T1=[T1], T2=[T2], det=[dl], T=4.0, NT=64)
    psi = np.array([1, 1]) / np.sqrt(2)
    rho0 = np.outer(psi, psi)[None].astype(complex)
    lam = 1j * 2 * np.pi * dl - 0.5 / T1 - 0.5 / T2
    h = s.dt / 2
    R = (1 + h * lam) / (1 - h * lam)
    _, st = oracle.imr_forward(s, np.zeros((1, s.Ns, 1, 2)), rho0, keep_states=True)
    for j, r in enumerate(st):
        assert abs(r[0, 0, 1] - 0.5 * R ** j) < 1e-14
    assert abs(st[-1][0, 0, 1] - 0.5 * np.exp(lam * s.T)) < 1e-3


def test_t1_cascade_continuum():
    # 3 levels from |2>: rho22 = e^{-2t/T1}, rho11 = 2(e^{-t/T1} - e^{-2t/T1});
    # this pins the jump weight sqrt((n+1)(m+1)).
    T1, T = 6.0, 4.0
    errs = []
    for NT in (25, 50):
        s = mk((3,), T1=[T1], T=T, NT=NT)
        r = oracle.imr_forward(s, np.zeros((1, s.Ns, 1, 2)), proj(3, 2)[None])[0]
        e22 = abs(r[2, 2] - np.exp(-2 * T / T1))
        e11 = abs(r[1, 1] - 2 * (np.exp(-T / T1) - np.exp(-2 * T / T1)))
        errs.append(max(e11, e22))
        assert abs(np.trace(r) - 1) < 1e-14
    assert errs[1] < 1e-4
    assert 3.6 < errs[0] / errs[1] < 4.4


@pytest.mark.parametrize("ar,ai", [(0.01, 0.0), (0.006, -0.008)])
def test_rabi_closed_two_level(ar, ai):
    # Constant drive d (all coefficients equal, partition of unity); H = d a + d* a^+
    # rotates the Bloch vector at rate 2|d|; IMR turns it by 2 atan(|d| dt) per step.
    s = mk((2,), Ns=5, T=30.0, NT=300)
    alpha = np.zeros((1, 5, 1, 2))
    alpha[..., 0] = ar
    alpha[..., 1] = ai
    dabs = 2 * np.pi * abs(ar + 1j * ai)
    _, st = oracle.imr_forward(s, alpha, proj(2, 0)[None], keep_states=True)
    for j in range(0, 301, 10):
        assert st[j][0, 1, 1].real == pytest.approx(np.sin(j * np.arctan(dabs * s.dt)) ** 2, abs=1e-13)
    assert abs(st[-1][0, 1, 1].real - np.sin(dabs * s.T) ** 2) < 5e-3


@pytest.mark.parametrize("ar,ai", [(0.006, -0.008), (-0.002, 0.009)])
def test_control_coupling_orientation_closed_two_level(ar, ai):
    # H_c = d a + conj(d) a^+ (Sec. II).  From |0><0| under a constant complex
    # d the exact solution has psi_1 = -i (conj(d)/|d|) sin(|d| t), so
    # rho_10 = -i (conj(d)/|d|) sin(|d| t) cos(|d| t).  M is normal with
    # eigenvalues 0 and -+2i|d|, which IMR maps to rotations by
    # 2 atan(|d| dt) per step: rho_10^j = -i (conj(d)/|d|) sin(phi_j) cos(phi_j)
    # with phi_j = j atan(|d| dt).  The phase of rho_10 fixes which of d and
    # conj(d) multiplies the lowering operator; P1 alone depends on |d| only.
    s = mk((2,), Ns=5, T=12.0, NT=120)
    alpha = np.zeros((1, 5, 1, 2))
    alpha[..., 0] = ar
    alpha[..., 1] = ai
    d = 2 * np.pi * (ar + 1j * ai)
    _, st = oracle.imr_forward(s, alpha, proj(2, 0)[None], keep_states=True)
    for j in range(0, 121, 5):
        phi = j * np.arctan(abs(d) * s.dt)
        ref = -1j * (np.conj(d) / abs(d)) * np.sin(phi) * np.cos(phi)
        assert abs(st[j][0, 1, 0] - ref) < 1e-13
        assert abs(st[j][0, 0, 1] - np.conj(ref)) < 1e-13


def test_trace_hermiticity_and_closed_norm():
    rng = np.random.default_rng(5)
    s = random_system(rng, (2, 3), NT=30, T=3.0)
    alpha = random_alpha(rng, s, amp=0.05)
    X = rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6))
    rho0 = X @ X.conj().T
    rho0 /= np.trace(rho0)
    _, st = oracle.imr_forward(s, alpha, rho0[None], keep_states=True)
    for r in st:
        assert abs(np.trace(r[0]) - 1) < 1e-13
        assert np.max(np.abs(r[0] - r[0].conj().T)) < 1e-14
    sc = mk((2, 3), det=s.detuning, sk=s.selfkerr, ck=s.crosskerr, Ns=s.Ns,
            car=s.carriers, T=s.T, NT=s.NT)
    _, st = oracle.imr_forward(sc, alpha, rho0[None], keep_states=True)
    n0 = np.linalg.norm(rho0)
    for r in st:
        assert abs(np.linalg.norm(r[0]) - n0) < 1e-13


def test_imr_against_matrix_exponential():
    # Constant M (constant drive): IMR error against expm(M T) is O(dt^2).
    rng = np.random.default_rng(11)
    base = random_system(rng, (2, 2), NT=10, T=2.0, Nf=1, some_terms_off=False)
    alpha = np.zeros((2, base.Ns, 1, 2))
    alpha[0, ..., 0] = 0.02
    alpha[1, ..., 1] = -0.015
    rho0 = proj(4, 0)[None]
    M = oracle.superoperator(base, alpha, 0.3)
    exact = oracle.unvec(sla.expm(M * base.T) @ oracle.vec(rho0[0]), 4)
    errs = []
    for NT in (20, 40):
        s = mk((2, 2), det=base.detuning, sk=base.selfkerr, ck=base.crosskerr,
               T1=base.T1, T2=base.T2, Ns=base.Ns, T=base.T, NT=NT)
        r = oracle.imr_forward(s, alpha, rho0)[0]
        errs.append(np.linalg.norm(r - exact))
    assert 3.6 < errs[0] / errs[1] < 4.4


def test_one_step_is_cayley_map():
    rng = np.random.default_rng(3)
    s = random_system(rng, (3, 2), NT=1, T=0.3)
    alpha = random_alpha(rng, s, amp=0.05)
    X = rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6))
    M = oracle.superoperator(s, alpha, 0.15)
    h = 0.15
    I = np.eye(36)
    ref = np.linalg.solve(I - h * M, (I + h * M) @ oracle.vec(X))
    out = oracle.imr_forward(s, alpha, X[None])[0]
    assert np.max(np.abs(oracle.vec(out) - ref)) < 1e-14 * np.max(np.abs(ref))


@pytest.mark.parametrize("jc", [0.0, 0.03])
def test_dense_and_operator_forms_agree_and_adjoint_identity(jc):
    rng = np.random.default_rng(7)
    s = random_system(rng, (3, 2, 2), NT=4, T=1.0, jc=jc)
    alpha = random_alpha(rng, s, amp=0.05)
    N = s.N
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    Y = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    t = 0.37
    M = oracle.superoperator(s, alpha, t)
    op = oracle.lindbladian(s, alpha, t, X)
    assert np.max(np.abs(M @ oracle.vec(X) - oracle.vec(op))) < 1e-13
    adj = oracle.lindbladian_adjoint(s, alpha, t, Y)
    assert np.max(np.abs(M.conj().T @ oracle.vec(Y) - oracle.vec(adj))) < 1e-13
    lhs = np.vdot(Y, op)
    rhs = np.vdot(adj, X)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # selected entries one by one
    rows = rng.integers(0, N, 20)
    cols = rng.integers(0, N, 20)
    ent = oracle.lindbladian_entries(s, alpha, t, X, rows, cols)
    assert np.max(np.abs(ent - op[rows, cols])) < 1e-13
    ent = oracle.lindbladian_entries(s, alpha, t, Y, rows, cols, adjoint=True)
    assert np.max(np.abs(ent - adj[rows, cols])) < 1e-13


@pytest.mark.parametrize("jc", [0.0, 0.03])
def test_lindbladian_trace_zero_and_hermiticity_preserving(jc):
    rng = np.random.default_rng(8)
    s = random_system(rng, (3, 3), NT=4, T=1.0, jc=jc)
    alpha = random_alpha(rng, s, amp=0.05)
    X = rng.standard_normal((9, 9)) + 1j * rng.standard_normal((9, 9))
    Hm = X + X.conj().T
    out = oracle.lindbladian(s, alpha, 0.2, Hm)
    assert abs(np.trace(out)) < 1e-12
    assert np.max(np.abs(out - out.conj().T)) < 1e-12


# ------------------------------------------------------------ Jaynes-Cummings coupling

def mk_jc(nlev, g, *, rot=None, det=None, T, NT):
    """Closed system with one coupling g_10 (subsystem 1 > subsystem 0)."""
    import dataclasses
    Q = len(nlev)
    jc = np.zeros((Q, Q))
    jc[1, 0] = g
    return dataclasses.replace(mk(nlev, det=det, T=T, NT=NT), jc=jc,
                               rotfreq=None if rot is None else np.asarray(rot, float))


def test_jaynes_cummings_single_excitation_closed_form():
    # Two qubits, one excitation, equal rotation frequencies: H = G (|10><01|
    # + |01><10|) on the span of |10> (index 2) and |01> (index 1), G = 2 pi g.
    # One implicit-midpoint step is the Cayley map, so after j steps
    # psi = cos(phi_j)|10> - i sin(phi_j)|01>, phi_j = j atan(G dt).
    g = 0.013
    s = mk_jc((2, 2), g, T=10.0, NT=100)
    _, st = oracle.imr_forward(s, np.zeros((2, 5, 1, 2)), proj(4, 2)[None], keep_states=True)
    for j in (1, 37, 100):
        ph = j * np.arctan(2 * np.pi * g * s.dt)
        r = st[j][0]
        assert abs(r[2, 2] - np.cos(ph) ** 2) < 1e-14
        assert abs(r[1, 1] - np.sin(ph) ** 2) < 1e-14
        assert abs(r[2, 1] - 1j * np.sin(ph) * np.cos(ph)) < 1e-14
        assert abs(r[1, 2] + 1j * np.sin(ph) * np.cos(ph)) < 1e-14
        assert abs(r[0, 0]) + abs(r[3, 3]) < 1e-15


def test_jaynes_cummings_two_excitations_closed_form():
    # Two qutrits from |1,1> (index 4): the coupling mixes |2,0>, |1,1>, |0,2>
    # with weights sqrt(2) (a^+|1> = sqrt2|2>), eigenvalues 0 and +-2G, so
    # P_11 = cos^2(j atan(2 G dt)) and P_20 = P_02 = sin^2(j atan(2 G dt)) / 2.
    g = 0.011
    s = mk_jc((3, 3), g, T=8.0, NT=80)
    _, st = oracle.imr_forward(s, np.zeros((2, 5, 1, 2)), proj(9, 4)[None], keep_states=True)
    for j in (1, 20, 80):
        th = j * np.arctan(2 * 2 * np.pi * g * s.dt)
        r = st[j][0]
        assert abs(r[4, 4] - np.cos(th) ** 2) < 1e-14
        assert abs(r[6, 6] - 0.5 * np.sin(th) ** 2) < 1e-14
        assert abs(r[2, 2] - 0.5 * np.sin(th) ** 2) < 1e-14


def test_jaynes_cummings_rotating_frame_covariance():
    # Sec. II: in a frame rotating at w_q^rot the detunings become
    # w_q - w_q^rot and the coupling picks up exp(+-i (w_p^rot - w_q^rot) t).
    # The lab-frame state U rho_rot U^+ (U = exp(-i sum_q w_q^rot n_q t)) must
    # equal the rotating-frame one up to the O(dt^2) error of the method; a
    # coupling phase of the wrong sign misses by O(1) (about 0.5 here).
    om = [0.05, -0.03]
    rng = np.random.default_rng(4)
    psi = rng.standard_normal(6) + 1j * rng.standard_normal(6)
    psi /= np.linalg.norm(psi)
    rho0 = np.outer(psi, psi.conj())[None]
    a = np.zeros((2, 5, 1, 2))
    lab = oracle.imr_forward(mk_jc((2, 3), 0.02, det=om, T=20.0, NT=4000), a, rho0)[0]
    rot = oracle.imr_forward(mk_jc((2, 3), 0.02, rot=om, T=20.0, NT=4000), a, rho0)[0]
    theta = np.array([2 * np.pi * (om[0] * (i // 3) + om[1] * (i % 3)) * 20.0 for i in range(6)])
    pred = np.exp(1j * theta)[:, None] * lab * np.exp(-1j * theta)[None, :]
    assert np.max(np.abs(pred - rot)) < 2e-5


def test_jaynes_cummings_gradient_against_central_differences():
    rng = np.random.default_rng(19)
    s = random_system(rng, (2, 3), NT=8, T=0.8, jc=0.05)
    alpha = random_alpha(rng, s, amp=0.05)
    rho0 = np.stack([proj(6, 1), proj(6, 4)])
    tar = np.stack([proj(6, 3), proj(6, 2)])
    beta = np.array([1.0, 0.7])
    _, g = oracle.value_and_gradient(s, alpha, rho0, tar, beta, 0)
    h = 1e-6
    for k in [(0, 1, 0, 0), (1, 2, 1, 1), (1, 4, 0, 1)]:
        ap, am = alpha.copy(), alpha.copy()
        ap[k] += h
        am[k] -= h
        fd = (oracle.value_and_gradient(s, ap, rho0, tar, beta, 0)[0]
              - oracle.value_and_gradient(s, am, rho0, tar, beta, 0)[0]) / (2 * h)
        assert abs(fd - g[k]) < 1e-7 * max(1.0, np.max(np.abs(g)))


# ------------------------------------------------------------ objective pins

def test_frobenius_trace_identity():
    # J_Frob = J_Tr - 1/2 (1 - Tr rho_tar^2) - 1/2 (1 - Tr rho^2), Sec. III-C.
    rng = np.random.default_rng(1)
    for _ in range(5):
        A = rng.standard_normal((5, 5)) + 1j * rng.standard_normal((5, 5))
        Bm = rng.standard_normal((5, 5)) + 1j * rng.standard_normal((5, 5))
        r = A @ A.conj().T
        r /= np.trace(r)
        t = Bm @ Bm.conj().T
        t /= np.trace(t)
        jf = oracle.merit(oracle.KIND_FROB, r, t)
        jt = oracle.merit(oracle.KIND_TR, r, t)
        pt = np.trace(t @ t).real
        pr = np.trace(r @ r).real
        assert jf == pytest.approx(jt - 0.5 * (1 - pt) - 0.5 * (1 - pr), abs=1e-14)
    t = proj(3, 1)
    assert oracle.merit(oracle.KIND_FROB, t, t) == 0.0
    assert oracle.merit(oracle.KIND_TR, t, t) == pytest.approx(0.0, abs=1e-15)
    assert oracle.fidelity(t, t) == pytest.approx(1.0)


def test_basis_matrices_are_pure_and_span():
    for n in (2, 3, 4):
        Bs = basis_density_matrices(n)
        for B in Bs:
            assert abs(np.trace(B) - 1) < 1e-15
            assert abs(np.trace(B @ B) - 1) < 1e-15
            assert np.max(np.abs(B - B.conj().T)) < 1e-15
            w = np.linalg.eigvalsh(B)
            assert w.min() > -1e-15 and np.sum(w > 1e-12) == 1
        V = np.stack([oracle.vec(B) for B in Bs])
        assert np.linalg.matrix_rank(V) == n * n


# ------------------------------------------------------------ gradient pins

def _tiny_problem(seed=0, NT=12, nlev=(2, 3), kind=0, gamma2=0.0):
    rng = np.random.default_rng(seed)
    s = random_system(rng, nlev, NT=NT, T=2.0, Ns=4, Nf=2)
    alpha = random_alpha(rng, s, amp=0.05)
    N = s.N
    from workloads import random_pure_states
    rho0 = random_pure_states(rng, N, 3)
    tar = random_pure_states(rng, N, 3)
    beta = rng.uniform(0.5, 2.0, 3)
    return s, alpha, rho0, tar, beta, kind, gamma2


def _G(s, alpha, rho0, tar, beta, kind, gamma2):
    return oracle.objective(kind, oracle.imr_forward(s, alpha, rho0), tar, beta, gamma2, alpha)


@pytest.mark.parametrize("kind,gamma2,NT", [(0, 0.0, 12), (1, 0.3, 12), (0, 0.0, 3)])
def test_gradient_against_central_differences(kind, gamma2, NT):
    s, alpha, rho0, tar, beta, kind, gamma2 = _tiny_problem(NT=NT, kind=kind, gamma2=gamma2)
    G, g = oracle.value_and_gradient(s, alpha, rho0, tar, beta, kind, gamma2)
    assert G == pytest.approx(_G(s, alpha, rho0, tar, beta, kind, gamma2), rel=1e-14)
    fd = np.zeros_like(alpha)
    h = 1e-6
    for idx in np.ndindex(alpha.shape):
        ap = alpha.copy()
        am = alpha.copy()
        ap[idx] += h
        am[idx] -= h
        fd[idx] = (_G(s, ap, rho0, tar, beta, kind, gamma2) - _G(s, am, rho0, tar, beta, kind, gamma2)) / (2 * h)
    assert np.max(np.abs(g - fd)) < 1e-7 * np.max(np.abs(g))


def test_gradient_taylor_remainder_is_second_order():
    s, alpha, rho0, tar, beta, kind, gamma2 = _tiny_problem(seed=2, NT=10)
    G, g = oracle.value_and_gradient(s, alpha, rho0, tar, beta, kind, gamma2)
    rng = np.random.default_rng(9)
    d = rng.standard_normal(alpha.shape)
    rem = []
    for eps in (2e-4, 1e-4):
        Ge = _G(s, alpha + eps * d, rho0, tar, beta, kind, gamma2)
        rem.append(abs(Ge - G - eps * np.sum(g * d)))
    assert 3.5 < rem[0] / rem[1] < 4.5


def test_literal_dM_dalpha_matches_chain_rule():
    # Build dM/dalpha_k densely from M(alpha + e_k) - M(alpha) (M is affine in
    # alpha) and contract with the stage vectors literally, for a few k.
    s, alpha, rho0, tar, beta, kind, gamma2 = _tiny_problem(seed=4, NT=5)
    _, g = oracle.value_and_gradient(s, alpha, rho0, tar, beta, kind, gamma2)
    N = s.N
    I = np.eye(N * N)
    rhoT, st = oracle.imr_forward(s, alpha, rho0, keep_states=True)
    qh = np.stack([oracle.vec(r) for r in oracle.terminal_adjoint(kind, rhoT, tar, beta)], 1)
    lit = np.zeros_like(alpha)
    for j in reversed(range(s.NT)):
        t = (j + 0.5) * s.dt
        M = oracle.superoperator(s, alpha, t)
        A = I - 0.5 * s.dt * M
        Z = np.linalg.solve(A, np.stack([oracle.vec(r) for r in st[j]], 1))
        Zh = np.linalg.solve(A.conj().T, qh)
        for idx in np.ndindex(alpha.shape):
            e = np.zeros_like(alpha)
            e[idx] = 1.0
            dM = oracle.superoperator(s, alpha + e, t) - M
            lit[idx] += s.dt * np.real(np.sum(Zh.conj() * (dM @ Z)))
        qh = qh + s.dt * (M.conj().T @ Zh)
    assert np.max(np.abs(lit - g)) < 1e-10 * np.max(np.abs(g))


def test_operator_form_path_matches_dense_path(monkeypatch):
    s, alpha, rho0, tar, beta, kind, gamma2 = _tiny_problem(seed=6, NT=6, nlev=(3, 2))
    Gd, gd = oracle.value_and_gradient(s, alpha, rho0, tar, beta, kind, gamma2)
    rd = oracle.imr_forward(s, alpha, rho0)
    import oracle.lindblad as L
    monkeypatch.setattr(L, "DENSE_MAX_N2", 1)
    ro = oracle.imr_forward(s, alpha, rho0)
    Go, go = oracle.value_and_gradient(s, alpha, rho0, tar, beta, kind, gamma2)
    assert np.max(np.abs(ro - rd)) < 1e-13
    assert Go == pytest.approx(Gd, rel=1e-12)
    assert np.max(np.abs(go - gd)) < 1e-11 * np.max(np.abs(gd))


# ------------------------------------------------------------ J_Nm, ensemble and gate states

def test_jnm_vanishes_only_at_its_target():
    # Sec. III-B: J_Nm(rho) >= 0, and = 0 iff rho = |m><m|.
    N, m = 6, 2
    O = observable_nm(N, m)
    assert abs(oracle.merit(oracle.KIND_NM, proj(N, m), O)) < 1e-15
    rng = np.random.default_rng(31)
    for r in random_pure_states(rng, N, 20):
        assert oracle.merit(oracle.KIND_NM, r, O) > 1e-3
    # the expected distance |l - m| of a basis state
    for l in range(N):
        assert abs(oracle.merit(oracle.KIND_NM, proj(N, l), O) - abs(l - m)) < 1e-15


def test_ensemble_state_replaces_the_basis():
    # Sec. III-B: the evolution is linear in rho(0) and J_Nm is linear in
    # rho(T), so the ensemble state rho_s = (1/N^2) sum B^kj with M = 1 gives the
    # objective and gradient of the N^2 basis matrices with M = N^2.
    rng = np.random.default_rng(32)
    s = random_system(rng, (2, 2), NT=10, T=1.0)
    alpha = random_alpha(rng, s, amp=0.05)
    N = s.N
    O = observable_nm(N, 0)
    basis = basis_density_matrices(N)
    G1, g1 = oracle.value_and_gradient(s, alpha, ensemble_state(N)[None], O[None], np.ones(1), oracle.KIND_NM)
    Gb, gb = oracle.value_and_gradient(s, alpha, basis, np.repeat(O[None], N * N, axis=0), np.ones(N * N),
                                       oracle.KIND_NM)
    assert abs(G1 - Gb) < 1e-14 * abs(Gb)
    assert np.max(np.abs(g1 - gb)) < 1e-13 * np.max(np.abs(gb))


def test_jnm_gradient_against_central_differences():
    rng = np.random.default_rng(33)
    s = random_system(rng, (2, 3), NT=8, T=0.8)
    alpha = random_alpha(rng, s, amp=0.05)
    N = s.N
    rho0 = random_pure_states(rng, N, 2)
    O = np.stack([observable_nm(N, 0), observable_nm(N, 4)])
    beta = np.array([1.0, 0.6])
    _, g = oracle.value_and_gradient(s, alpha, rho0, O, beta, oracle.KIND_NM)
    h = 1e-6
    for k in [(0, 1, 0, 0), (1, 3, 1, 1), (0, 4, 1, 0)]:
        ap, am = alpha.copy(), alpha.copy()
        ap[k] += h
        am[k] -= h
        fd = (oracle.value_and_gradient(s, ap, rho0, O, beta, oracle.KIND_NM)[0]
              - oracle.value_and_gradient(s, am, rho0, O, beta, oracle.KIND_NM)[0]) / (2 * h)
        assert abs(fd - g[k]) < 1e-7 * max(1.0, np.max(np.abs(g)))


def test_gate_initial_states():
    # Sec. III-C: rho_1 diagonal with distinct non-negative weights, rho_2 the
    # pure uniform superposition, rho_3 = I/N; all density matrices.
    N = 5
    r1, r2, r3 = gate_initial_states(N)
    d = np.real(np.diag(r1))
    assert np.allclose(r1, np.diag(d)) and (d >= 0).all() and len(set(np.round(d, 14))) == N
    assert abs(np.trace(r2 @ r2) - 1) < 1e-14 and np.allclose(r2 @ np.ones(N), np.ones(N))
    assert np.allclose(r3, np.eye(N) / N)
    for r in (r1, r2, r3):
        assert abs(np.trace(r) - 1) < 1e-14 and np.allclose(r, r.conj().T)


# ------------------------------------------------------------ running penalty

def _decay_penalty_integral(T, T1, a):
    """int_0^T (1/a) exp(-((t-T)/a)^2) exp(-t/T1) dt by completing the square."""
    from scipy.special import erf
    c = a * a / (2 * T1)
    return 0.5 * np.sqrt(np.pi) * np.exp(a * a / (4 * T1 * T1) - T / T1) * (erf(c / a) + erf((T - c) / a))


def test_running_penalty_matches_the_integral_for_a_decaying_qubit():
    # J_Nm with m = 0 on a decaying qubit is rho_11(t) = exp(-t/T1) in the
    # continuum.  The left rectangle sum differs from the integral by
    # -(dt/2)(f(T) - f(0)) + O(dt^2) (Euler-Maclaurin): with that term added
    # the error falls fourfold per halving of dt.  A right rectangle sum, a
    # missing dt or a wrong weight fails this.
    T, T1, a, g1 = 5.0, 7.0, 1.3, 0.8
    I = _decay_penalty_integral(T, T1, a)
    f = lambda t: np.exp(-(((t - T) / a) ** 2)) / a * np.exp(-t / T1)
    O = observable_nm(2, 0)[None]
    errs = []
    for NT in (40, 80, 160):
        s = mk((2,), T1=[T1], T=T, NT=NT)
        alpha = np.zeros((1, s.Ns, 1, 2))
        _, states = oracle.imr_forward(s, alpha, proj(2, 1)[None], keep_states=True)
        P = oracle.running_penalty(s, oracle.KIND_NM, states, O, g1, a)
        G, _ = oracle.value_and_gradient(s, alpha, proj(2, 1)[None], O, np.zeros(1), oracle.KIND_NM, gamma1=g1,
                                         penalty_a=a)
        assert G == pytest.approx(P, rel=1e-14)  # beta = 0 leaves only the penalty
        errs.append(abs(P / g1 + 0.5 * s.dt * (f(T) - f(0.0)) - I))
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5
    assert errs[-1] < 3e-5 * I


@pytest.mark.parametrize("kind", [oracle.KIND_FROB, oracle.KIND_TR, oracle.KIND_NM])
def test_running_penalty_gradient_against_central_differences(kind):
    rng = np.random.default_rng(40 + kind)
    s = random_system(rng, (2, 3), NT=14, T=2.0, Ns=4, Nf=2)
    alpha = random_alpha(rng, s, amp=0.05)
    from workloads import random_pure_states
    rho0 = random_pure_states(rng, s.N, 3)
    tar = random_pure_states(rng, s.N, 3) if kind != oracle.KIND_NM else np.repeat(observable_nm(s.N, 1)[None], 3, 0)
    beta = rng.uniform(0.5, 2.0, 3)
    kw = dict(gamma1=0.7, penalty_a=0.6)
    G, g = oracle.value_and_gradient(s, alpha, rho0, tar, beta, kind, 0.1, **kw)
    G0, g0 = oracle.value_and_gradient(s, alpha, rho0, tar, beta, kind, 0.1)
    assert abs(G - G0) > 1e-3 * abs(G0) and np.max(np.abs(g - g0)) > 1e-3 * np.max(np.abs(g0))

    def Gof(al):
        return oracle.value_and_gradient(s, al, rho0, tar, beta, kind, 0.1, **kw)[0]

    h = 1e-6
    fd = np.zeros_like(alpha)
    for idx in np.ndindex(alpha.shape):
        ap = alpha.copy()
        am = alpha.copy()
        ap[idx] += h
        am[idx] -= h
        fd[idx] = (Gof(ap) - Gof(am)) / (2 * h)
    assert np.max(np.abs(g - fd)) < 1e-7 * np.max(np.abs(g))
