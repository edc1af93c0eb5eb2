"""Oracle: Lindblad master equation, implicit midpoint rule, discrete adjoint.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed, and where the paper defines it:

* System and control Hamiltonians, collapse operators: Sec. II, eq.
  (mastereq) and the equations for H_sys, H_c and the Lindbladian.
* Control parameterisation by quadratic B-splines times carrier waves:
  Sec. II, eq. (rotctrl) and the knot-spacing statement after it.
* Vectorised equation dq/dt = M(t) q with column stacking: App. A, eq.
  (mastereq_vectorized).  Built densely from Kronecker products.
* Implicit midpoint rule: App. A, eqs. (IMR) and (linsystem_primal).  The
  oracle solves each stage system directly (dense LU) or with GMRES, and
  applies the update q + dt*M*z literally.
* Objective and merit functionals: Sec. III, eqs. (optimproblem) and
  (Jmeasure); fidelity eq. (fidelity).
* Discrete adjoint and reduced gradient: App. B, eqs. (linsystem_adjoint)
  and (reducedgradient).

Readings of passages that are silent or garbled:

* All frequencies enter as 2*pi times the GHz value; times are in ns.
  Control coefficients alpha are GHz values as well, so d_q carries 2*pi.
* The dephasing operator is a^dagger a / sqrt(T2) literally.
* Splines: S_s(t) = B((t - tau_s)/dtau), dtau = T/(Ns-2),
  tau_s = (s - 1/2) dtau, s = 0..Ns-1, with B the centred quadratic
  B-spline.
* Controls are evaluated once per step, at the midpoint t_j + dt/2.
* Gradient: dG/dalpha_k = sum_j dt Re <zhat^j, (dM/dalpha_k) z^j>, with
  <a, b> = a^H b and the adjoint seeded with dJ/d(conj q) (the
  conjugate-Wirtinger gradient of the merit functional).
* The terminal condition is (beta_i / M) dJ/d(conj q) with M the number of
  initial states of the system.
* Running penalty (gamma1 term of eq. optimproblem): averaged over the
  initial states with the same 1/M as the final-time term, without the
  weights beta_i, and integrated by the left rectangle rule on the time grid,
  dt sum_{j=0}^{NT-1} beta(t_j) J(q^j), t_j = j dt; the adjoint source at step
  j is then gamma1 dt beta(t_j) (1/M) dJ/d(conj q^j) (the source term of App.
  B, with the rectangle weight dt).

Parity pins (tests/test_oracle_pins.py): discrete and continuum T1 decay,
dephasing rate and phase, the T1 cascade, closed two-level Rabi oscillation
and the phase of its coherence (which fixes d a + conj(d) a^+ against the
swapped coupling),
trace and Hermiticity preservation, norm preservation without collapse
operators, IMR against the matrix exponential (second order), the Cayley form
of one IMR step, the J_Frob/J_Tr identity, basis-matrix purity, B-spline
partition of unity and agreement with scipy's B-spline basis, dense against
operator form, the adjoint dot-product identity, and the gradient against
central finite differences and a Taylor remainder test.  The running penalty
against the closed-form integral of a decaying qubit (its left-rectangle
error term included), and its gradient against central differences.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from threadpoolctl import threadpool_limits

TWO_PI = 2.0 * np.pi
KIND_FROB = 0
KIND_TR = 1
KIND_NM = 2

# Dense superoperators are built while N^2 stays at or below this size;
# above it the oracle works on density matrices with sparse operators.
DENSE_MAX_N2 = 1024

# The solvers factor many small matrices; a multi-threaded BLAS spends most
# of its time waking threads on them, so they run on one BLAS thread.
ORACLE_BLAS_THREADS = 1


def _one_blas_thread(fn):
    import functools

    @functools.wraps(fn)
    def wrapped(*args, **kwargs):
        with threadpool_limits(ORACLE_BLAS_THREADS, user_api="blas"):
            return fn(*args, **kwargs)
    return wrapped

__all__ = [
    "TWO_PI", "KIND_FROB", "KIND_TR", "KIND_NM", "DENSE_MAX_N2",
    "lowering", "embed", "system_hamiltonian", "coupling_hamiltonian", "bspline2", "spline_basis",
    "controls", "control_hamiltonian", "hamiltonian", "collapse_operators",
    "vec", "unvec", "superoperator", "lindbladian", "lindbladian_adjoint",
    "lindbladian_entries", "imr_forward", "merit", "objective",
    "terminal_adjoint", "value_and_gradient", "fidelity", "penalty_weight", "running_penalty",
]


# ----------------------------------------------------------------------------
# Operators of Sec. II
# ----------------------------------------------------------------------------

def lowering(n: int) -> np.ndarray:
    """Lowering operator a of one subsystem: a|k> = sqrt(k)|k-1>."""
    a = np.zeros((n, n))
    for k in range(1, n):
        a[k - 1, k] = np.sqrt(k)
    return a


def embed(op, q: int, nlev, sparse: bool = False):
    """I x ... x op x ... x I with op in slot q (slot 0 leftmost)."""
    mats = [op if p == q else np.eye(nlev[p]) for p in range(len(nlev))]
    if sparse:
        out = sp.csr_matrix(np.ones((1, 1)))
        for m in mats:
            out = sp.kron(out, sp.csr_matrix(m), format="csr")
        return out
    out = np.ones((1, 1))
    for m in mats:
        out = np.kron(out, m)
    return out


def system_hamiltonian(sys, sparse: bool = False):
    """Time-independent part of H_sys of Sec. II in rad/ns (the
    Jaynes-Cummings coupling is ``coupling_hamiltonian``).

    H_sys = sum_q (omega_q - omega_q^rot) a_q^+ a_q - xi_q/2 a_q^+ a_q^+ a_q a_q
            - sum_{p>q} xi_pq a_p^+ a_p a_q^+ a_q
    """
    nlev = sys.nlev
    N = sys.N
    H = sp.csr_matrix((N, N)) if sparse else np.zeros((N, N))
    ops = []
    for q in range(sys.Q):
        a = embed(lowering(nlev[q]), q, nlev, sparse)
        ad = a.T
        ops.append((a, ad))
        H = H + TWO_PI * sys.detuning[q] * (ad @ a)
        H = H - TWO_PI * 0.5 * sys.selfkerr[q] * (ad @ ad @ a @ a)
    for q in range(sys.Q):
        for p in range(q + 1, sys.Q):
            xi = sys.crosskerr[q, p]
            if xi != 0.0:
                ap, adp = ops[p]
                aq, adq = ops[q]
                H = H - TWO_PI * xi * (adp @ ap @ adq @ aq)
    return H


def coupling_hamiltonian(sys, t, sparse: bool = False):
    """Jaynes-Cummings coupling of H_sys (Sec. II) at time t, rad/ns:

        sum_{p>q} g_pq ( e^{+i (w_p^rot - w_q^rot) t} a_p^+ a_q
                         + e^{-i (w_p^rot - w_q^rot) t} a_p a_q^+ ),

    the general form with unequal rotation frequencies, whose phases
    multiply a_p^+ a_q and a_p a_q^+ respectively.  Zero when the system has
    no coupling (sys.jc None); missing rotation frequencies are all equal.
    """
    N = sys.N
    H = sp.csr_matrix((N, N), dtype=np.complex128) if sparse else np.zeros((N, N), dtype=np.complex128)
    g = getattr(sys, "jc", None)
    if g is None:
        return H
    rot = getattr(sys, "rotfreq", None)
    rot = np.zeros(sys.Q) if rot is None else np.asarray(rot, dtype=np.float64)
    for p in range(sys.Q):
        ap = embed(lowering(sys.nlev[p]), p, sys.nlev, sparse)
        for q in range(p):
            if g[p, q] == 0.0:
                continue
            aq = embed(lowering(sys.nlev[q]), q, sys.nlev, sparse)
            ph = np.exp(1j * TWO_PI * (rot[p] - rot[q]) * t)
            H = H + TWO_PI * g[p, q] * (ph * (ap.T @ aq) + np.conj(ph) * (ap @ aq.T))
    return H


def bspline2(x):
    """Centred quadratic B-spline (support |x| < 3/2, integral 1)."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    return np.where(x <= 0.5, 0.75 - x * x,
                    np.where(x <= 1.5, 0.5 * (x - 1.5) ** 2, 0.0))


def spline_basis(sys, s: int, t):
    """S_s(t): B-spline wavelet s on the uniform grid of Sec. II.

    Knot spacing dtau = T/(Ns-2); centre tau_s = (s - 1/2) dtau.
    """
    dtau = sys.T / (sys.Ns - 2)
    return bspline2((np.asarray(t) - (s - 0.5) * dtau) / dtau)


def controls(sys, alpha, t):
    """d_q(alpha, t) of eq. (rotctrl) for every subsystem, in rad/ns.

    alpha[q, s, f] = (Re, Im) in GHz; carriers Omega/2pi in GHz.
    """
    d = np.zeros(sys.Q, dtype=np.complex128)
    for q in range(sys.Q):
        for s in range(sys.Ns):
            S = float(spline_basis(sys, s, t))
            if S == 0.0:
                continue
            for f in range(sys.Nf):
                coef = alpha[q, s, f, 0] + 1j * alpha[q, s, f, 1]
                d[q] += S * coef * np.exp(1j * TWO_PI * sys.carriers[q, f] * t)
    return TWO_PI * d


def control_hamiltonian(sys, d, sparse: bool = False):
    """H_c = sum_q d_q a_q + conj(d_q) a_q^+ (Sec. II, rotating frame)."""
    N = sys.N
    H = sp.csr_matrix((N, N), dtype=np.complex128) if sparse else np.zeros((N, N), np.complex128)
    for q in range(sys.Q):
        a = embed(lowering(sys.nlev[q]), q, sys.nlev, sparse)
        H = H + d[q] * a + np.conj(d[q]) * a.T
    return H


def hamiltonian(sys, alpha, t, sparse: bool = False):
    """H(t) = H_sys(t) + H_c(t) (the Jaynes-Cummings part of H_sys may depend on t)."""
    return (system_hamiltonian(sys, sparse) + coupling_hamiltonian(sys, t, sparse)
            + control_hamiltonian(sys, controls(sys, alpha, t), sparse))


def collapse_operators(sys, sparse: bool = False):
    """L_1q = a_q/sqrt(T1_q) (decay), L_2q = a_q^+ a_q/sqrt(T2_q) (dephasing).

    A time that is not finite and positive switches its operator off.
    """
    out = []
    for q in range(sys.Q):
        a = embed(lowering(sys.nlev[q]), q, sys.nlev, sparse)
        for T, op in ((sys.T1[q], a), (sys.T2[q], a.T @ a)):
            if np.isfinite(T) and T > 0:
                out.append(op / np.sqrt(T))
    return out


# ----------------------------------------------------------------------------
# Vectorised form, App. A
# ----------------------------------------------------------------------------

def vec(rho):
    """Column stacking: vec(rho)[i + N*j] = rho[i, j]."""
    return np.asarray(rho).reshape(rho.shape[:-2] + (-1,), order="F") if rho.ndim == 2 \
        else np.stack([vec(r) for r in rho])


def unvec(v, N: int):
    """Inverse of vec."""
    return np.asarray(v).reshape((N, N), order="F")


def superoperator(sys, alpha, t):
    """Dense M(t) of eq. (mastereq_vectorized).

    M = -i (I x H - H^T x I) + sum_L L x L - 1/2 (I x L^T L + L^T L x I).
    The collapse operators here are real, which is what makes L x L (no
    conjugate) and L^T L (no dagger) valid in the printed form.
    """
    N = sys.N
    I = np.eye(N)
    H = hamiltonian(sys, alpha, t)
    M = -1j * (np.kron(I, H) - np.kron(H.T, I))
    for L in collapse_operators(sys):
        assert np.isrealobj(L)
        LtL = L.T @ L
        M = M + np.kron(L, L) - 0.5 * (np.kron(I, LtL) + np.kron(LtL, I))
    return M


def lindbladian(sys, alpha, t, rho, ops=None):
    """M(t) applied to one density matrix, in the form of eq. (mastereq).

    -i [H, rho] + sum_L L rho L^+ - 1/2 (L^+ L rho + rho L^+ L).
    ``ops`` = (H_sys, collapse list) may be passed to avoid rebuilding them.
    """
    Hs, Ls = ops if ops is not None else (system_hamiltonian(sys, True), collapse_operators(sys, True))
    H = Hs + coupling_hamiltonian(sys, t, True) + control_hamiltonian(sys, controls(sys, alpha, t), True)
    out = -1j * (H @ rho - (H.T @ rho.T).T)
    for L in Ls:
        Ld = L.conj().T
        LdL = Ld @ L
        out = out + L @ (Ld.T @ rho.T).T - 0.5 * (LdL @ rho + (LdL.T @ rho.T).T)
    return np.asarray(out)


def lindbladian_adjoint(sys, alpha, t, X, ops=None):
    """Adjoint of ``lindbladian`` for <A, B> = Tr(A^+ B).

    i [H, X] + sum_L L^+ X L - 1/2 (L^+ L X + X L^+ L).
    """
    Hs, Ls = ops if ops is not None else (system_hamiltonian(sys, True), collapse_operators(sys, True))
    H = Hs + coupling_hamiltonian(sys, t, True) + control_hamiltonian(sys, controls(sys, alpha, t), True)
    out = 1j * (H @ X - (H.T @ X.T).T)
    for L in Ls:
        Ld = L.conj().T
        LdL = Ld @ L
        out = out + Ld @ (L.T @ X.T).T - 0.5 * (LdL @ X + (LdL.T @ X.T).T)
    return np.asarray(out)


def lindbladian_entries(sys, alpha, t, x, rows, cols, adjoint=False):
    """Selected entries (rows[k], cols[k]) of M(t) x (or M(t)^+ x).

    Each entry is formed from one row of each sparse operator, so a handful
    of entries of a very large state can be checked one by one.
    """
    Hs = system_hamiltonian(sys, True)
    H = sp.csr_matrix(Hs + coupling_hamiltonian(sys, t, True)
                      + control_hamiltonian(sys, controls(sys, alpha, t), True))
    Ls = [sp.csr_matrix(L) for L in collapse_operators(sys, True)]
    sgn = 1j if adjoint else -1j
    out = np.empty(len(rows), dtype=np.complex128)
    HT = sp.csr_matrix(H.T)
    for k, (i, j) in enumerate(zip(rows, cols)):
        hi = H.getrow(i)
        hj = HT.getrow(j)          # column j of H
        v = sgn * (hi.dot(x[:, j])[0] - hj.dot(x[i, :])[0])
        for L in Ls:
            Ld = sp.csr_matrix(L.conj().T)
            LdL = sp.csr_matrix(Ld @ L)
            left, right = (Ld, L) if adjoint else (L, Ld)
            # (left x right)_{ij} = sum_{k,l} left[i,k] x[k,l] right[l,j]
            li = left.getrow(i)
            rj = sp.csr_matrix(right.T).getrow(j)
            jump = 0.0j
            for kk, lv in zip(li.indices, li.data):
                jump += lv * rj.dot(x[kk, :])[0]
            anti = LdL.getrow(i).dot(x[:, j])[0] + sp.csr_matrix(LdL.T).getrow(j).dot(x[i, :])[0]
            v += jump - 0.5 * anti
        out[k] = v
    return out


# ----------------------------------------------------------------------------
# Implicit midpoint rule, App. A
# ----------------------------------------------------------------------------

# Bytes the GMRES Krylov basis may take: the restart length shrinks for very
# large systems (it sets the solver's memory, not its converged result, which
# the residual check below fixes).
GMRES_BASIS_BYTES = 16 << 30


def _gmres_solve(matvec, b, n):
    """Solve A x = b with GMRES plus one refinement pass (rtol ~1e-15)."""
    A = spla.LinearOperator((n, n), matvec=matvec, dtype=np.complex128)
    restart = int(min(80, max(10, GMRES_BASIS_BYTES // (16 * n) - 1)))
    x, info = spla.gmres(A, b, rtol=1e-14, atol=0.0, restart=restart, maxiter=50)
    r = b - matvec(x)
    if np.linalg.norm(r) > 0:
        dx, info2 = spla.gmres(A, r, rtol=1e-10, atol=0.0, restart=restart, maxiter=50)
        x = x + dx
    res = np.linalg.norm(b - matvec(x)) / max(np.linalg.norm(b), 1e-300)
    if res > 1e-13:
        raise RuntimeError(f"oracle GMRES did not converge: residual {res:.3e}")
    return x


def _dense_mode(sys):
    return sys.N * sys.N <= DENSE_MAX_N2


@_one_blas_thread
def imr_forward(sys, alpha, rho0, keep_states: bool = False, nsteps=None):
    """Implicit midpoint rule, eqs. (IMR) and (linsystem_primal).

    For j = 0..NT-1 with M = M(t_j + dt/2):
        (I - dt/2 M) z^j = q^j,     q^{j+1} = q^j + dt M z^j.
    rho0: [B, N, N].  Returns rho(T) [B, N, N] and, with ``keep_states``,
    the list of all q^j as [B, N, N] arrays (j = 0..NT).
    """
    N = sys.N
    dt = sys.dt
    NT = sys.NT if nsteps is None else nsteps
    rho = np.array(rho0, dtype=np.complex128)
    states = [rho.copy()] if keep_states else None
    if _dense_mode(sys):
        Qm = np.stack([vec(r) for r in rho], axis=1)  # [N^2, B]
        I = np.eye(N * N)
        for j in range(NT):
            M = superoperator(sys, alpha, (j + 0.5) * dt)
            lu = sla.lu_factor(I - 0.5 * dt * M)
            Z = sla.lu_solve(lu, Qm)
            Qm = Qm + dt * (M @ Z)
            if keep_states:
                states.append(np.stack([unvec(Qm[:, b], N) for b in range(Qm.shape[1])]))
        rho = np.stack([unvec(Qm[:, b], N) for b in range(Qm.shape[1])])
    else:
        ops = (system_hamiltonian(sys, True), collapse_operators(sys, True))
        for j in range(NT):
            t = (j + 0.5) * dt
            for b in range(rho.shape[0]):
                Mv = lambda v, t=t: vec(lindbladian(sys, alpha, t, unvec(v, N), ops))
                z = _gmres_solve(lambda v: v - 0.5 * dt * Mv(v), vec(rho[b]), N * N)
                rho[b] = rho[b] + dt * unvec(Mv(z), N)
            if keep_states:
                states.append(rho.copy())
    return (rho, states) if keep_states else rho


# ----------------------------------------------------------------------------
# Objective, Sec. III
# ----------------------------------------------------------------------------

def merit(kind: int, rho, rhotar) -> float:
    """J_Frob = 1/2 ||rho_tar - rho||_F^2;  J_Tr = 1 - Re Tr(rho_tar^+ rho);
    J_Nm = Tr(N_m rho), eq. (Jmeasure), with the observable N_m passed as
    rhotar (real diagonal, so the trace is Re Tr(N_m^+ rho))."""
    if kind == KIND_FROB:
        return 0.5 * float(np.sum(np.abs(rhotar - rho) ** 2))
    if kind == KIND_TR:
        return 1.0 - float(np.real(np.trace(rhotar.conj().T @ rho)))
    if kind == KIND_NM:
        return float(np.real(np.trace(rhotar.conj().T @ rho)))
    raise ValueError(kind)


def fidelity(rho, rhotar) -> float:
    """F = Tr(rho_tar^+ rho), eq. (fidelity) (real part)."""
    return float(np.real(np.trace(rhotar.conj().T @ rho)))


def objective(kind, rhoT, rhotar, beta, gamma2, alpha) -> float:
    """G = (1/M) sum_i beta_i J(rho_tar_i, rho_i(T)) + gamma2/2 ||alpha||^2.

    Eq. (optimproblem) with the running-penalty weight gamma1 = 0.
    """
    Mst = rhoT.shape[0]
    J = sum(beta[i] * merit(kind, rhoT[i], rhotar[i]) for i in range(Mst))
    return J / Mst + 0.5 * gamma2 * float(np.sum(np.asarray(alpha) ** 2))


def penalty_weight(sys, a: float, t):
    """beta(t) = (1/a) exp(-((t - T)/a)^2), the weight of the running penalty
    in Sec. III (a > 0, in ns)."""
    return np.exp(-(((np.asarray(t, dtype=np.float64) - sys.T) / a) ** 2)) / a


def running_penalty(sys, kind, states, rhotar, gamma1, a) -> float:
    """gamma1 (1/M) sum_i dt sum_{j=0}^{NT-1} beta(t_j) J(rho_tar_i, q_i^j):
    the gamma1 term of eq. (optimproblem) by the left rectangle rule.
    states: the list of q^j [M, N, N], j = 0..NT."""
    if gamma1 == 0.0:
        return 0.0
    Mst = rhotar.shape[0]
    tot = 0.0
    for j in range(sys.NT):
        w = sys.dt * float(penalty_weight(sys, a, j * sys.dt))
        tot += w * sum(merit(kind, states[j][i], rhotar[i]) for i in range(Mst))
    return gamma1 * tot / Mst


def terminal_adjoint(kind, rhoT, rhotar, beta):
    """qhat^{NT} = (beta_i/M) dJ/d(conj q), App. B terminal condition."""
    Mst = rhoT.shape[0]
    w = (np.asarray(beta) / Mst)[:, None, None]
    if kind == KIND_FROB:
        return w * (rhoT - rhotar)
    if kind == KIND_TR:
        return -w * rhotar
    if kind == KIND_NM:
        return w * rhotar
    raise ValueError(kind)


# ----------------------------------------------------------------------------
# Discrete adjoint and reduced gradient, App. B
# ----------------------------------------------------------------------------

def _dcontrol_dalpha(sys, t):
    """c[q, s, f, r] = d(d_q)/d(alpha_q^{s,f}[r]) at time t, r = Re/Im."""
    c = np.zeros((sys.Q, sys.Ns, sys.Nf, 2), dtype=np.complex128)
    for q in range(sys.Q):
        for s in range(sys.Ns):
            S = float(spline_basis(sys, s, t))
            for f in range(sys.Nf):
                e = TWO_PI * S * np.exp(1j * TWO_PI * sys.carriers[q, f] * t)
                c[q, s, f, 0] = e
                c[q, s, f, 1] = 1j * e
    return c


@_one_blas_thread
def value_and_gradient(sys, alpha, rho0, rhotar, beta, kind, gamma2=0.0, return_final=False, gamma1=0.0,
                       penalty_a=1.0):
    """Objective G and its exact discrete gradient, App. B.

    Backward for j = NT-1..0 with M = M(t_j + dt/2):
        (I - dt/2 M^+) zhat^j = qhat^{j+1}
        grad += dt Re <zhat^j, (dM/dalpha) z^j>
        qhat^j = qhat^{j+1} + dt M^+ zhat^j + (source of the running penalty)
    The source is gamma1 dt beta(t_j) (1/M) dJ/d(conj q^j), i.e. the terminal
    condition's formula with gamma1 dt beta(t_j) in place of beta_i
    (``penalty_a`` is the width a of beta(t)).
    with z^j from (linsystem_primal).  M depends on alpha only through the
    control Hamiltonian, which is linear in d_q and conj(d_q):
        dM/dalpha_k = c_k Sa_q + conj(c_k) Sad_q,
    with Sa_q, Sad_q the superoperators of X -> -i[a_q, X] and
    X -> -i[a_q^+, X] and c_k = d(d_q)/d(alpha_k).  Returns (G, grad) with
    grad shaped like alpha, and rho(T) as a third item with return_final.
    """
    N = sys.N
    dt = sys.dt
    rhoT, states = imr_forward(sys, alpha, rho0, keep_states=True)
    G = objective(kind, rhoT, rhotar, beta, gamma2, alpha)
    G += running_penalty(sys, kind, states, rhotar, gamma1, penalty_a)
    qhat = terminal_adjoint(kind, rhoT, rhotar, beta)
    Mst = rhotar.shape[0]

    def source(j):
        w = gamma1 * sys.dt * float(penalty_weight(sys, penalty_a, j * dt))
        return terminal_adjoint(kind, states[j], rhotar, np.full(Mst, w))
    grad = np.zeros_like(np.asarray(alpha, dtype=np.float64))
    avec = [embed(lowering(sys.nlev[q]), q, sys.nlev) for q in range(sys.Q)]
    if _dense_mode(sys):
        I = np.eye(N * N)
        IN = np.eye(N)
        Sa = [-1j * (np.kron(IN, a) - np.kron(a.T, IN)) for a in avec]
        Sad = [-1j * (np.kron(IN, a.T) - np.kron(a, IN)) for a in avec]
        Qh = np.stack([vec(r) for r in qhat], axis=1)
        for j in reversed(range(sys.NT)):
            t = (j + 0.5) * dt
            M = superoperator(sys, alpha, t)
            lu = sla.lu_factor(I - 0.5 * dt * M)
            Z = sla.lu_solve(lu, np.stack([vec(r) for r in states[j]], axis=1))
            Zh = sla.lu_solve(lu, Qh, trans=2)
            c = _dcontrol_dalpha(sys, t)
            for q in range(sys.Q):
                u = np.sum(Zh.conj() * (Sa[q] @ Z))
                v = np.sum(Zh.conj() * (Sad[q] @ Z))
                grad[q] += dt * np.real(c[q] * u + np.conj(c[q]) * v)
            Qh = Qh + dt * (M.conj().T @ Zh)
            if gamma1 != 0.0:
                Qh = Qh + np.stack([vec(r) for r in source(j)], axis=1)
    else:
        ops = (system_hamiltonian(sys, True), collapse_operators(sys, True))
        aS = [embed(lowering(sys.nlev[q]), q, sys.nlev, True) for q in range(sys.Q)]
        for j in reversed(range(sys.NT)):
            t = (j + 0.5) * dt
            c = _dcontrol_dalpha(sys, t)
            for b in range(qhat.shape[0]):
                Mv = lambda v: vec(lindbladian(sys, alpha, t, unvec(v, N), ops))
                MHv = lambda v: vec(lindbladian_adjoint(sys, alpha, t, unvec(v, N), ops))
                z = unvec(_gmres_solve(lambda v: v - 0.5 * dt * Mv(v), vec(states[j][b]), N * N), N)
                zh = unvec(_gmres_solve(lambda v: v - 0.5 * dt * MHv(v), vec(qhat[b]), N * N), N)
                for q in range(sys.Q):
                    a = aS[q]
                    ad = sp.csr_matrix(a.T)
                    Saz = -1j * (a @ z - (a.T @ z.T).T)
                    Sadz = -1j * (ad @ z - (ad.T @ z.T).T)
                    u = np.sum(zh.conj() * Saz)
                    v = np.sum(zh.conj() * Sadz)
                    grad[q] += dt * np.real(c[q] * u + np.conj(c[q]) * v)
                qhat[b] = qhat[b] + dt * unvec(MHv(vec(zh)), N)
            if gamma1 != 0.0:
                qhat = qhat + source(j)
    grad = grad + gamma2 * np.asarray(alpha)
    return (G, grad, rhoT) if return_final else (G, grad)
