"""Seeded system descriptions, controls and density matrices.

Units follow the paper's footnotes: every frequency-like parameter is given
as an ordinary frequency (the value divided by 2*pi) in GHz, every time in
ns.  Decay and dephasing times are in ns; ``inf`` switches a term off.

Random numbers come from ``numpy.random.Generator(PCG64(seed))`` with
``seed = CONFIG_SEED_BASE + config_index`` for the five named workloads.
The order of the draws is part of each generator's definition: changing it
changes every fixture derived from it.
"""
from __future__ import annotations

from dataclasses import dataclass, replace
from typing import Optional, List, Sequence

import numpy as np

CONFIG_SEED_BASE = 20211020

KIND_FROB = 0
KIND_TR = 1


@dataclass(frozen=True)
class System:
    """One composite qudit system (Section II of the paper).

    nlev[q] is the number of levels of subsystem q; subsystem 0 is the
    leftmost Kronecker factor (most significant digit of a basis index).
    """

    nlev: tuple
    detuning: np.ndarray   # [Q]   (omega_q - omega_q^rot)/2pi   [GHz]
    selfkerr: np.ndarray   # [Q]   xi_q/2pi                      [GHz]
    crosskerr: np.ndarray  # [Q,Q] xi_pq/2pi, entries p<q used   [GHz]
    T1: np.ndarray         # [Q]   decay time   [ns], inf = off
    T2: np.ndarray         # [Q]   dephasing time [ns], inf = off
    Ns: int                # B-spline basis functions per control
    carriers: np.ndarray   # [Q,Nf] carrier frequencies Omega/2pi [GHz]
    T: float               # horizon [ns]
    NT: int                # implicit-midpoint steps
    jc: Optional[np.ndarray] = None       # [Q,Q] g_pq/2pi, entries p>q used [GHz] (Jaynes-Cummings)
    rotfreq: Optional[np.ndarray] = None  # [Q] omega_q^rot/2pi [GHz] (None: all equal)

    @property
    def Q(self) -> int:
        return len(self.nlev)

    @property
    def N(self) -> int:
        return int(np.prod(self.nlev))

    @property
    def Nf(self) -> int:
        return int(self.carriers.shape[1])

    @property
    def dt(self) -> float:
        return self.T / self.NT


@dataclass
class Problem:
    """A batch of systems with their controls, initial and target states."""

    name: str
    systems: List[System]
    alpha: List[np.ndarray]   # per system [Q, Ns, Nf, 2] (Re, Im) [GHz]
    rho0: List[np.ndarray]    # per system [B, N, N] complex128
    rhotar: List[np.ndarray]  # per system [B, N, N] complex128
    beta: List[np.ndarray]    # per system [B] weights
    kind: int = KIND_FROB     # 0 = Frobenius merit, 1 = trace merit
    gamma2: float = 0.0       # Tikhonov weight
    ckpt_every: int = 1       # forward states kept every this many steps

    @property
    def batch(self) -> List[int]:
        return [int(r.shape[0]) for r in self.rho0]


def n_alpha(sys: System) -> int:
    """Number of real control parameters of a system (2*Ns*Nf per qudit)."""
    return 2 * sys.Q * sys.Ns * sys.Nf


# ---------------------------------------------------------------- states

def random_pure_states(rng: np.random.Generator, N: int, B: int) -> np.ndarray:
    """B pure states psi psi^dagger with complex Gaussian psi, normalised."""
    out = np.empty((B, N, N), dtype=np.complex128)
    for b in range(B):
        x = rng.standard_normal(N)
        y = rng.standard_normal(N)
        psi = x + 1j * y
        psi /= np.linalg.norm(psi)
        out[b] = np.outer(psi, psi.conj())
    return out


def basis_density_matrices(n: int) -> np.ndarray:
    """The n^2 basis density matrices B^{kj} of eq. (basismats), Sec. III-B.

    Returned in the order k-major: index k*n + j.  The third case of the
    printed definition is garbled; it is read as (i/2)(|j><k| - |k><j|),
    which makes every B^{kj} a pure state as the text requires.
    """
    out = np.zeros((n * n, n, n), dtype=np.complex128)
    for k in range(n):
        for j in range(n):
            B = np.zeros((n, n), dtype=np.complex128)
            B[k, k] += 0.5
            B[j, j] += 0.5
            if k < j:
                B[k, j] += 0.5
                B[j, k] += 0.5
            elif k > j:
                B[j, k] += 0.5j
                B[k, j] -= 0.5j
            out[k * n + j] = B
    return out


def observable_nm(N: int, m: int) -> np.ndarray:
    """The observable N_m of J_Nm (Sec. III): diagonal, lambda_l = |l - m|."""
    return np.diag(np.abs(np.arange(N) - m).astype(np.float64)).astype(np.complex128)


def ensemble_state(N: int) -> np.ndarray:
    """rho_s(0) = (1/N^2) sum_kj B^kj (Sec. III-B), from the basis matrices."""
    return basis_density_matrices(N).sum(axis=0) / (N * N)


def gate_initial_states(N: int) -> np.ndarray:
    """The three initial states of gate optimisation (Sec. III-C): rho_1
    diagonal with distinct weights lambda_j = 2 (N - j) / (N (N + 1)) (any
    distinct non-negative values qualify; these sum to one), rho_2 the pure
    uniform superposition, rho_3 = I / N."""
    lam = 2.0 * (N - np.arange(N)) / (N * (N + 1))
    psi = np.full(N, 1.0 / np.sqrt(N))
    return np.stack([np.diag(lam), np.outer(psi, psi), np.eye(N) / N]).astype(np.complex128)


def gate_weights(rho0: np.ndarray, first: float = 20.0) -> np.ndarray:
    """beta_i = {first, 1, 1} / Tr(rho_i(0)^2): the emphasis on the first state
    and the purity scaling suggested for J_Tr (Sec. III-C)."""
    w = np.ones(rho0.shape[0])
    w[0] = first
    return w / np.real(np.einsum("bij,bji->b", rho0, rho0))


def essential_embedding(nlev: Sequence[int], ness: Sequence[int]) -> np.ndarray:
    """Full-space basis index of every essential-level basis index.

    Essential index (k_0, ..., k_{Q-1}) with k_q < ness[q], ordered with
    subsystem 0 most significant, maps to the full index with the same
    digits in radix nlev.
    """
    Q = len(nlev)
    idx = []
    for e in range(int(np.prod(ness))):
        rem = e
        digits = []
        for q in reversed(range(Q)):
            digits.append(rem % ness[q])
            rem //= ness[q]
        digits = digits[::-1]
        full = 0
        for q in range(Q):
            full = full * nlev[q] + digits[q]
        idx.append(full)
    return np.array(idx, dtype=np.int64)


def cnot_essential() -> np.ndarray:
    """CNOT on two qubits, control = subsystem 0 (most significant)."""
    V = np.zeros((4, 4))
    V[0, 0] = V[1, 1] = 1.0
    V[2, 3] = V[3, 2] = 1.0
    return V


def _embed_states(states_ess: np.ndarray, emb: np.ndarray, N: int) -> np.ndarray:
    B = states_ess.shape[0]
    out = np.zeros((B, N, N), dtype=np.complex128)
    for b in range(B):
        out[b][np.ix_(emb, emb)] = states_ess[b]
    return out


def _basis_state(N: int, index: int) -> np.ndarray:
    r = np.zeros((N, N), dtype=np.complex128)
    r[index, index] = 1.0
    return r


# ---------------------------------------------------------------- systems

def random_alpha(rng: np.random.Generator, sys: System, amp: float = 0.005) -> np.ndarray:
    """Control coefficients with Re and Im uniform in [-amp, amp] GHz."""
    return rng.uniform(-amp, amp, size=(sys.Q, sys.Ns, sys.Nf, 2))


def _pm_uniform(rng, lo, hi, size):
    sign = rng.choice([-1.0, 1.0], size=size)
    return sign * rng.uniform(lo, hi, size=size)


def random_system(rng: np.random.Generator, nlev: Sequence[int], *, NT: int = 40,
                  T: float = 4.0, Ns: int = 5, Nf: int = 2,
                  strong_dissipation: bool = True,
                  some_terms_off: bool = True, jc: float = 0.0) -> System:
    """A random system for parity and property tests.

    With ``strong_dissipation`` the decay and dephasing times are a few tens
    of ns so that every term of the Lindbladian contributes visibly over a
    short horizon.  With ``some_terms_off`` roughly one in four T1/T2 values
    is switched off (inf).  With ``jc`` > 0 every pair p > q gets a
    Jaynes-Cummings coupling g_pq/2pi uniform in +-[jc/2, jc] GHz (one in
    four switched off) and the subsystems rotation frequencies uniform in
    [-0.2, 0.2] GHz.  These draws come after all the others, so a system
    drawn with jc = 0 is the same as before.
    """
    Q = len(nlev)
    detuning = rng.uniform(-0.3, 0.3, size=Q)
    selfkerr = rng.uniform(-0.3, 0.3, size=Q)
    ck = np.zeros((Q, Q))
    for p in range(Q):
        for q in range(p + 1, Q):
            ck[p, q] = rng.uniform(-0.02, 0.02)
    if strong_dissipation:
        T1 = rng.uniform(10.0, 60.0, size=Q)
        T2 = rng.uniform(10.0, 60.0, size=Q)
    else:
        T1 = rng.uniform(5e4, 1.5e5, size=Q)
        T2 = rng.uniform(4e4, 1.2e5, size=Q)
    if some_terms_off:
        off1 = rng.uniform(size=Q) < 0.25
        off2 = rng.uniform(size=Q) < 0.25
        T1 = np.where(off1, np.inf, T1)
        T2 = np.where(off2, np.inf, T2)
    carriers = rng.uniform(-0.05, 0.05, size=(Q, Nf))
    carriers[:, 0] = 0.0
    g = rot = None
    if jc > 0.0:
        g = np.zeros((Q, Q))
        for p in range(Q):
            for q in range(p):
                mag = rng.uniform(0.5 * jc, jc) * rng.choice([-1.0, 1.0])
                g[p, q] = 0.0 if rng.uniform() < 0.25 else mag
        rot = rng.uniform(-0.2, 0.2, size=Q)
    return System(nlev=tuple(int(n) for n in nlev), detuning=detuning,
                  selfkerr=selfkerr, crosskerr=ck, T1=T1, T2=T2, Ns=Ns,
                  carriers=carriers, T=float(T), NT=int(NT), jc=g, rotfreq=rot)


def _uniform_qudits(Q, n, *, crosskerr, T=100.0, NT=5000, Ns=10, Nf=1):
    """Qudits with detuning 0, self-Kerr -0.2 GHz, T1 = 100 us, T2 = 80 us."""
    return System(nlev=tuple([n] * Q), detuning=np.zeros(Q),
                  selfkerr=np.full(Q, -0.2), crosskerr=crosskerr,
                  T1=np.full(Q, 1.0e5), T2=np.full(Q, 8.0e4), Ns=Ns,
                  carriers=np.zeros((Q, Nf)), T=float(T), NT=int(NT))


def _config1(rng):
    sys = _uniform_qudits(1, 3, crosskerr=np.zeros((1, 1)), T=100.0, NT=2000, Ns=10)
    alpha = random_alpha(rng, sys)
    rho0 = _basis_state(3, 0)[None]
    rhotar = _basis_state(3, 1)[None]
    return Problem("c1_qutrit", [sys], [alpha], [rho0], [rhotar], [np.ones(1)],
                   kind=KIND_FROB)


def _config2(rng):
    Q, n = 2, 4
    detuning = _pm_uniform(rng, 0.1, 0.3, Q)
    selfkerr = _pm_uniform(rng, 0.1, 0.3, Q)
    ck = np.zeros((Q, Q))
    ck[0, 1] = -0.001
    T1 = rng.uniform(50.0, 150.0, size=Q) * 1e3
    T2 = rng.uniform(40.0, 120.0, size=Q) * 1e3
    carriers = np.array([[0.0, -ck[0, 1]]] * Q)
    sys = System(nlev=(n, n), detuning=detuning, selfkerr=selfkerr, crosskerr=ck,
                 T1=T1, T2=T2, Ns=20, carriers=carriers, T=200.0, NT=10000)
    alpha = random_alpha(rng, sys)
    emb = essential_embedding((n, n), (2, 2))
    Bess = basis_density_matrices(4)
    V = cnot_essential()
    tar_ess = np.einsum("ab,kbc,dc->kad", V, Bess, V)
    rho0 = _embed_states(Bess, emb, n * n)
    rhotar = _embed_states(tar_ess, emb, n * n)
    return Problem("c2_cnot_2x4", [sys], [alpha], [rho0], [rhotar],
                   [np.ones(16)], kind=KIND_FROB)


def _chain_crosskerr(rng, Q, ring=False):
    ck = np.zeros((Q, Q))
    pairs = [(q, q + 1) for q in range(Q - 1)]
    if ring and Q > 2:
        pairs.append((0, Q - 1))
    for p, q in pairs:
        ck[p, q] = rng.uniform(-0.002, -0.0005)
    return ck


def _config3(rng, nsys=96):
    systems, alphas, rho0s, tars, betas = [], [], [], [], []
    for _ in range(nsys):
        Q = int(rng.integers(2, 5))
        nlev = tuple(int(v) for v in rng.integers(3, 6, size=Q))
        B = int(rng.integers(1, 9))
        ck = _chain_crosskerr(rng, Q)
        sys = System(nlev=nlev, detuning=np.zeros(Q), selfkerr=np.full(Q, -0.2),
                     crosskerr=ck, T1=np.full(Q, 1.0e5), T2=np.full(Q, 8.0e4),
                     Ns=10, carriers=np.zeros((Q, 1)), T=100.0, NT=5000)
        N = sys.N
        systems.append(sys)
        alphas.append(random_alpha(rng, sys))
        rho0s.append(random_pure_states(rng, N, B))
        tars.append(np.repeat(_basis_state(N, 0)[None], B, axis=0))
        betas.append(np.ones(B))
    # the full state history of the streamed systems would take ~0.9 TB: checkpoint every ~sqrt(NT)
    return Problem("c3_uneven_96", systems, alphas, rho0s, tars, betas, kind=KIND_FROB, ckpt_every=0)


def _config4(rng):
    Q = 5
    sys = _uniform_qudits(Q, 3, crosskerr=_chain_crosskerr(rng, Q), T=300.0,
                          NT=20000, Ns=30)
    alpha = random_alpha(rng, sys)
    rho0 = random_pure_states(rng, sys.N, 10)
    return Problem("c4_5qutrit_chain", [sys], [alpha], [rho0], [rho0.copy()],
                   [np.ones(10)], kind=KIND_TR, ckpt_every=200)


def _config5(rng):
    Q = 8
    sys = _uniform_qudits(Q, 3, crosskerr=_chain_crosskerr(rng, Q, ring=True),
                          T=100.0, NT=5000, Ns=20)
    alpha = random_alpha(rng, sys)
    N = sys.N
    ones = sum(3 ** (Q - 1 - q) for q in range(Q))  # |1...1> in radix 3
    rho0 = _basis_state(N, 0)[None]
    rhotar = _basis_state(N, ones)[None]
    return Problem("c5_8qutrit_ring", [sys], [alpha], [rho0], [rhotar],
                   [np.ones(1)], kind=KIND_FROB, ckpt_every=0)


_MAKERS = {1: _config1, 2: _config2, 3: _config3, 4: _config4, 5: _config5}


def make_config(index: int) -> Problem:
    """The five named workloads, 1-based, each from its own seed."""
    rng = np.random.Generator(np.random.PCG64(CONFIG_SEED_BASE + index))
    return _MAKERS[index](rng)


def with_random_states(prob: Problem, extra: int, seed: int) -> Problem:
    """The same systems and controls with `extra` seeded random pure initial
    states and targets (weight 1) appended to every system's batch."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rho0, tar, beta = [], [], []
    for k, s in enumerate(prob.systems):
        rho0.append(np.concatenate([prob.rho0[k], random_pure_states(rng, s.N, extra)]))
        tar.append(np.concatenate([prob.rhotar[k], random_pure_states(rng, s.N, extra)]))
        beta.append(np.concatenate([prob.beta[k], np.ones(extra)]))
    return Problem(prob.name + f"_plus{extra}", prob.systems, prob.alpha, rho0, tar, beta, prob.kind,
                   prob.gamma2, prob.ckpt_every)


def truncate_steps(prob: Problem, NT: int) -> Problem:
    """Same inputs with fewer steps at the same step size (T = dt*NT)."""
    systems = [replace(s, T=s.dt * NT, NT=NT) for s in prob.systems]
    return Problem(prob.name + f"_nt{NT}", systems, prob.alpha, prob.rho0,
                   prob.rhotar, prob.beta, prob.kind, prob.gamma2,
                   min(prob.ckpt_every, NT) if prob.ckpt_every else 0)
