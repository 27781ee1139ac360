"""Exact singlet yields from dense matrices.  Test infrastructure only.

For one field B the wavepacket |S,Omega;t> = exp(-iGt)|S,Omega> with
G = H - iK (Eq. 13, Eq. 6), so the finite-horizon single-wavepacket yield of
Eq. 22,

    phi_S(Omega) = k_S int_0^T <S,Omega;t| P_S |S,Omega;t> dt,

is the quadratic form k_S <S,Omega| X_T |S,Omega> of the one operator

    X_T = int_0^T exp(+iG^dag t) P_S exp(-iGt) dt.

The deterministic trace of Eq. 14 with A = P_S, integrated as in Eq. 20, is
Phi_S(T) = (k_S / Z) Tr[P_S X_T] (rho(0) = P_S / Z).

X_T is obtained with Van Loan's block-triangular matrix exponential
(C. Van Loan, IEEE TAC 23 (1978) 395):  for C = [[-iG^dag, A], [0, -iG]],
exp(TC) = [[E11, F], [0, E22]] with E22 = exp(-iGT) and F = int_0^T
exp(-iG^dag (T-s)) A exp(-iGs) ds, hence X_T = E22^dag F.  The matrix
exponential is scipy's (a library primitive); nothing else is approximated.
"""
import numpy as np
import scipy.linalg as sla

from .coherent import initial_wavepacket


def integrated_operator(G, A, T):
    """X_T = int_0^T exp(iG^dag t) A exp(-iGt) dt via the Van Loan block exponential."""
    n = G.shape[0]
    C = np.zeros((2 * n, 2 * n), complex)
    C[:n, :n] = -1j * G.conj().T
    C[:n, n:] = A
    C[n:, n:] = -1j * G
    E = sla.expm(T * C)
    return E[n:, n:].conj().T @ E[:n, n:]


def integrated_operator_eig(G, A, T):
    """Same X_T from the eigendecomposition G = V diag(lam) V^-1 (cross-check route).

    (V^dag X_T V)_{jl} = (V^dag A V)_{jl} * int_0^T exp(i(conj(lam_j) - lam_l)t) dt.
    Only well conditioned when V is (no defective or nearly defective G).
    """
    lam, V = np.linalg.eig(G)
    Vi = np.linalg.inv(V)
    mu = lam.conj()[:, None] - lam[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        w = np.where(np.abs(mu * T) < 1e-8, T + 0.5j * mu * T * T,
                     (np.exp(1j * mu * T) - 1.0) / (1j * mu))
    core = (V.conj().T @ A @ V) * w
    return Vi.conj().T @ core @ Vi


class FieldOracle:
    """Exact per-field quantities for one system at one field and horizon."""

    def __init__(self, system, B_mT, T):
        self.sys = system
        self.B = float(B_mT)
        self.T = float(T)
        self.G = system.G(B_mT)
        self.X = integrated_operator(self.G, system.PS, self.T)

    def phi(self, psi0):
        """phi_S = k_S <psi0|X_T|psi0> (Eq. 22 on [0, T])."""
        return float(self.sys.kS * np.real(np.vdot(psi0, self.X @ psi0)))

    def phi_samples(self, angles):
        """phi_S for every sample of an [M][N][2] angle array."""
        return np.array([self.phi(initial_wavepacket(self.sys, a)) for a in angles])

    def trace_yield(self):
        """Deterministic Phi_S(T) = (k_S/Z) Tr[P_S X_T] (Eq. 14 and 20)."""
        return float(self.sys.kS * np.real(np.trace(self.sys.PS @ self.X)) / self.sys.Z)

    def survival(self, psi0, t):
        """Population N(t) = ||exp(-iGt) psi0||^2."""
        v = sla.expm(-1j * self.G * t) @ psi0
        return float(np.real(np.vdot(v, v)))

    def singlet_probability(self, psi0, t):
        """<psi0(t)|P_S|psi0(t)> at one time t (the integrand of Eq. 22)."""
        v = sla.expm(-1j * self.G * t) @ psi0
        return float(np.real(np.vdot(v, self.sys.PS @ v)))
