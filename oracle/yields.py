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
from .spin import spin_ops


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

    def singlet_block(self):
        """A = <S|X_T|S>, the nuclear-space operator with phi_S(Omega) = k_S <Omega|A|Omega>
        (the electron part of every wavepacket of Eq. 19 is the singlet)."""
        Z = self.sys.Z
        X4 = self.X.reshape(4, Z, 4, Z)
        s = self.sys.singlet.astype(complex)
        return np.einsum("e,eifj,f->ij", s.conj(), X4, s)

    def second_moment(self):
        """E_Omega[phi_S^2] over directions uniform on every sphere (Eq. 18), exactly.

        phi_S^2 = k_S^2 <Omega,Omega| A (x) A |Omega,Omega>, and the directions of distinct
        nuclei are independent, so the mean factorises over nuclei into the second moment
        E[|Omega_k><Omega_k| (x) |Omega_k><Omega_k|] of one coherent state.  |Omega>(x)|Omega>
        is the coherent state of spin 2I in I (x) I, and averaging it over the sphere gives,
        by rotation invariance and irreducibility (Schur's lemma), the projector onto the
        spin-2I subspace divided by its dimension 4I + 1.  For spin 1/2 this is
        (1 + SWAP) / 6, the symmetric-subspace (unitary 2-design) moment.
        """
        N = len(self.sys.two_I)
        kS = self.sys.kS
        if N == 0:
            return float((kS * np.real(self.singlet_block()[0, 0])) ** 2)
        dims = [t + 1 for t in self.sys.two_I]
        A = self.singlet_block().reshape(dims + dims)
        Qs = []
        for t in self.sys.two_I:
            d = t + 1
            ops = spin_ops(t)[:3]
            J2 = sum(np.kron(o, np.eye(d)) @ np.kron(o, np.eye(d)) + 2 * np.kron(o, o)
                     + np.kron(np.eye(d), o) @ np.kron(np.eye(d), o) for o in ops)
            w, V = np.linalg.eigh(J2)
            top = t * (t + 1)                        # J(J+1) with J = 2I = t
            sel = np.abs(w - top) < 1e-8
            assert sel.sum() == 2 * t + 1
            P = V[:, sel] @ V[:, sel].conj().T
            Qs.append((P / (2 * t + 1)).reshape(d, d, d, d))   # [(b, b'), (a, a')]
        letters = iter("abcdefghijklmnopqrstuvwxyzABCDEFGHIJKLMNOPQRSTUVWXYZ")
        i = [next(letters) for _ in range(N)]
        j = [next(letters) for _ in range(N)]
        ip = [next(letters) for _ in range(N)]
        jp = [next(letters) for _ in range(N)]
        terms = ["".join(i + j), "".join(ip + jp)] + [j[k] + jp[k] + i[k] + ip[k] for k in range(N)]
        val = np.einsum(",".join(terms) + "->", A, A, *Qs, optimize="greedy")
        return float(kS * kS * np.real(val))

    def sample_sigma(self):
        """Exact standard deviation of one sample's yield: sqrt(E[phi^2] - Phi_S(T)^2)."""
        return float(np.sqrt(max(0.0, self.second_moment() - self.trace_yield() ** 2)))

    def survival(self, psi0, t):
        """Population N(t) = ||exp(-iGt) psi0||^2."""
        v = sla.expm(-1j * self.G * t) @ psi0
        return float(np.real(np.vdot(v, v)))

    def singlet_probability(self, psi0, t):
        """<psi0(t)|P_S|psi0(t)> at one time t (the integrand of Eq. 22)."""
        v = sla.expm(-1j * self.G * t) @ psi0
        return float(np.real(np.vdot(v, self.sys.PS @ v)))
