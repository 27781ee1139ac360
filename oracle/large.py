"""Exact single-wavepacket yields for state sizes beyond dense matrices.  Test infrastructure only.

The integrand of Eq. 22 is quadratic in the wavepacket, but its time integral
follows from a linear system of twice the size.  With psi' = -iG psi
(Eq. 13) and chi' = -iG^dag chi + P_S psi, chi(t0) = 0, one has

    <psi(t0+tau) | chi(t0+tau)> = int_{t0}^{t0+tau} <psi(t)|P_S|psi(t)> dt,

because chi(t0+tau) = int exp(-iG^dag (t0+tau-t)) P_S psi(t) dt.  The block
lower-triangular generator [[-iG, 0], [P_S, -iG^dag]] is applied with
scipy's expm_multiply (Al-Mohy & Higham), a library primitive.  chi grows like
exp(k_max t/2) while psi decays, so the horizon is cut into chunks of length
``tau`` and chi restarts from zero in each chunk; the yield is k_S times the
sum of the chunk integrals.

Operators are the same Eq. 1-4 terms as ``spin.DenseSystem``, assembled as
sparse Kronecker products in the same ordering (S_1, S_2, nuclei).
"""
import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import expm_multiply

from .spin import GAMMA_E, spin_ops


def _embed(op, pos, dims):
    out = sp.identity(1, dtype=complex, format="csr")
    for i, d in enumerate(dims):
        out = sp.kron(out, sp.csr_matrix(op) if i == pos else sp.identity(d, format="csr"), format="csr")
    return out


class SparseSystem:
    """Sparse operators of Eq. 1-4 (same parameters as ``spin.DenseSystem``)."""

    def __init__(self, n_nuc, two_I, a_mT, J_mT=0.0, kS=1.0, kT=1.0, gamma=GAMMA_E):
        self.N1, self.N2 = int(n_nuc[0]), int(n_nuc[1])
        self.two_I = [int(t) for t in two_I]
        self.a = np.asarray(a_mT, float) * gamma
        self.J = float(J_mT) * gamma
        self.kS, self.kT, self.gamma = float(kS), float(kT), float(gamma)
        N = self.N1 + self.N2
        self.dims = [2, 2] + [t + 1 for t in self.two_I]
        self.Z = int(np.prod([t + 1 for t in self.two_I])) if N else 1
        self.dim = 4 * self.Z
        e = spin_ops(1)
        S = [[_embed(e[c], s, self.dims) for c in range(3)] for s in (0, 1)]
        S1dotS2 = sum(S[0][c] @ S[1][c] for c in range(3))
        one = sp.identity(self.dim, dtype=complex, format="csr")
        self.PS = (0.25 * one - S1dotS2).tocsr()
        Hhf = 2.0 * self.J * S1dotS2
        for k in range(N):
            rad = 0 if k < self.N1 else 1
            nuc = spin_ops(self.two_I[k])
            for c in range(3):
                Hhf = Hhf + self.a[k] * (_embed(nuc[c], 2 + k, self.dims) @ S[rad][c])
        self.Hhf = Hhf.tocsr()
        self.Sz_tot = (S[0][2] + S[1][2]).tocsr()
        PT = (0.75 * one + S1dotS2)
        self.K = (0.5 * self.kS * self.PS + 0.5 * self.kT * PT).tocsr()
        up, dn = np.array([1.0, 0.0]), np.array([0.0, 1.0])
        self.singlet = (np.kron(up, dn) - np.kron(dn, up)) / np.sqrt(2.0)

    def G(self, B_mT):
        return (self.Hhf + self.gamma * float(B_mT) * self.Sz_tot - 1j * self.K).tocsr()

    def wavepacket(self, angles):
        from .coherent import coherent_state
        v = self.singlet.astype(complex)
        for k, t in enumerate(self.two_I):
            v = np.kron(v, coherent_state(t, float(angles[k][0]), float(angles[k][1])))
        return v


def yield_augmented(system, B_mT, T, psi0, tau=1.0):
    """phi_S = k_S int_0^T <psi|P_S|psi> dt by the chunked augmented system."""
    G = system.G(B_mT)
    n = system.dim
    Aug = sp.bmat([[-1j * G, None], [system.PS, -1j * G.conj().T]], format="csr")
    nchunk = max(1, int(np.ceil(T / tau)))
    h = T / nchunk
    psi = np.asarray(psi0, complex)
    total = 0.0
    for _ in range(nchunk):
        v = np.concatenate([psi, np.zeros(n, complex)])
        w = expm_multiply(h * Aug, v)
        psi, chi = w[:n], w[n:]
        total += float(np.real(np.vdot(psi, chi)))
    return system.kS * total, psi
