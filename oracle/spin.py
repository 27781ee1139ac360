"""Dense radical-pair operators (Sec. II, Eqs. 1-4).  Test infrastructure only.

Basis and ordering (the oracle's own; the GPU library chooses its own layout):
the full space is the Kronecker product  S_1 (x) S_2 (x) I_1 (x) ... (x) I_N,
radical-1 nuclei first, each spin in its |I, m> basis ordered m = I, I-1, ..., -I.
Units: couplings, exchange and field in mT are multiplied by gamma to give
angular frequencies in rad/us; rate constants are in 1/us; hbar = 1.
"""
import numpy as np

GAMMA_E = 176.085963023  # |gamma_e| in rad us^-1 mT^-1 (CODATA 2018)


def spin_ops(two_I):
    """Spin operators (Ix, Iy, Iz, I+, I-) of spin I = two_I/2 in |I,m>, m descending."""
    d = two_I + 1
    I = two_I / 2.0
    m = I - np.arange(d)
    Iz = np.diag(m).astype(complex)
    Ip = np.zeros((d, d), complex)
    for col in range(1, d):           # |m> -> |m+1>, row index one lower
        mm = m[col]
        Ip[col - 1, col] = np.sqrt(I * (I + 1) - mm * (mm + 1))
    Im = Ip.conj().T
    Ix = 0.5 * (Ip + Im)
    Iy = -0.5j * (Ip - Im)
    return Ix, Iy, Iz, Ip, Im


def _embed(op, pos, dims):
    """Kronecker embedding of a single-spin operator at slot ``pos``."""
    out = np.array([[1.0 + 0j]])
    for i, d in enumerate(dims):
        out = np.kron(out, op if i == pos else np.eye(d))
    return out


class DenseSystem:
    """Operators of Eq. 1-4 for one radical pair.

    Parameters mirror the problem statement: ``n_nuc = (N1, N2)``,
    ``two_I`` (2I per nucleus, radical 1 first), ``a_mT`` (isotropic a_ik/gamma
    in mT), ``J_mT`` (exchange, term 2J S1.S2), ``kS``, ``kT`` (1/us).
    """

    def __init__(self, n_nuc, two_I, a_mT, J_mT=0.0, kS=1.0, kT=1.0, gamma=GAMMA_E):
        self.N1, self.N2 = int(n_nuc[0]), int(n_nuc[1])
        self.two_I = [int(t) for t in two_I]
        self.a = np.asarray(a_mT, float) * gamma
        self.J = float(J_mT) * gamma
        self.kS, self.kT, self.gamma = float(kS), float(kT), float(gamma)
        N = self.N1 + self.N2
        assert len(self.two_I) == N and len(self.a) == N
        self.dims = [2, 2] + [t + 1 for t in self.two_I]
        self.Z = int(np.prod([t + 1 for t in self.two_I])) if N else 1
        self.dim = 4 * self.Z
        e = spin_ops(1)
        S = [[_embed(e[c], s, self.dims) for c in range(3)] for s in (0, 1)]
        self.S = S
        S1dotS2 = sum(S[0][c] @ S[1][c] for c in range(3))
        one = np.eye(self.dim)
        # Eq. 3-4: singlet and triplet projectors
        self.PS = 0.25 * one - S1dotS2
        self.PT = 0.75 * one + S1dotS2
        # Eq. 1 without the Zeeman term (added per field)
        Hhf = 2.0 * self.J * S1dotS2
        for k in range(N):
            rad = 0 if k < self.N1 else 1
            nuc = spin_ops(self.two_I[k])
            for c in range(3):
                Hhf = Hhf + self.a[k] * _embed(nuc[c], 2 + k, self.dims) @ S[rad][c]
        self.Hhf = Hhf
        self.Sz_tot = S[0][2] + S[1][2]
        # Eq. 2: Haberkorn operator
        self.K = 0.5 * self.kS * self.PS + 0.5 * self.kT * self.PT
        self.singlet = self._singlet_vector()

    def H(self, B_mT):
        """Eq. 1 with omega = gamma*B along z (the yield is even in omega)."""
        return self.Hhf + self.gamma * float(B_mT) * self.Sz_tot

    def G(self, B_mT):
        """Non-Hermitian generator G = H - iK of exp(-iHt - Kt) (Eq. 6, 13)."""
        return self.H(B_mT) - 1j * self.K

    @staticmethod
    def _singlet_vector():
        up, dn = np.array([1.0, 0.0]), np.array([0.0, 1.0])
        return (np.kron(up, dn) - np.kron(dn, up)) / np.sqrt(2.0)

    def Bhyp(self):
        """Effective hyperfine field of each radical in mT (Eq. 21)."""
        out = []
        for lo, hi in ((0, self.N1), (self.N1, self.N1 + self.N2)):
            s = sum((self.a[k] / self.gamma) ** 2 * (self.two_I[k] / 2) * (self.two_I[k] / 2 + 1)
                    for k in range(lo, hi))
            out.append(np.sqrt(s))
        return out
