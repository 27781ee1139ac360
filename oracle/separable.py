"""Per-radical route for single-wavepacket yields when J = 0 and k_S = k_T.  Test
infrastructure only.

With no exchange term, Eq. 1 is a sum H_1 + H_2 of one Hamiltonian per radical (electron i
with its own nuclei and the Zeeman term), and with k_S = k_T = k the Haberkorn operator of
Eqs. 2-4 is the scalar k/2 (P_S + P_T = 1).  The wavepacket of Eq. 19 evolves as

    psi(t) = e^{-kt/2} (U_1(t) (x) U_2(t)) psi0,    U_i(t) = exp(-i H_i t),

and psi0 = sum_{e1 e2} s_{e1 e2} |e1, Omega^(1)> (x) |e2, Omega^(2)> with the singlet
coefficients s (Eq. 10: s_ab = 1/sqrt2, s_ba = -1/sqrt2).  Write a_e(t) = U_1(t)|e, Omega^(1)>
and a_e^f for its part with radical-1 electron state f (a vector over radical-1 nuclei), and
b likewise for radical 2.  The singlet amplitude of psi(t) is the nuclear vector

    chi(t) = e^{-kt/2} sum_{e, f} s_{e,1-e} s_{f,1-f} a_e^f (x) b_{1-e}^{1-f},

so <psi|P_S|psi> = ||chi||^2 is a contraction of the two 4x4 Gram matrices
G_1[(e f), (e' f')] = <a_e^f | a_e'^f'> and G_2 of radical 2.  The yield of Eq. 22 on [0, T]
is k times the time integral of that, done here by composite 20-point Gauss-Legendre with
panels short against the largest frequency of the integrand.  Each radical is propagated
from node to node by scipy's expm_multiply (Al-Mohy & Higham), a library primitive, on spaces
of dimension 2 Z_i instead of 4 Z.

Ordering (the oracle's own): electron of the radical first, then its nuclei in the caller's
order, each spin in |I, m> with m descending, as in ``spin``.
"""
import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import expm_multiply

from .coherent import coherent_state
from .spin import GAMMA_E, spin_ops

_SIGN = (1.0, -1.0)   # s_{e,1-e} = _SIGN[e] / sqrt(2)


def _embed(op, pos, dims):
    out = sp.identity(1, dtype=complex, format="csr")
    for i, d in enumerate(dims):
        out = sp.kron(out, sp.csr_matrix(op) if i == pos else sp.identity(d, format="csr"), format="csr")
    return out


class Radical:
    """Electron i with its nuclei: H_i = omega S_z + sum_k a_k I_k . S (Eq. 1 with J = 0)."""

    def __init__(self, two_I, a_mT, gamma=GAMMA_E):
        self.two_I = [int(t) for t in two_I]
        self.a = np.asarray(a_mT, float) * gamma
        self.gamma = float(gamma)
        self.dims = [2] + [t + 1 for t in self.two_I]
        self.Zi = int(np.prod(self.dims[1:])) if self.two_I else 1
        e = spin_ops(1)
        S = [_embed(e[c], 0, self.dims) for c in range(3)]
        H = sp.csr_matrix((2 * self.Zi, 2 * self.Zi), dtype=complex)
        for k, t in enumerate(self.two_I):
            nuc = spin_ops(t)
            for c in range(3):
                H = H + self.a[k] * (_embed(nuc[c], 1 + k, self.dims) @ S[c])
        self.Hhf = H.tocsr()
        self.Sz = S[2].tocsr()

    def H(self, B_mT):
        return (self.Hhf + self.gamma * float(B_mT) * self.Sz).tocsr()

    def states(self, angles):
        """Columns |alpha, Omega> and |beta, Omega> (angles: [n][2] of (cos theta, phi))."""
        nuc = np.array([1.0 + 0j])
        for k, t in enumerate(self.two_I):
            nuc = np.kron(nuc, coherent_state(t, float(angles[k][0]), float(angles[k][1])))
        out = np.zeros((2 * self.Zi, 2), complex)
        out[:self.Zi, 0] = nuc
        out[self.Zi:, 1] = nuc
        return out


def _gram(v, Zi):
    """G[(e f), (e' f')] = <v_e^f | v_e'^f'> for v = [a_alpha, a_beta] (2 Zi x 2)."""
    parts = np.stack([v[f * Zi:(f + 1) * Zi, e] for e in (0, 1) for f in (0, 1)], axis=1)   # (e f) = 2e+f
    return parts.conj().T @ parts


def _singlet_population(G1, G2):
    """||chi||^2 / e^{-kt} from the two Gram matrices."""
    tot = 0.0 + 0j
    for e in (0, 1):
        for f in (0, 1):
            for e2 in (0, 1):
                for f2 in (0, 1):
                    w = _SIGN[e] * _SIGN[f] * _SIGN[e2] * _SIGN[f2] / 4.0
                    tot += w * G1[2 * e + f, 2 * e2 + f2] * G2[2 * (1 - e) + (1 - f), 2 * (1 - e2) + (1 - f2)]
    return float(tot.real)


def yield_separable(n_nuc, two_I, a_mT, k, B_mT, T, angles, gamma=GAMMA_E, nodes=20):
    """phi_S = k int_0^T <psi|P_S|psi> dt for J = 0 and k_S = k_T = k (Eq. 22 on [0, T]).

    ``angles`` is [N][2] (cos theta, phi) per nucleus, radical 1 first.
    """
    N1 = int(n_nuc[0])
    rads = [Radical(two_I[:N1], a_mT[:N1], gamma), Radical(two_I[N1:], a_mT[N1:], gamma)]
    Hs = [r.H(B_mT) for r in rads]
    vs = [rads[0].states(angles[:N1]), rads[1].states(angles[N1:])]
    # Largest frequency of the integrand: differences of eigenvalues of both radicals, bounded
    # by twice the sum of the 1-norms.
    W = 2.0 * sum(abs(H).sum(axis=0).max() for H in Hs)
    n_panels = max(1, int(np.ceil(W * T / 2.0)))
    x, w = np.polynomial.legendre.leggauss(nodes)
    h = T / n_panels
    t_prev = 0.0
    total = 0.0
    for p in range(n_panels):
        t0 = p * h
        for xi, wi in zip(x, w):
            t = t0 + 0.5 * h * (xi + 1.0)
            dt = t - t_prev
            vs = [expm_multiply(-1j * dt * H, v) for H, v in zip(Hs, vs)]
            t_prev = t
            ps = _singlet_population(_gram(vs[0], rads[0].Zi), _gram(vs[1], rads[1].Zi))
            total += 0.5 * h * wi * np.exp(-k * t) * ps
    return k * total
