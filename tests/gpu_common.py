"""Shared helpers of the GPU tests: oracle evaluation for a workload system."""
import numpy as np

from oracle import coherent, large, philox, spin, yields


def dense(sysd):
    return spin.DenseSystem((sysd.n1, sysd.n2), sysd.two_I, sysd.a_mT, J_mT=sysd.J_mT, kS=sysd.kS,
                            kT=sysd.kT, gamma=sysd.gamma)


def oracle_phi(sysd, fields, angles, basis=False):
    """[nB][M] exact yields from the dense oracle."""
    d = dense(sysd)
    out = np.zeros((len(fields), len(angles)))
    for b, B in enumerate(fields):
        fo = yields.FieldOracle(d, B, sysd.T_us)
        for s, a in enumerate(angles):
            psi = (coherent.basis_wavepacket(d, a[:, 0].astype(int)) if basis
                   else coherent.initial_wavepacket(d, a))
            out[b, s] = fo.phi(psi)
    return out


def oracle_phi_sparse(sysd, fields, angles):
    sp = large.SparseSystem((sysd.n1, sysd.n2), sysd.two_I, sysd.a_mT, J_mT=sysd.J_mT, kS=sysd.kS,
                            kT=sysd.kT, gamma=sysd.gamma)
    out = np.zeros((len(fields), len(angles)))
    for b, B in enumerate(fields):
        for s, a in enumerate(angles):
            out[b, s], _ = large.yield_augmented(sp, B, sysd.T_us, sp.wavepacket(a))
    return out


def oracle_trace(sysd, B):
    return yields.FieldOracle(dense(sysd), B, sysd.T_us).trace_yield()
