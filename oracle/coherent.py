"""Spin coherent states and product initial wavepackets (Sec. III).  Test infrastructure only.

A direction is given as (cos theta, phi) with 0 <= theta <= pi, 0 <= phi < 2 pi.
"""
import math

import numpy as np

from .spin import spin_ops


def coherent_state(two_I, cos_theta, phi):
    """|Omega_J> of Eq. 15 in the |J,m> basis (m descending), J = two_I/2.

    Eq. 15 is (cos theta/2)^{2J} exp(tan(theta/2) e^{i phi} J_-)|J,J>.  The
    exponential of the nilpotent J_- is its finite power series; the prefactor
    (cos theta/2)^{2J} is distributed over the series terms so that the
    n-th term carries (cos theta/2)^{2J-n} (sin theta/2)^n, which is the same
    vector but stays finite at theta = pi (where tan diverges).
    """
    d = two_I + 1
    c = math.sqrt(max(0.0, 0.5 * (1.0 + cos_theta)))   # cos(theta/2), theta in [0, pi]
    s = math.sqrt(max(0.0, 0.5 * (1.0 - cos_theta)))   # sin(theta/2)
    Jm = spin_ops(two_I)[4]
    top = np.zeros(d, complex)
    top[0] = 1.0                                        # |J, J>
    out = np.zeros(d, complex)
    term = top.copy()                                   # J_-^n |J,J>
    for n in range(d):
        out += (c ** (two_I - n)) * (s * np.exp(1j * phi)) ** n / math.factorial(n) * term
        term = Jm @ term
    return out


def initial_wavepacket(system, angles):
    """|S> (x) |Omega_1> (x) ... (x) |Omega_N> (Eq. 18-19), in the oracle's ordering.

    ``angles`` is an (N, 2) array of (cos theta, phi), radical-1 nuclei first.
    """
    v = system.singlet.astype(complex)
    for k, t in enumerate(system.two_I):
        v = np.kron(v, coherent_state(t, float(angles[k][0]), float(angles[k][1])))
    return v


def basis_wavepacket(system, digits):
    """|S, M_1, M_2> of Eq. 12: nuclear digit n_k = I_k - m_k selects |I_k, m_k>."""
    v = system.singlet.astype(complex)
    for k, t in enumerate(system.two_I):
        e = np.zeros(t + 1, complex)
        e[int(digits[k])] = 1.0
        v = np.kron(v, e)
    return v


def unit_vector(cos_theta, phi):
    """n(Omega) of Eq. 16."""
    st = math.sqrt(max(0.0, 1.0 - cos_theta * cos_theta))
    return np.array([st * math.cos(phi), st * math.sin(phi), cos_theta])
