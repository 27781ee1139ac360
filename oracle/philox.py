"""Counter-based random directions for the Monte Carlo trace (Eq. 18).  Test infrastructure only.

Philox4x64-10 as published by Salmon, Moraes, Dror & Shaw, "Parallel random
numbers: as easy as 1, 2, 3" (SC'11): a 4x64-bit counter, a 2x64-bit key,
ten rounds of two 64x64->128 multiplications with a Weyl-sequence key bump.

Stream layout (the paper does not specify one): for sample s (global index)
and nucleus k the block is Philox(counter = (s, k, 0, 0), key = (seed, stream)).
Word 0 gives u1, word 1 gives u2, each as u = (floor(w / 2^12) + 1/2) * 2^-52,
which is exact in binary64 and lies strictly inside (0, 1).  The direction is
uniform on the unit sphere (the measure dOmega / 4 pi of Eq. 18):
cos theta = 2 u1 - 1 and phi = 2 pi u2.
"""
import math

import numpy as np
from scipy.linalg import hadamard

_MASK = (1 << 64) - 1
_M0, _M1 = 0xD2E7470EE14C6C93, 0xCA5A826395121157      # round multipliers
_W0, _W1 = 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B      # key increments

STREAM_EVAL, STREAM_TRAIN, STREAM_QUAD, STREAM_SYSTEM = 0, 1, 2, 3


def philox4x64(counter, key, rounds=10):
    """One Philox4x64 block: four 64-bit outputs for a 4-word counter and 2-word key."""
    c = [int(x) & _MASK for x in counter]
    k = [int(x) & _MASK for x in key]
    for r in range(rounds):
        if r:
            k = [(k[0] + _W0) & _MASK, (k[1] + _W1) & _MASK]
        p0, p1 = _M0 * c[0], _M1 * c[2]
        c = [(p1 >> 64) ^ c[1] ^ k[0], p1 & _MASK, (p0 >> 64) ^ c[3] ^ k[1], p0 & _MASK]
    return c


def word_to_unit(w):
    """Map a 64-bit word to (q + 1/2) 2^-52, q = its top 52 bits."""
    return ((int(w) >> 12) + 0.5) * 2.0 ** -52


TWO_PI = 2.0 * math.pi


def sample_angles(seed, first_sample, M, N, stream=STREAM_EVAL):
    """Directions for samples first_sample .. first_sample+M-1: array [M][N][2] of (cos theta, phi)."""
    out = np.empty((M, N, 2), float)
    for s in range(M):
        for k in range(N):
            w = philox4x64((first_sample + s, k, 0, 0), (seed, stream))
            u1, u2 = word_to_unit(w[0]), word_to_unit(w[1])
            out[s, k, 0] = 2.0 * u1 - 1.0
            out[s, k, 1] = TWO_PI * u2
    return out


def flip(angles, mask):
    """Antipodal direction n -> -n for the nuclei selected by ``mask`` (bool array [N])."""
    a = np.array(angles, float, copy=True)
    a[mask, 0] = -a[mask, 0]
    a[mask, 1] = np.mod(a[mask, 1] + math.pi, TWO_PI)
    return a


def design_rows(N, mode):
    """Sign-flip design for N nuclei as a [R][N] array of +-1 (row r, nucleus k).

    mode 3, antithetic pairs: R = 2, rows (+1, ..., +1) and (-1, ..., -1).
    mode 4, fold-over of the Sylvester-Hadamard matrix H of order n (n the smallest power of
    two >= N, columns 0 .. N-1): rows H[r] for r < n and -H[r - n] for r >= n, R = 2n.  The
    fold-over cancels every odd product of columns and the orthogonality of Hadamard columns
    every product of two, so the rows form an orthogonal array of strength 3.
    mode 5, columns 1 .. N of the Sylvester-Hadamard matrix of order n (n the smallest power
    of two > N), R = n: every column but the first is balanced and any two are orthogonal, an
    orthogonal array of strength 2.
    """
    if mode == 3:
        return np.array([[1] * N, [-1] * N], int)
    n = 1
    while n < (N + 1 if mode == 5 else N):
        n *= 2
    if mode == 5:
        return hadamard(n)[:, 1:N + 1]
    H = hadamard(n)[:, :N]
    return np.concatenate([H, -H], axis=0)


def sample_design(seed, first_sample, M, N, mode, stream=STREAM_EVAL):
    """Directions of a sign-flip design (modes 3, 4 and 5 of the sampler): global sample index
    q = first_sample + s belongs to group g = q // R and row r = q % R of ``design_rows``; the
    group draws one set of directions as ``sample_angles`` does for sample g, and row r takes
    n_k -> -n_k wherever its sign is -1.  Every sample is marginally uniform on the spheres, so
    the mean over a group is an unbiased estimate of the Eq. 18 trace, and the groups are
    independent."""
    D = design_rows(N, mode)
    R = D.shape[0]
    out = np.empty((M, N, 2), float)
    for s in range(M):
        q = first_sample + s
        base = sample_angles(seed, q // R, 1, N, stream)[0]
        out[s] = flip(base, D[q % R] < 0)
    return out


def sample_basis_digits(seed, first_sample, M, two_I, stream=STREAM_EVAL):
    """Random J_z eigenstates (Sec. V, last paragraph): digit n_k = floor(u1 (2I_k + 1)),
    u1 from word 0 of the same Philox block as the coherent-state sampler."""
    N = len(two_I)
    out = np.zeros((M, N, 2), float)
    for s in range(M):
        for k in range(N):
            w = philox4x64((first_sample + s, k, 0, 0), (seed, stream))
            d = two_I[k] + 1
            out[s, k, 0] = min(int(word_to_unit(w[0]) * d), d - 1)
    return out


def enumerate_basis_digits(first_sample, M, two_I):
    """Deterministic enumeration of the basis of Eq. 12: sample s -> mixed-radix digits of s
    (first nucleus fastest), so samples 0..Z-1 visit every |M_1, M_2> once (Eq. 14)."""
    N = len(two_I)
    out = np.zeros((M, N, 2), float)
    for s in range(M):
        q = first_sample + s
        for k in range(N):
            d = two_I[k] + 1
            out[s, k, 0] = q % d
            q //= d
    return out
