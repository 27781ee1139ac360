"""FP64 reference of the control-variate network.  Test infrastructure only.

Features: unit vectors n(Omega_k) of Eq. 16 for every nucleus, then log(B/mT + 0.05),
zero-padded to a multiple of 16.  Network: `depth` hidden layers of `width` units with
the exact (erf) GELU, then a linear scalar output.  Loss: mean squared error.
Parameters are packed per hidden layer as W [fan_in][width] then b [width], followed by
the output weights [width] and the output bias.  Optimiser: Adam (Kingma & Ba 2015).

Parity status: the forward pass is the definition written out; the backward pass is
pinned by central finite differences of the forward pass in the tests.  ``forward`` and
``loss_and_grad`` take an optional operand map ``q`` applied to both operands of every
hidden-layer product (the identity by default, so the oracle stays FP64); a test may pass a
rounding of its own to model a device that rounds those operands.
"""
import numpy as np
from scipy.special import erf


def in_pad(n_in):
    return (n_in + 15) // 16 * 16


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def unpack(p, n_in, width, depth):
    p = np.asarray(p, float)
    layers, o, fan = [], 0, in_pad(n_in)
    for _ in range(depth):
        W = p[o:o + fan * width].reshape(fan, width)
        o += fan * width
        b = p[o:o + width]
        o += width
        layers.append((W, b))
        fan = width
    w = p[o:o + width]
    o += width
    bo = p[o]
    o += 1
    assert o == len(p)
    return layers, w, bo


def param_count(n_in, width, depth):
    return in_pad(n_in) * width + width + (depth - 1) * (width * width + width) + width + 1


def init_params(n_in, width, depth, rng):
    """He-style initialisation (inputs to the library are produced here as well)."""
    parts, fan = [], in_pad(n_in)
    for _ in range(depth):
        parts.append(rng.normal(0.0, np.sqrt(2.0 / fan), fan * width))
        parts.append(np.zeros(width))
        fan = width
    parts.append(rng.normal(0.0, np.sqrt(1.0 / width), width))
    parts.append(np.zeros(1))
    return np.concatenate(parts)


def splitmix_unit(seed, r):
    """u in (0, 1) from SplitMix64 (Steele, Lea & Flood 2014) of seed + (r + 1) * golden gamma:
    the top 53 bits plus one half, times 2^-53."""
    mask = (1 << 64) - 1
    z = (seed + (r + 1) * 0x9E3779B97F4A7C15) & mask
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
    z ^= z >> 31
    return ((z >> 11) + 0.5) * 2.0 ** -53


def features(angles, B_mT, rot_seed=0):
    """Rows field-major: row b*M + s.  rot_seed != 0 advances every azimuth of row r by
    2 pi u_r (a common rotation of the nuclear directions about the field axis)."""
    angles = np.asarray(angles, float)
    M, N = angles.shape[0], angles.shape[1]
    B = np.atleast_1d(np.asarray(B_mT, float))
    x = np.zeros((len(B) * M, in_pad(3 * N + 1)))
    for b, Bv in enumerate(B):
        for s in range(M):
            r = b * M + s
            ct, ph = angles[s, :, 0], angles[s, :, 1].copy()
            if rot_seed:
                ph = ph + 2.0 * np.pi * splitmix_unit(rot_seed, r)
            st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
            x[r, :3 * N] = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=1).reshape(3 * N)
            x[r, 3 * N] = np.log(abs(Bv) + 0.05)
    return x


def _identity(a):
    return a


def forward(p, x, n_in, width, depth, q=None):
    q = q or _identity
    layers, w, bo = unpack(p, n_in, width, depth)
    h = np.asarray(x, float)
    cache = []
    for W, b in layers:
        z = q(h) @ q(W) + b
        cache.append((h, z))
        h = gelu(z)
    return h @ w + bo, (cache, h)


def loss_and_grad(p, x, t, n_in, width, depth, q=None):
    q = q or _identity
    layers, w, bo = unpack(p, n_in, width, depth)
    y, (cache, hl) = forward(p, x, n_in, width, depth, q)
    R = len(t)
    e = y - np.asarray(t, float)
    loss = np.mean(e * e)
    dy = 2.0 * e / R
    gw, gbo = hl.T @ dy, dy.sum()
    dh = np.outer(dy, w)
    grads = []
    for (W, b), (h_in, z) in zip(reversed(layers), reversed(cache)):
        dz = dh * gelu_grad(z)
        grads.append((q(h_in).T @ q(dz), dz.sum(axis=0)))
        dh = q(dz) @ q(W).T
    parts = []
    for gW, gb in reversed(grads):
        parts += [gW.reshape(-1), gb]
    parts += [gw, np.array([gbo])]
    return loss, np.concatenate(parts)


def adam(p, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def cv_beta(phi, g):
    """Per-field regression coefficient Cov(phi, g) / Var(g) over the samples."""
    phi, g = np.asarray(phi, float), np.asarray(g, float)
    pc = phi - phi.mean(axis=-1, keepdims=True)
    gc = g - g.mean(axis=-1, keepdims=True)
    return (pc * gc).sum(axis=-1) / np.maximum((gc * gc).sum(axis=-1), 1e-300)
