"""Host-side checks of librp that need no GPU: exports, argument validation and the
Chebyshev/quadrature plan (Bessel coefficients, in-step quadrature factor), the
latter checked by driving a dense CPU emulation of the propagation with the
library's own plan and comparing against the oracle."""
import ctypes
import dataclasses
import math
import os
import re

import numpy as np
import pytest
import scipy.special as ss

from oracle import coherent, philox, spin, yields
from paper_1612_09517_amd import rp
from paper_1612_09517_amd.workloads import SpinSystem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "rp.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(rp_\w+)\s*\(", src, re.M)))


def test_header_declares_expected_entry_points():
    assert set(_declared()) == set(rp.EXPORTS)


def test_library_loads_and_exports_every_declared_symbol():
    L = rp.lib()
    for name in _declared():
        assert hasattr(L, name), name


@pytest.mark.parametrize("x", [0.0, 1e-3, 0.7, 5.0, 39.9, 80.0, 200.0, 600.0])
def test_bessel_matches_scipy(x):
    nmax = int(x) + 60
    got = rp.bessel_j(x, nmax)
    want = ss.jv(np.arange(nmax + 1), x)
    assert np.max(np.abs(got - want)) < 2e-14 * max(1.0, math.sqrt(x) / 3)


def _sys(**kw):
    d = dict(n1=2, n2=1, two_I=[1, 1, 1], a_mT=[0.8, 0.3, 0.5], J_mT=0.0, kS=1.0, kT=1.0, T_us=10.0)
    d.update(kw)
    return SpinSystem(**d)


def test_plan_coefficients_are_bessel_series():
    s = _sys(kS=2.0, kT=0.5)
    p = rp.plan_field(s, 1.0)
    n = np.arange(p["n_terms"])
    want = np.where(n == 0, 1.0, 2.0) * (-1j) ** n * ss.jv(n, p["x"]) * np.exp(-1j * p["c"] * p["dt"])
    assert np.max(np.abs(p["coef"] - want)) < 1e-14
    assert abs(p["c"].imag - (-0.25 * 1.5)) < 1e-15
    assert abs(p["n_steps"] * p["dt"] - s.T_us) < 1e-12
    assert abs(p["x"] - p["r"] * p["dt"]) < 1e-12
    assert p["x"] <= 100.0 + 1e-9                       # default step


@pytest.mark.parametrize("two_I,J,B", [([1, 1, 1], 0.0, 0.0), ([1, 2, 1], 0.7, 2.5), ([2, 1, 3], -0.4, 6.0)])
def test_plan_spectral_interval_contains_spectrum(two_I, J, B):
    """[c - r, c + r] contains every eigenvalue of H (dense eigvalsh) and is tight."""
    s = _sys(two_I=two_I, J_mT=J, a_mT=[0.8, -0.3, 0.5])
    d = spin.DenseSystem((s.n1, s.n2), s.two_I, s.a_mT, J_mT=J)
    ev = np.linalg.eigvalsh(d.H(B))
    p = rp.plan_field(s, B)
    c, r = p["c"].real, p["r"]
    assert c - r <= ev.min() and ev.max() <= c + r
    assert r <= 1.02 * (0.5 * (ev.max() - ev.min())) + 1.5 * abs(J) * s.gamma + 1e-9


def test_plan_quadrature_factor():
    """ell ell^T equals (2-d_m0)(2-d_n0)/2 int_0^dt J_m(rs) J_n(rs) exp(-(kS+kT)s/2) ds."""
    s = _sys(kS=2.0, kT=0.5)
    p = rp.plan_field(s, 0.3, rdt=12.0)
    nt = p["n_terms"]
    xg, wg = np.polynomial.legendre.leggauss(200)
    sq = 0.5 * p["dt"] * (xg + 1)
    w = 0.5 * p["dt"] * wg * np.exp(-1.25 * sq)
    Jm = ss.jv(np.arange(nt)[:, None], p["r"] * sq[None, :])
    K = (Jm * w) @ Jm.T
    f = np.where(np.arange(nt) == 0, 1.0, 2.0) / math.sqrt(2)
    assert np.max(np.abs(p["ell"] @ p["ell"].T - np.outer(f, f) * K)) < 1e-15 * 4 * p["dt"] + 1e-17


def _emulate(sysd, B, angles, precision=64):
    """Dense CPU emulation of the GPU algorithm, driven by the library's plan."""
    d = spin.DenseSystem((sysd.n1, sysd.n2), sysd.two_I, sysd.a_mT, J_mT=sysd.J_mT, kS=sysd.kS, kT=sysd.kT)
    p = rp.plan_field(sysd, B, precision=precision)
    kmin = min(sysd.kS, sysd.kT)
    Gp = d.G(B) + 0.5j * kmin * np.eye(d.dim)
    Gh = (Gp - p["c"] * np.eye(d.dim)) / p["r"]
    psi = coherent.initial_wavepacket(d, angles)
    out = 0.0
    for j in range(p["n_steps"]):
        ph = [psi, Gh @ psi]
        for _ in range(2, p["n_terms"]):
            ph.append(2 * Gh @ ph[-1] - ph[-2])
        # singlet amplitude times sqrt 2 in the oracle's ordering (S1, S2, nuclei)
        amp = np.array([np.kron(d.singlet * math.sqrt(2), np.eye(d.Z)).conj() @ v for v in ph])
        rot = (-1j) ** np.arange(p["n_terms"])
        W = p["ell"].T @ (rot[:, None] * amp)
        out += sysd.kS * math.exp(-kmin * j * p["dt"]) * np.sum(np.abs(W) ** 2)
        psi = sum(a * v for a, v in zip(p["coef"], ph))
    return out


@pytest.mark.parametrize("kS,kT,J,B", [(1.0, 1.0, 0.0, 0.0), (2.0, 0.5, 0.0, 3.0), (0.3, 2.5, 0.6, 1.0)])
def test_plan_drives_exact_yield(kS, kT, J, B):
    sysd = _sys(kS=kS, kT=kT, J_mT=J, T_us=2.0)
    d = spin.DenseSystem((sysd.n1, sysd.n2), sysd.two_I, sysd.a_mT, J_mT=J, kS=kS, kT=kT)
    fo = yields.FieldOracle(d, B, sysd.T_us)
    for a in philox.sample_angles(4, 0, 2, 3):
        want = fo.phi(coherent.initial_wavepacket(d, a))
        assert abs(_emulate(sysd, B, a) - want) < 1e-11 * want


def test_argument_validation_without_device():
    L = rp.lib()
    good = _sys()
    cs = rp._CSystem(good)
    bad = rp._CSystem(_sys(kS=-1.0))
    B = np.zeros(2)
    dp = B.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    fake = ctypes.c_void_p(16)
    assert L.rp_propagate(ctypes.byref(bad.c), 1, dp, 2, fake, 4, None, fake, None, None) == rp.RP_EINVAL
    assert L.rp_propagate(ctypes.byref(cs.c), 1, dp, 2, fake, 4, None, fake, fake, None) == rp.RP_EINVAL   # ps_t_len 0
    oa = rp._opts(flags=rp.RP_FLAG_ARNOLDI, ps_t_len=4)
    assert L.rp_propagate(ctypes.byref(cs.c), 1, dp, 2, fake, 4, ctypes.byref(oa), fake, fake, None) == rp.RP_ENOTIMPL
    on = rp._opts(ps_t_len=-1)
    assert L.rp_propagate(ctypes.byref(cs.c), 1, dp, 2, fake, 4, ctypes.byref(on), fake, None, None) == rp.RP_EINVAL
    assert L.rp_propagate(ctypes.byref(cs.c), 1, None, 2, fake, 4, None, fake, None, None) == rp.RP_EINVAL
    o = rp._opts(precision=16)
    assert L.rp_propagate(ctypes.byref(cs.c), 1, dp, 2, fake, 4, ctypes.byref(o), fake, None, None) == rp.RP_EINVAL
    assert L.rp_sample(ctypes.byref(cs.c), 1, 0, 0, -1, 0, fake, None) == rp.RP_EINVAL
    assert L.rp_sample(ctypes.byref(cs.c), 1, 0, 0, 4, 7, fake, None) == rp.RP_EINVAL
    assert L.rp_sample(ctypes.byref(cs.c), 1, 0, 0, 4, 6, fake, None) == rp.RP_EINVAL
    assert L.rp_group_mean(fake, 3, 10, 4, fake, None) == rp.RP_EINVAL       # 4 does not divide 10
    assert L.rp_group_mean(fake, 3, 10, 0, fake, None) == rp.RP_EINVAL
    assert L.rp_group_mean(None, 3, 10, 5, fake, None) == rp.RP_EINVAL
    assert L.rp_group_mean(fake, 0, 10, 5, fake, None) == rp.RP_OK           # nothing to do
    big = rp._CSystem(SpinSystem(1, 0, [5], [0.1]))
    assert L.rp_sample(ctypes.byref(big.c), 1, 0, 0, 4, 0, fake, None) == rp.RP_EINVAL
    assert L.rp_yield(None, 3, 4, None, None, None, None, fake, fake, None) == rp.RP_EINVAL
    assert L.rp_yield(fake, 3, 4, fake, None, None, None, fake, fake, None) == rp.RP_EINVAL
    assert b"two_I" in L.rp_last_error() or len(L.rp_last_error()) > 0
    assert L.rp_strerror(rp.RP_ENOTCONV).startswith(b"propagation")


def test_autotune_cache_hit_needs_no_probe(tmp_path):
    """A cached entry for the system's shape is returned as it is (no timed probes, so no
    device is needed); the key carries the precision, the spins per radical and the spectral
    scale, so another precision misses."""
    import json
    from paper_1612_09517_amd import autotune
    s = _sys(kS=2.0, kT=0.5)
    B = [0.0, 2.0, 4.0]
    r_max = max(rp.plan_field(s, b, precision=32)["r"] for b in (0.0, 4.0))
    key = autotune._key(s, 32, r_max)
    cache = tmp_path / "tune.json"
    cache.write_text(json.dumps({key: {"best": {"rdt": 120.0, "xcd": "spread"}, "probes": []}}))
    assert autotune.tune(s, B, precision=32, cache=str(cache)) == {"rdt": 120.0, "xcd": "spread"}
    assert autotune._key(s, 64, r_max) != key


def test_design_size_matches_oracle_design():
    """Samples per group of the sign-flip designs against the oracle's design matrices."""
    from oracle import philox
    for N in range(0, 41):
        for mode in (0, 1, 2):
            assert rp.design_size(N, mode) == 1
        for mode in (3, 4, 5):
            if N:
                assert rp.design_size(N, mode) == philox.design_rows(N, mode).shape[0]
    assert rp.lib().rp_design_size(3, 6) == rp.RP_EINVAL
    assert rp.lib().rp_design_size(-1, 4) == rp.RP_EINVAL
    with pytest.raises(rp.RpError):
        rp.design_size(3, 9)


def test_bench_refuses_more_than_one_gpu():
    """bench.py --gpus N > 1 stops with a message before touching a GPU."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stdout


def test_autotune_dimensions_follow_the_system():
    """The tuner searches only the choices that exist for a system: the tile kernel's index pairs
    need complex FP32 and 8 leading spin-1/2 nuclei; the LDS-resident path needs a small state;
    the axis order matters only when spins are mixed."""
    from paper_1612_09517_amd import autotune
    big = SpinSystem(7, 7, [1] * 14, [0.1] * 14)
    small = SpinSystem(4, 4, [1] * 8, [0.1] * 8)
    mixed = SpinSystem(5, 5, [2] + [1] * 9, [0.1] * 10)
    names = lambda s, p: [n for n, _ in autotune.dimensions(s, p)]
    assert names(big, 32) == ["xcd", "term_scalar"]
    assert names(big, 64) == ["xcd"]
    assert names(small, 32) == ["xcd", "term_scalar", "tiled"]
    assert names(small, 64) == ["xcd", "tiled"]
    assert names(mixed, 32) == ["xcd", "term_scalar", "axes_high_first"]


def test_autotune_probe_horizon_is_whole_steps():
    """Every candidate step length is probed over exactly 12 of its own steps at the highest
    field (as the library's planner counts them), so that rounding the step count up costs every
    candidate the same; a horizon shorter than that is probed as it is."""
    from paper_1612_09517_amd import autotune, workloads
    s = workloads.sweep_c2().systems[0]
    B = 10.0
    for prec in (32, 64):
        r_max = rp.plan_field(s, B, precision=prec)["r"]
        for rdt in autotune.RDT:
            T = autotune.probe_horizon(s, rdt, r_max)
            probe = dataclasses.replace(s, T_us=T)
            assert rp.plan_field(probe, B, precision=prec, rdt=rdt)["n_steps"] == 12, (prec, rdt)
    short = dataclasses.replace(s, T_us=0.01)
    assert autotune.probe_horizon(short, 150.0, 100.0) == 0.01


def test_sequential_stopping_rule_reaches_eps():
    """The bench's stopping rule (shared by every estimator of the headline) on synthetic units
    of known spread: every field ends at or below eps, with about (sigma/eps)^2 units (the rule
    adds 5 % and rounds up), in a few rounds; fields that start below eps get no more units."""
    import torch
    import bench
    rng = np.random.default_rng(3)
    sig = np.array([0.02, 0.05, 0.0005, 0.03])
    eps = 1e-3

    def draw(fields, n, first):
        return torch.tensor(rng.normal(0.5, 1.0, (len(fields), n)) * sig[fields][:, None])

    def stats(f, u):
        u = u.numpy()
        e = u.std(ddof=1) / np.sqrt(len(u))
        return float(u.mean()), float(e), float(e / eps)

    mean, err, done, rounds = bench.sequential_sweep(len(sig), eps, 64, draw, stats, lambda m: None, "test")
    assert np.all(err <= eps) and rounds <= 4
    need = (sig / eps) ** 2
    assert done[2] == 64                                   # already below eps after the first round
    for f in (0, 1, 3):
        assert 0.8 * need[f] < done[f] < 1.6 * need[f], (f, done[f], need[f])
