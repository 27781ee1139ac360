"""Seeded synthetic radical-pair workloads.

This module only draws and lists inputs (spin quantum numbers, hyperfine
couplings, rate constants, fields, horizons, sample counts).  It holds none of
the method's arithmetic, imports nothing else from this package, and is the
one module read both by the GPU path and by the CPU checker.

Units: couplings, exchange and fields in mT; rate constants in 1/us; times in
us.  Couplings are drawn with numpy's PCG64 generator from a fixed per-workload
seed.
"""
from dataclasses import dataclass, field
from typing import List

import numpy as np

GAMMA_E = 176.085963023  # |gamma_e| / (rad us^-1 mT^-1), CODATA 2018


@dataclass
class SpinSystem:
    """One radical pair: nuclei of radical 1 first, then radical 2."""
    n1: int
    n2: int
    two_I: List[int]
    a_mT: List[float]
    J_mT: float = 0.0
    kS: float = 1.0
    kT: float = 1.0
    T_us: float = 10.0
    gamma: float = GAMMA_E
    name: str = ""

    @property
    def N(self):
        return self.n1 + self.n2

    @property
    def Z(self):
        return int(np.prod([t + 1 for t in self.two_I])) if self.two_I else 1

    @property
    def dim(self):
        return 4 * self.Z


@dataclass
class Workload:
    name: str
    systems: List[SpinSystem]
    fields_mT: np.ndarray          # [n_sys][nB]
    M: int
    seed: int
    notes: str = ""
    extra: dict = field(default_factory=dict)


def tiny_c1():
    """Two spin-1/2 nuclei (0.8, 0.3 mT) on radical 1, one (0.5 mT) on radical 2; Z=8."""
    s = SpinSystem(2, 1, [1, 1, 1], [0.8, 0.3, 0.5], 0.0, 1.0, 1.0, 10.0, name="c1_tiny_Z8")
    return Workload("c1_tiny_Z8", [s], np.linspace(0.0, 5.0, 16)[None, :], M=64, seed=1001)


def sweep_c2(n_fields=64, M=200):
    """7+7 spin-1/2 nuclei, a ~ U(-1,1) mT, kS=2, kT=0.5 /us, T=20 us; Z=2^14."""
    rng = np.random.default_rng(1002)
    a = rng.uniform(-1.0, 1.0, 14)
    s = SpinSystem(7, 7, [1] * 14, list(a), 0.0, 2.0, 0.5, 20.0, name="c2_7+7_Z16384")
    return Workload("c2_7+7_Z16384", [s], np.linspace(0.0, 10.0, n_fields)[None, :], M=M, seed=1002)


def batched_c3(n_sys=256, n_fields=32, M=64):
    """Uneven systems: N ~ U{8..18} spin-1/2, N1 = ceil(N/2), a ~ N(0, 0.7) mT,
    kS, kT log-uniform on [0.1, 5] /us, T = min(10/min(kS,kT), 20) us."""
    rng = np.random.default_rng(1003)
    systems = []
    for i in range(n_sys):
        N = int(rng.integers(8, 19))
        n1 = (N + 1) // 2
        a = rng.normal(0.0, 0.7, N)
        kS, kT = np.exp(rng.uniform(np.log(0.1), np.log(5.0), 2))
        T = min(10.0 / min(kS, kT), 20.0)
        systems.append(SpinSystem(n1, N - n1, [1] * N, list(a), 0.0, float(kS), float(kT), float(T),
                                  name=f"c3_sys{i}_N{N}"))
    B = np.tile(np.linspace(0.0, 5.0, n_fields), (n_sys, 1))
    return Workload("c3_batched_256", systems, B, M=M, seed=1003)


def large_c4(n_fields=128, M=200):
    """Radical 1: 4 I=1 (a ~ U(0.2,0.6)) + 6 I=1/2 (a ~ U(-0.5,0.5)); radical 2: 2 I=1 + 6 I=1/2
    with the same laws; kS=kT=1 /us, T=10 us; Z = 3^6 * 2^12 = 2,985,984."""
    rng = np.random.default_rng(1004)
    a1 = list(rng.uniform(0.2, 0.6, 4)) + list(rng.uniform(-0.5, 0.5, 6))
    a2 = list(rng.uniform(0.2, 0.6, 2)) + list(rng.uniform(-0.5, 0.5, 6))
    two_I = [2] * 4 + [1] * 6 + [2] * 2 + [1] * 6
    s = SpinSystem(10, 8, two_I, a1 + a2, 0.0, 1.0, 1.0, 10.0, name="c4_large_Z2985984")
    return Workload("c4_large_Z2985984", [s], np.linspace(0.0, 5.0, n_fields)[None, :], M=M, seed=1004)


def cv_c5():
    """The first N=14 system of the batched set, for the learned control variate."""
    w = batched_c3()
    for i, s in enumerate(w.systems):
        if s.N == 14:
            return Workload("c5_cv_" + s.name, [s], w.fields_mT[i:i + 1], M=64, seed=1005,
                            extra={"n_train": 20000})
    raise RuntimeError("no N=14 system")


# Table I of the paper: a_1k/gamma and a_2k/gamma in mT for the model radical pair.
TABLE_I_A1 = [-0.999985, -0.736925, 0.511210, -0.0826998, 0.0655341,
              -0.562082, -0.905911, 0.357729, 0.358593, 0.869386]
TABLE_I_A2 = [-0.232996, 0.0388327, 0.661931, -0.930856, -0.893077,
              0.0594001, 0.342299, -0.984604, -0.233169, -0.866316]


def paper_model(n_fields=64, M=200):
    """Sec. IV model: 10+10 spin-1/2 (Table I), J/gamma=1.75 mT, kS/gamma=0.1 mT,
    kT/gamma=1.0 mT; Z = 2^20.  The horizon leaves e^-14 of the population."""
    kS, kT = 0.1 * GAMMA_E, 1.0 * GAMMA_E
    s = SpinSystem(10, 10, [1] * 20, TABLE_I_A1 + TABLE_I_A2, 1.75, kS, kT, 14.0 / kS,
                   name="paper_model_Z1048576")
    return Workload("paper_model_Z1048576", [s], np.linspace(0.0, 10.0, n_fields)[None, :], M=M,
                    seed=1000)


def max_state():
    """The largest state of the parity checks: 12+11 spin-1/2 (Z = 2^23, 8.4e6 nuclear states),
    a ~ U(-0.5, 0.5) mT, J = 0, kS = kT = 1.5 /us (so the oracle's per-radical route applies),
    T = 0.15 us (two Chebyshev steps at 2 mT)."""
    rng = np.random.default_rng(1023)
    a = rng.uniform(-0.5, 0.5, 23)
    s = SpinSystem(12, 11, [1] * 23, list(a), 0.0, 1.5, 1.5, 0.15, name="max_Z8388608")
    return Workload("max_Z8388608", [s], np.array([[2.0]]), M=1, seed=1023)


def one_nucleus(a_mT=0.5, k=1.0, T=10.0):
    """One spin-1/2 nucleus on radical 1 and none on radical 2 (closed-form case)."""
    return SpinSystem(1, 0, [1], [a_mT], 0.0, k, k, T, name="one_nucleus")
