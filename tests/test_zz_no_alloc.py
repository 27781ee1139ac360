"""rp_propagate_static (no device allocation; the library's static workspace area) against
rp_propagate, through the C ABI, on identical seeded inputs: two calls in a row, the second
smaller; the LDS-resident kernel and the tiled kernels; several systems of unequal size in one
call (the job queue); an input beyond the static area is refused with RP_ENOMEM."""
import sys

import numpy as np
import pytest

from oracle import philox
from paper_1612_09517_amd import rp, workloads
from paper_1612_09517_amd.workloads import SpinSystem

import gpu_common as gc

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rp.lib()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


TOL = {64: 1e-10, 32: 1e-5}


def _rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))


@pytest.mark.parametrize("prec", [64, 32])
def test_static_matches_allocating_entry_point(prec):
    rng = np.random.default_rng(70)
    big = [SpinSystem(6, 6, [1] * 12, list(rng.normal(0, 0.7, 12)), kS=1.2, kT=0.4, T_us=0.8),
           SpinSystem(5, 5, [1] * 9 + [2], list(rng.normal(0, 0.6, 10)), J_mT=0.2, kS=0.5, kT=1.5, T_us=0.6),
           SpinSystem(4, 4, [1] * 8, list(rng.normal(0, 0.7, 8)), kS=2.0, kT=0.5, T_us=1.0)]
    B = np.array([[0.0, 1.5, 4.0]] * len(big))
    M = 6
    angs = [rp.sample(s, 80 + i, M) for i, s in enumerate(big)]
    cat = torch.cat([a.reshape(-1) for a in angs])
    for tiled in (False, True):
        _say("static entry point, precision", prec, "tiled", tiled, "call 1: three systems, Z =", [s.Z for s in big])
        want = rp.propagate(big, B, cat, M, precision=prec, tiled=tiled).cpu().numpy()
        got = rp.propagate(big, B, cat, M, precision=prec, tiled=tiled, static=True).cpu().numpy()
        _say("  max relative difference", _rel(got, want))
        assert _rel(got, want) < TOL[prec]
        # second call, smaller: one system, fewer fields and samples (the area keeps the first
        # call's contents; everything that must start at zero is cleared by the call)
        s = big[2]
        _say("static entry point, call 2: one system, Z =", s.Z)
        ang = rp.sample(s, 90, 3)
        want2 = rp.propagate(s, B[2:, :2], ang, 3, precision=prec, tiled=tiled).cpu().numpy()
        got2 = rp.propagate(s, B[2:, :2], ang, 3, precision=prec, tiled=tiled, static=True).cpu().numpy()
        _say("  max relative difference", _rel(got2, want2))
        assert _rel(got2, want2) < TOL[prec]
        ref = gc.oracle_phi_sparse(s, B[2, :2], philox.sample_angles(90, 0, 3, s.N))
        assert np.max(np.abs(got2[0] - ref) / ref) < (1e-10 if prec == 64 else 1e-5)


def test_static_refuses_inputs_beyond_the_area():
    """The Sec. IV model (Z = 2^20): one complex-FP64 wavepacket needs three 64 MiB vectors and
    about 140 amplitude slabs of 16 MiB, beyond the static area: RP_ENOMEM, nothing launched."""
    w = workloads.paper_model()
    s = w.systems[0]
    ang = rp.sample(s, 1, 1)
    _say("static entry point, oversized input")
    with pytest.raises(rp.RpError) as ei:
        rp.propagate(s, np.array([[1.0]]), ang, 1, precision=64, static=True)
    assert ei.value.code == rp.RP_ENOMEM
