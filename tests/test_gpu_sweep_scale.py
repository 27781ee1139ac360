"""Parity at the full size of the sweep workload (7+7 spin-1/2, Z = 2^14, T = 20 us), in the
launch configuration the benchmark uses (all fields of a batch in one call).

Expected values: tests/golden/sweep_golden.json, written by tests/golden/make_sweep_golden.py
from the oracle's sparse augmented-system route (scipy expm_multiply, agreeing with the dense
route to ~1e-12 on small systems).  Tolerances: relative 1e-10 per yield for complex FP64
(measured agreement with every golden here: 1e-13 or better), 1e-5 for complex FP32."""
import json
import os
import sys

import numpy as np
import pytest

from paper_1612_09517_amd import rp, workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sweep_golden.json")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rp.lib()


def _run(prec, B, M, rdt=0.0):
    w = workloads.sweep_c2()
    s = w.systems[0]
    ang = rp.sample(s, w.seed, M)
    print("sweep scale: precision", prec, "fields", list(B), "samples", M, "rdt", rdt, flush=True)
    return rp.propagate(s, np.asarray(B)[None, :], ang, M, precision=prec, rdt=rdt).cpu().numpy()[0]


@pytest.mark.parametrize("rdt", [0.0, 150.0])
def test_full_size_against_oracle_golden(rdt):
    """At the default step (ranks 45-46 in complex FP32: three 16-column blocks of the
    matrix-core quadrature) and at r*dt = 150, the step the autotuner picks for this workload
    (ranks 61-63: four blocks; 80-87 in FP64: three passes of the vector kernel)."""
    g = json.load(open(GOLDEN))
    B = g["fields_mT"]
    M = max(g["samples"]) + 1
    for prec, tol in ((64, 1e-10), (32, 1e-5)):
        phi = _run(prec, B, M, rdt)
        for b, Bv in enumerate(B):
            for i in g["samples"]:
                want = g["phi"][f"{Bv}:{i}"]
                assert abs(phi[b, i] - want) < tol * want, (prec, Bv, i, phi[b, i], want)


def test_full_size_fp32_tracks_fp64():
    B = [0.0, 2.5, 10.0]
    p64 = _run(64, B, 8)
    p32 = _run(32, B, 8)
    assert np.max(np.abs(p32 - p64) / p64) < 1e-5
    assert np.all((p64 > 0) & (p64 < 1))


def test_streaming_hints_leave_results_unchanged():
    """A chunk whose three wavepacket buffers exceed the 256 MB Infinity Cache is propagated with
    non-temporal loads and stores of phi_{n-1}, phi_{n+1} and the accumulator; a smaller
    workspace (fewer jobs per launch) takes the cached path.  Both give bit-identical yields,
    which agree with the sparse oracle (9+9 spin-1/2, Z = 2^18, one short step)."""
    import gpu_common as gc
    from oracle import philox
    a = list(np.random.default_rng(18).normal(0.0, 0.7, 18))
    s = workloads.SpinSystem(9, 9, [1] * 18, a, 0.0, 2.0, 0.5, 0.02)
    B = np.array([[0.5, 3.0, 6.0]])
    M = 4
    ang = rp.sample(s, 77, M)
    want = gc.oracle_phi_sparse(s, [0.5], philox.sample_angles(77, 0, 1, 18))[0, 0]
    for prec, tol in ((32, 1e-5), (64, 1e-10)):
        cb = 8 * (prec // 32)
        vec = 4 * s.Z * cb
        nt = max(rp.plan_field(s, float(b), precision=prec)["n_terms"] for b in B[0])
        per_job = 3 * vec + nt * s.Z * cb + (s.Z // 256) * 24 + 32
        assert 3 * B.shape[1] * M * vec > 256 << 20          # default chunk streams
        print("streaming: precision", prec, "n_terms", nt, flush=True)
        big = rp.propagate(s, B, ang, M, precision=prec).cpu().numpy()
        small = rp.propagate(s, B, ang, M, precision=prec, workspace_bytes=int(2.5 * per_job)).cpu().numpy()
        assert np.array_equal(big, small)
        assert abs(big[0, 0, 0] - want) < tol * want, (prec, big[0, 0, 0], want)


@pytest.mark.parametrize("name", ["paper", "large", "large_full"])
def test_full_size_short_horizon_against_oracle_golden(name):
    """The two largest states at their full size (the Sec. IV model, Z = 2^20, and the spin-1
    workload, Z = 2,985,984) on a horizon shortened to a few Chebyshev steps -- and the spin-1
    workload on its own horizon, T = 10 us -- against yields the oracle computed one by one
    (tests/golden/make_paper_golden.py, make_large_golden.py [--full])."""
    import dataclasses
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", f"{name}_golden.json")))
    w = workloads.paper_model() if name == "paper" else workloads.large_c4()
    s = dataclasses.replace(w.systems[0], T_us=g["T_us"])
    B = np.asarray(g["fields_mT"])[None, :]
    M = max(g["samples"]) + 1
    ang = rp.sample(s, w.seed, M)
    for prec, tol in ((64, 1e-10), (32, 1e-5)):
        print(f"{name} full size: precision {prec} fields {list(B[0])} samples {M}", flush=True)
        phi = rp.propagate(s, B, ang, M, precision=prec).cpu().numpy()[0]
        for b, Bv in enumerate(g["fields_mT"]):
            for i in g["samples"]:
                want = g["phi"][f"{Bv}:{i}"]
                assert abs(phi[b, i] - want) < tol * want, (name, prec, Bv, i, phi[b, i], want)


def test_batched_subset_against_oracle_golden():
    """A subset of the batched workload of 256 uneven systems: the first system of every size
    N = 8..18 (Z = 2^8 .. 2^18, one per size class), each with its own rates, horizon and
    fields, all in ONE call -- the LDS-resident launches for the small ones and one job queue
    of unequal Z for the tiled ones -- against yields the oracle computed one by one
    (tests/golden/make_batched_golden.py; systems beyond N = 12 on a horizon cut to 0.5 us)."""
    import dataclasses
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "batched_golden.json")))
    w = workloads.batched_c3()
    systems = [dataclasses.replace(w.systems[e["index"]], T_us=e["T_us"]) for e in g["systems"]]
    B = np.array([e["fields_mT"] for e in g["systems"]])
    M = max(g["samples"]) + 1
    ang = torch.cat([rp.sample(s, w.seed, M).reshape(-1) for s in systems])
    for prec, tol in ((64, 1e-10), (32, 1e-5)):
        print("batched subset: precision", prec, "Z =", [s.Z for s in systems], flush=True)
        phi = rp.propagate(systems, B, ang, M, precision=prec).cpu().numpy()
        worst = 0.0
        for i, e in enumerate(g["systems"]):
            for b, Bv in enumerate(e["fields_mT"]):
                for j in g["samples"]:
                    want = g["phi"][f"{e['index']}:{Bv}:{j}"]
                    worst = max(worst, abs(phi[i, b, j] - want) / want)
                    assert abs(phi[i, b, j] - want) < tol * want, (prec, e["N"], Bv, j, phi[i, b, j], want)
        print("  max relative error", worst, flush=True)


def test_maximum_state_against_oracle_golden():
    """The largest state of the checks, Z = 2^23 (12+11 spin-1/2; 256 MB per complex-FP32
    wavepacket, 32,768 workgroups per launch), against the oracle's per-radical route
    (tests/golden/make_large_golden.py --max)."""
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "max_golden.json")))
    w = workloads.max_state()
    s = w.systems[0]
    assert s.T_us == g["T_us"]
    ang = rp.sample(s, w.seed, 1)
    want = g["phi"][f"{g['fields_mT'][0]}:0"]
    for prec, tol in ((64, 1e-10), (32, 1e-5)):
        print("maximum state: precision", prec, flush=True)
        phi = rp.propagate(s, w.fields_mT, ang, 1, precision=prec).cpu().numpy()[0, 0, 0]
        assert abs(phi - want) < tol * want, (prec, phi, want)


def test_zero_couplings_large_mixed_radix_closed_form():
    """Degenerate case at a large size: with every a_k = 0 the singlet is an eigenstate of
    omega (S1z + S2z) + 2J S1.S2 and of P_S, so phi_S = 1 - exp(-kS T) for every sample,
    whatever the nuclei (8 spin-1/2 + 10 spin-1 nuclei, Z = 15,116,544; partners along all 18
    axes are read with zero coefficients)."""
    s = workloads.SpinSystem(9, 9, [1] * 8 + [2] * 10, [0.0] * 18, 0.6, 2.5, 0.4, 0.3)
    ang = rp.sample(s, 3, 1)
    want = 1.0 - np.exp(-2.5 * 0.3)
    for prec, tol in ((64, 1e-12), (32, 1e-6)):
        print("zero couplings: precision", prec, flush=True)
        phi = rp.propagate(s, np.array([[0.7, 3.0]]), ang, 1, precision=prec).cpu().numpy()[0]
        assert np.max(np.abs(phi - want)) < tol, (prec, phi, want)


def test_paper_model_full_horizon_fp32_tracks_fp64():
    """The Sec. IV model on its own horizon (T = 14/kS, strong triplet dissipation): complex
    FP32 with its default growth bound tracks FP64 per yield, and the yield dips near
    omega = 2J (Sec. IV) for these samples."""
    w = workloads.paper_model()
    s = w.systems[0]
    B = np.array([[0.0, 3.5, 9.0]])
    ang = rp.sample(s, w.seed, 2)
    print("paper model full horizon", flush=True)
    p64 = rp.propagate(s, B, ang, 2, precision=64).cpu().numpy()[0]
    p32 = rp.propagate(s, B, ang, 2, precision=32).cpu().numpy()[0]
    assert np.max(np.abs(p32 - p64) / p64) < 1e-5
    assert np.all((p64 > 0) & (p64 < 1))
    m = p64.mean(axis=1)
    assert m[1] < m[0] and m[1] < m[2]
