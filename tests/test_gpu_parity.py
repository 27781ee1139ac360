"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, element by element
on identical seeded inputs.  Tolerances: relative 1e-10 per yield for complex-FP64
wavepackets, 1e-5 for complex-FP32 wavepackets with FP64 reductions."""
import math
import sys

import numpy as np
import pytest

from oracle import coherent, philox, stats, yields
from paper_1612_09517_amd import rp, workloads
from paper_1612_09517_amd.workloads import SpinSystem

import gpu_common as gc

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = {64: 1e-10, 32: 1e-5}


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rp.lib()   # raises if the library is missing


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(got, want):
    return np.max(np.abs(got - want) / np.maximum(np.abs(want), 1e-300))


# --------------------------------------------------------------------------- sampler
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_sampler_bit_exact(mode):
    s = SpinSystem(3, 2, [1, 2, 1, 4, 1], [0.1] * 5)
    _say("sampler mode", mode)
    got = rp.sample(s, seed=1234, M=37, first=5, stream_id=2, basis_mode=mode).cpu().numpy()
    if mode == 0:
        want = philox.sample_angles(1234, 5, 37, 5, stream=2)
    elif mode == 1:
        want = philox.sample_basis_digits(1234, 5, 37, s.two_I, stream=2)
    else:
        want = philox.enumerate_basis_digits(5, 37, s.two_I)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("mode", [3, 4, 5])
def test_design_sampler_bit_exact(mode):
    """Sign-flip designs: groups of rp_design_size samples share one draw; a ragged first
    sample and count; five nuclei use Hadamard columns 0..4 of order 8 (16 rows) or columns
    1..5 of order 8 (8 rows)."""
    s = SpinSystem(3, 2, [1, 2, 1, 4, 1], [0.1] * 5)
    _say("design sampler mode", mode)
    R = rp.design_size(s.N, mode)
    assert R == {3: 2, 4: 16, 5: 8}[mode]
    got = rp.sample(s, seed=99, M=45, first=7, stream_id=1, basis_mode=mode).cpu().numpy()
    want = philox.sample_design(99, 7, 45, s.N, mode, stream=1)
    assert np.array_equal(got, want)
    # the Sec. IV model's 20 nuclei: Hadamard order 32 (64 rows for mode 4), a ragged window
    # spanning three groups
    p = workloads.paper_model().systems[0]
    R20 = rp.design_size(p.N, mode)
    assert R20 == {3: 2, 4: 64, 5: 32}[mode]
    got = rp.sample(p, seed=5, M=2 * R20 + 3, first=R20 - 2, basis_mode=mode).cpu().numpy()
    assert np.array_equal(got, philox.sample_design(5, R20 - 2, 2 * R20 + 3, p.N, mode))


def test_design_group_means_recover_trace():
    """Three spin-1/2 nuclei: every group of the strength-3 design (8 samples) averages to the
    Eq. 14 trace exactly (phi_S multilinear in the Bloch vectors), so the design estimate
    has zero spread; rp_group_mean against a plain mean; the antithetic pair keeps spread;
    two nuclei in the strength-2 design (4 samples per group) also give the trace."""
    s = SpinSystem(2, 1, [1, 1, 1], [0.8, -0.3, 0.5], J_mT=0.4, kS=2.0, kT=0.5, T_us=5.0)
    B = np.array([[1.2, 3.0]])
    _say("design group means")
    R = rp.design_size(s.N, 4)
    ang = rp.sample(s, 13, 4 * R, basis_mode=4)
    phi = rp.propagate(s, B, ang, 4 * R, precision=64)[0]
    gm = rp.group_mean(phi, R)
    ref = phi.cpu().numpy().reshape(2, 4, R).mean(axis=2)
    assert gm.shape == (2, 4) and np.max(np.abs(gm.cpu().numpy() - ref)) < 1e-15
    mean, err = rp.yield_stats(gm)
    for b, Bv in enumerate(B[0]):
        tr = gc.oracle_trace(s, Bv)
        assert np.max(np.abs(gm.cpu().numpy()[b] - tr)) < 1e-10
        assert abs(mean.cpu().numpy()[b] - tr) < 1e-10 and err.cpu().numpy()[b] < 1e-10
    pair = rp.propagate(s, B, rp.sample(s, 13, 8, basis_mode=3), 8, precision=64)[0]
    _, perr = rp.yield_stats(rp.group_mean(pair, 2))
    assert np.all(perr.cpu().numpy() > 1e-6)
    s2 = SpinSystem(1, 1, [1, 1], [0.7, -0.45], J_mT=-0.2, kS=0.9, kT=1.7, T_us=4.0)
    R2 = rp.design_size(s2.N, 5)
    gm2 = rp.group_mean(rp.propagate(s2, B, rp.sample(s2, 17, 3 * R2, basis_mode=5), 3 * R2, precision=64)[0], R2)
    for b, Bv in enumerate(B[0]):
        assert np.max(np.abs(gm2.cpu().numpy()[b] - gc.oracle_trace(s2, Bv))) < 1e-10


# --------------------------------------------------------------------------- tiny workload (Z = 8)
@pytest.mark.parametrize("tiled", [False, True])
@pytest.mark.parametrize("prec", [64, 32])
def test_tiny_workload_parity(prec, tiled):
    """Both paths: LDS-resident (default for small systems) and the tiled kernels."""
    w = workloads.tiny_c1()
    s = w.systems[0]
    _say("tiny workload parity, precision", prec, "tiled", tiled)
    ang = rp.sample(s, w.seed, w.M)
    phi = rp.propagate(s, w.fields_mT, ang, w.M, precision=prec, tiled=tiled).cpu().numpy()[0]
    want = gc.oracle_phi(s, w.fields_mT[0], philox.sample_angles(w.seed, 0, w.M, s.N))
    assert _rel(phi, want) < TOL[prec]


@pytest.mark.parametrize("tiled", [False, True])
@pytest.mark.parametrize("prec", [64, 32])
def test_general_spins_exchange_triplet_dissipation(prec, tiled):
    """Spin-1 nucleus (mixed radix), J != 0 and kT > kS (P_T is the dissipative projector)."""
    s = SpinSystem(2, 1, [1, 2, 1], [0.8, -0.3, 0.5], J_mT=0.4, kS=0.5, kT=2.0, T_us=3.0)
    B = np.array([[0.0, 1.7, 4.0]])
    _say("general spins, precision", prec, "tiled", tiled)
    ang = rp.sample(s, 77, 8)
    phi = rp.propagate(s, B, ang, 8, precision=prec, tiled=tiled).cpu().numpy()[0]
    want = gc.oracle_phi(s, B[0], philox.sample_angles(77, 0, 8, 3))
    assert _rel(phi, want) < TOL[prec]


@pytest.mark.parametrize("rdt", [250.0, 400.0])
@pytest.mark.parametrize("prec", [64, 32])
def test_long_steps_several_quadrature_passes(prec, rdt):
    """Long Chebyshev steps: ranks of 86-183 need two to four quadrature passes; in complex FP32
    the matrix-core kernel runs them at r*dt = 250 (275 terms), and the factor of r*dt = 400
    (422 terms) no longer fits its LDS, so the vector kernel takes over."""
    s = SpinSystem(3, 2, [1, 2, 1, 1, 1], [0.8, -0.3, 0.5, 0.6, -0.7], J_mT=0.4, kS=0.5, kT=2.0, T_us=3.0)
    B = np.array([[0.0, 2.0, 5.0]])
    _say("long steps, precision", prec, "rdt", rdt)
    ang = rp.sample(s, 21, 4)
    phi = rp.propagate(s, B, ang, 4, precision=prec, tiled=True, rdt=rdt).cpu().numpy()[0]
    want = gc.oracle_phi(s, B[0], philox.sample_angles(21, 0, 4, s.N))
    assert _rel(phi, want) < TOL[prec]


@pytest.mark.parametrize("prec", [64, 32])
def test_singlet_population_trajectory(prec):
    """ps_t: <psi(t)|P_S|psi(t)> at every step start t_j = j dt of each system and field (dt and
    n_steps from the planner), against the oracle's propagator, NaN past the last step; two
    systems of different horizons in one call; the yields equal those of a call without it;
    a workspace of a few wavepackets (several chunks) gives the same trajectories."""
    s1 = SpinSystem(2, 1, [1, 2, 1], [0.8, -0.3, 0.5], J_mT=0.4, kS=0.5, kT=2.0, T_us=3.0)
    s2 = SpinSystem(1, 1, [1, 1], [0.6, -0.9], J_mT=-0.2, kS=1.5, kT=0.3, T_us=1.2)
    B = np.array([[0.0, 1.7, 4.0], [0.3, 2.2, 6.0]])
    M = 3
    _say("trajectory, precision", prec)
    plans = [[rp.plan_field(s, b, precision=prec) for b in row] for s, row in zip((s1, s2), B)]
    L = max(p["n_steps"] for row in plans for p in row) + 2
    ang = torch.cat([rp.sample(s1, 61, M).reshape(-1), rp.sample(s2, 62, M).reshape(-1)])
    phi, ps = rp.propagate([s1, s2], B, ang, M, precision=prec, ps_t_len=L)
    ref = rp.propagate([s1, s2], B, ang, M, precision=prec, tiled=True)
    assert torch.equal(phi, ref)
    # several chunks per system (the workspace holds a few wavepackets): same trajectories
    phi_c, ps_c = rp.propagate([s1, s2], B, ang, M, precision=prec, ps_t_len=L, workspace_bytes=80000)
    ps = ps.cpu().numpy()
    assert torch.equal(phi_c, phi) and np.array_equal(ps_c.cpu().numpy(), ps, equal_nan=True)
    tol = 1e-11 if prec == 64 else 2e-6
    for i, (s, seed) in enumerate(((s1, 61), (s2, 62))):
        d = gc.dense(s)
        angs = philox.sample_angles(seed, 0, M, s.N)
        for b, Bv in enumerate(B[i]):
            fo = yields.FieldOracle(d, Bv, s.T_us)
            n, dt = plans[i][b]["n_steps"], plans[i][b]["dt"]
            assert np.all(np.isnan(ps[i, b, :, n:]))
            for m in range(M):
                psi0 = coherent.initial_wavepacket(d, angs[m])
                for j in sorted({0, 1, n // 2, n - 1}):
                    assert abs(ps[i, b, m, j] - fo.singlet_probability(psi0, j * dt)) < tol
            assert np.all(np.abs(ps[i, b, :, 0] - 1.0) < tol)     # P_S(0) = 1 for |S> (Eq. 10)


def test_deterministic_trace_by_enumeration():
    """Basis states |S, M> (init_mode 1) over all Z give the Eq. 14 trace."""
    w = workloads.tiny_c1()
    s = w.systems[0]
    B = np.array([[0.0, 1.0, 5.0]])
    _say("enumerated trace")
    dig = rp.sample(s, 0, s.Z, basis_mode=2)
    phi = rp.propagate(s, B, dig, s.Z, init_mode=1).cpu().numpy()[0]
    want = gc.oracle_phi(s, B[0], philox.enumerate_basis_digits(0, s.Z, s.two_I), basis=True)
    assert _rel(phi, want) < 1e-10
    for b, Bv in enumerate(B[0]):
        assert abs(phi[b].mean() - gc.oracle_trace(s, Bv)) < 1e-10


@pytest.mark.parametrize("prec", [64, 32])
def test_monte_carlo_within_3_sigma_of_trace(prec):
    """Stochastic against deterministic trace (Eq. 18 against Eq. 14) with the exact sigma: the
    tiny workload's plain Monte Carlo mean (M = 64 seeded samples, all 16 fields, rp_yield on
    the GPU) lies within 3 sigma / sqrt(M) of the oracle trace at every field, where sigma is
    the exact single-sample deviation from the oracle's coherent-state second moment; the
    GPU's estimated error agrees with sigma / sqrt(M) within the chi-square spread; and at
    1 mT a long run (M = 8192) is within 3 sigma / sqrt(M) with its sample deviation within 5 %
    of the exact 9.7054e-3."""
    w = workloads.tiny_c1()
    s = w.systems[0]
    d = gc.dense(s)
    _say("Monte Carlo against the trace, 3 sigma exact, precision", prec)
    ang = rp.sample(s, w.seed, w.M)
    phi = rp.propagate(s, w.fields_mT, ang, w.M, precision=prec)[0]
    mean, err = (x.cpu().numpy() for x in rp.yield_stats(phi))
    for b, Bv in enumerate(w.fields_mT[0]):
        fo = yields.FieldOracle(d, Bv, s.T_us)
        tr, sig = fo.trace_yield(), fo.sample_sigma()
        assert abs(mean[b] - tr) < 3 * sig / math.sqrt(w.M), (Bv, mean[b], tr, sig)
        assert abs(err[b] * math.sqrt(w.M) / sig - 1) < 4 / math.sqrt(2 * (w.M - 1)), (Bv, err[b], sig)
    M = 8192
    ang = rp.sample(s, w.seed, M, first=10 ** 5)
    phi = rp.propagate(s, np.array([[1.0]]), ang, M, precision=prec)[0]
    mean, err = (x.cpu().numpy()[0] for x in rp.yield_stats(phi))
    fo = yields.FieldOracle(d, 1.0, s.T_us)
    sig = fo.sample_sigma()
    assert abs(sig - 9.7054e-3) < 5e-8
    assert abs(mean - fo.trace_yield()) < 3 * sig / math.sqrt(M)
    assert abs(err * math.sqrt(M) / sig - 1) < 0.05


def test_no_nuclei_closed_form():
    s = SpinSystem(0, 0, [], [], J_mT=0.9, kS=1.3, kT=0.2, T_us=2.5)
    _say("no nuclei")
    phi = rp.propagate(s, np.array([[0.0, 3.0]]), None, 4).cpu().numpy()[0]
    assert np.max(np.abs(phi - (1 - math.exp(-1.3 * 2.5)))) < 1e-12


# --------------------------------------------------------------------------- several tiles, ragged tail
def test_multi_block_ragged_mixed_radix():
    """Z = 2^9 * 3 = 1536 nuclear states: six 256-thread tiles per wavepacket, spin-1 slowest."""
    rng = np.random.default_rng(5)
    a = list(rng.uniform(-0.4, 0.4, 10))
    s = SpinSystem(5, 5, [1] * 9 + [2], a, J_mT=0.2, kS=1.5, kT=0.5, T_us=0.6)
    B = np.array([[0.0, 2.0]])
    _say("multi-block ragged, Z =", s.Z)
    ang = rp.sample(s, 9, 3)
    want = gc.oracle_phi_sparse(s, B[0], philox.sample_angles(9, 0, 3, s.N))
    for prec in (64, 32):
        phi = rp.propagate(s, B, ang, 3, precision=prec).cpu().numpy()[0]
        assert _rel(phi, want) < TOL[prec], _rel(phi, want)


def test_reordered_axes_spin1_first():
    """Spin-1 nuclei first in the caller's order (one per radical): the library reorders the
    axes internally (spin-1/2 first) for the tiled kernel; Z = 9 * 2^8 = 2304."""
    rng = np.random.default_rng(6)
    a = list(rng.uniform(-0.4, 0.4, 10))
    s = SpinSystem(5, 5, [2, 1, 1, 1, 1, 2, 1, 1, 1, 1], a, J_mT=-0.2, kS=0.6, kT=1.4, T_us=0.5)
    B = np.array([[0.5, 3.0]])
    _say("reordered axes, Z =", s.Z)
    ang = rp.sample(s, 12, 3)
    want = gc.oracle_phi_sparse(s, B[0], philox.sample_angles(12, 0, 3, s.N))
    for prec in (64, 32):
        phi = rp.propagate(s, B, ang, 3, precision=prec).cpu().numpy()[0]
        assert _rel(phi, want) < TOL[prec], _rel(phi, want)
        # the other axis order (spin-1 nuclei on the fastest axes, mixed-radix kernel)
        high = rp.propagate(s, B, ang, 3, precision=prec, axes_high_first=True).cpu().numpy()[0]
        assert _rel(high, want) < TOL[prec], _rel(high, want)


def test_pair_term_kernel_matches_scalar_term_kernel():
    """Complex FP32 terms on index pairs (16-byte accesses; the default with 8 or more leading
    spin-1/2 nuclei) against one index per thread (RP_FLAG_TERM_SCALAR): the same sums in the
    same order, except that the compiler may fuse a product and a sum into one FMA in one
    kernel and not in the other, so they agree to a few FP32 roundings per step (relative
    2e-6, against the 1e-5 FP32 parity bound).  Exchange, unequal rates, radicals interleaved,
    spin-1 nuclei above the spin-1/2 axes, several tiles per wavepacket."""
    rng = np.random.default_rng(43)
    B = np.array([[0.0, 0.8, 2.6]])
    for n1, two_I in ((5, [1] * 10), (6, [1] * 8 + [2, 2]), (7, [1] * 13 + [2])):
        a = list(rng.uniform(-0.5, 0.5, len(two_I)))
        s = SpinSystem(n1, len(two_I) - n1, two_I, a, J_mT=0.15, kS=1.3, kT=0.45, T_us=0.6)
        _say("pair term kernel, Z =", s.Z)
        ang = rp.sample(s, 51, 3)
        pair = rp.propagate(s, B, ang, 3, precision=32, tiled=True).cpu().numpy()
        scal = rp.propagate(s, B, ang, 3, precision=32, tiled=True, term_scalar=True).cpu().numpy()
        assert _rel(pair, scal) < 2e-6 and np.all(pair > 0)


# --------------------------------------------------------------------------- batching and chunking
def test_multi_system_call_and_chunking_are_consistent():
    w = workloads.tiny_c1()
    s1 = w.systems[0]
    s2 = SpinSystem(1, 2, [2, 1, 1], [0.6, 0.2, -0.7], kS=2.0, kT=0.7, T_us=4.0)
    B = np.array([[0.0, 2.0, 4.5], [1.0, 0.5, 3.0]])
    _say("multi-system")
    a1, a2 = rp.sample(s1, 3, 6), rp.sample(s2, 4, 6)
    both = rp.propagate([s1, s2], B, torch.cat([a1.reshape(-1), a2.reshape(-1)]), 6).cpu().numpy()
    one = rp.propagate(s1, B[:1], a1, 6).cpu().numpy()[0]
    two = rp.propagate(s2, B[1:], a2, 6).cpu().numpy()[0]
    assert np.array_equal(both[0], one) and np.array_equal(both[1], two)
    small = rp.propagate(s2, B[1:], a2, 6, workspace_bytes=3 * 2 * 6000).cpu().numpy()[0]
    assert np.array_equal(small, two)
    again = rp.propagate(s2, B[1:], a2, 6).cpu().numpy()[0]
    assert np.array_equal(again, two)


def test_job_queue_of_unequal_tiled_systems():
    """Tiled systems of unequal Z in one call share the Chebyshev launches (job queue: per-tile
    job index, per-job offsets, per-system constants): the yields agree with one call per
    system (uniform launches) to the rounding of a possibly different FMA contraction, with the
    oracle for the smallest, and with a workspace small enough to cut the queue into chunks
    that mix systems differently."""
    rng = np.random.default_rng(31)
    systems = [SpinSystem(6, 5, [1] * 11, list(rng.normal(0, 0.7, 11)), kS=1.6, kT=2.9, T_us=0.4),
               SpinSystem(4, 4, [1] * 8, list(rng.normal(0, 0.7, 8)), kS=0.3, kT=0.2, T_us=0.9),
               SpinSystem(7, 6, [1] * 13, list(rng.normal(0, 0.7, 13)), J_mT=0.1, kS=0.5, kT=0.8, T_us=0.3),
               SpinSystem(5, 5, [1] * 10, list(rng.normal(0, 0.7, 10)), kS=2.0, kT=0.5, T_us=0.6)]
    B = np.array([[0.0, 2.0, 5.0]] * len(systems))
    M = 4
    angs = [rp.sample(s, 20 + i, M) for i, s in enumerate(systems)]
    cat = torch.cat([a.reshape(-1) for a in angs])
    for prec, tol in ((64, 1e-12), (32, 2e-6)):
        _say("job queue, precision", prec, "Z =", [s.Z for s in systems])
        both = rp.propagate(systems, B, cat, M, precision=prec, tiled=True).cpu().numpy()
        one = np.stack([rp.propagate(s, B[i:i + 1], angs[i], M, precision=prec, tiled=True).cpu().numpy()[0]
                        for i, s in enumerate(systems)])
        _say("  queue against one call per system:", _rel(both, one), "bit-identical:", np.array_equal(both, one))
        assert _rel(both, one) < tol
        ws = 3 * (12 + 160) * max(s.Z for s in systems) * (16 if prec == 64 else 8)   # about three of the largest
        small = rp.propagate(systems, B, cat, M, precision=prec, tiled=True, workspace_bytes=ws).cpu().numpy()
        assert _rel(small, both) < tol
        want = gc.oracle_phi_sparse(systems[1], B[1], philox.sample_angles(21, 0, M, systems[1].N))
        assert _rel(both[1], want) < TOL[prec]


# --------------------------------------------------------------------------- statistics and errors
def test_yield_statistics():
    rng = np.random.default_rng(2)
    phi = rng.uniform(0, 1, (5, 33))
    g = phi + rng.normal(0, 0.1, phi.shape)
    mu = rng.uniform(0, 1, 5)
    be = rng.uniform(0, 1, 5)
    T = lambda x: torch.tensor(x, dtype=torch.float64, device="cuda")
    m, e = rp.yield_stats(T(phi))
    wm, we = stats.mc_mean_error(phi)
    assert np.max(np.abs(m.cpu().numpy() - wm)) < 1e-14 and np.max(np.abs(e.cpu().numpy() - we)) < 1e-14
    m, e = rp.yield_stats(T(phi), T(g), T(mu), T(be))
    wm, we = stats.cv_mean_error(phi, g, mu, be)
    assert np.max(np.abs(m.cpu().numpy() - wm)) < 1e-14 and np.max(np.abs(e.cpu().numpy() - we)) < 1e-14
    me = rng.uniform(0, 0.01, 5)
    m, e = rp.yield_stats(T(phi), T(g), T(mu), T(be), T(me))
    wm, we = stats.cv_mean_error(phi, g, mu, be, me)
    assert np.max(np.abs(m.cpu().numpy() - wm)) < 1e-14 and np.max(np.abs(e.cpu().numpy() - we)) < 1e-14


@pytest.mark.parametrize("tiled", [False, True])
def test_underestimated_spectrum_is_reported(tiled):
    w = workloads.tiny_c1()
    s = w.systems[0]
    _say("notconv, tiled", tiled)
    ang = rp.sample(s, 1, 2)
    with pytest.raises(rp.RpError) as ei:
        rp.propagate(s, np.array([[4.0]]), ang, 2, r_scale=0.3, tiled=tiled)
    assert ei.value.code == rp.RP_ENOTCONV


def test_resident_batch_of_unequal_systems():
    """Systems of 8, 64, 256 and 1024 nuclear states (spin-1/2 and spin-1 mixes) in one call:
    the LDS-resident launches agree with the tiled kernels and with the oracle (dense route for
    the two small systems; sparse augmented-system route, on the first three samples, for the
    256- and 1024-state ones, which run in the largest resident class: 1024-thread workgroups)."""
    rng = np.random.default_rng(11)
    systems = [SpinSystem(2, 1, [1, 1, 1], [0.8, 0.3, 0.5], kS=1.0, kT=1.0, T_us=4.0),
               SpinSystem(3, 2, [1, 2, 1, 2, 1], list(rng.uniform(-0.8, 0.8, 5)), J_mT=0.3, kS=0.4, kT=2.2, T_us=3.0),
               SpinSystem(4, 4, [1] * 8, list(rng.normal(0, 0.7, 8)), kS=2.0, kT=0.5, T_us=3.0),
               SpinSystem(5, 5, [1] * 10, list(rng.normal(0, 0.7, 10)), kS=0.3, kT=1.1, T_us=2.0)]
    B = np.array([[0.0, 1.0, 3.0]] * 4)
    M = 5
    angs = [rp.sample(s, 40 + i, M) for i, s in enumerate(systems)]
    cat = torch.cat([a.reshape(-1) for a in angs])
    oracle_large = {}
    for prec in (32, 64):
        _say("resident batch, precision", prec)
        res = rp.propagate(systems, B, cat, M, precision=prec).cpu().numpy()
        til = rp.propagate(systems, B, cat, M, precision=prec, tiled=True).cpu().numpy()
        assert np.max(np.abs(res - til) / til) < (1e-11 if prec == 64 else 2e-5)
        for i in (0, 1):
            want = gc.oracle_phi(systems[i], B[i], philox.sample_angles(40 + i, 0, M, systems[i].N))
            assert _rel(res[i], want) < TOL[prec]
        for i in (2, 3):
            want = oracle_large[i] if i in oracle_large else oracle_large.setdefault(
                i, gc.oracle_phi_sparse(systems[i], B[i], philox.sample_angles(40 + i, 0, 3, systems[i].N)))
            assert _rel(res[i][:, :3], want) < TOL[prec], (i, prec)


def test_autotuner_picks_valid_parameters_and_caches(tmp_path):
    from paper_1612_09517_amd import autotune
    s = SpinSystem(5, 5, [1] * 10, list(np.random.default_rng(3).normal(0, 0.6, 10)), kS=1.5, kT=0.5, T_us=2.0)
    B = np.linspace(0.0, 4.0, 6)
    cache = str(tmp_path / "tune.json")
    _say("autotune")
    best = autotune.tune(s, B, precision=32, samples=4, cache=cache)
    assert best["rdt"] in autotune.RDT and best["xcd"] in autotune.XCD
    assert set(best) == {"rdt", "xcd", "term_scalar", "tiled"}             # Z = 1024: resident or tiled
    assert autotune.tune(s, B, precision=32, cache=cache) == best          # served from the cache
    ang = rp.sample(s, 5, 4)
    a = rp.propagate(s, B[None, :], ang, 4, precision=32, **best).cpu().numpy()
    b = rp.propagate(s, B[None, :], ang, 4, precision=64).cpu().numpy()
    assert np.max(np.abs(a - b) / b) < 1e-5


def test_graph_replay_matches_direct_launches():
    """Captured step graphs (default) and direct launches give bit-identical yields, on the
    default stream and on a stream of the caller's, over chunks and fields that finish early."""
    s = SpinSystem(5, 5, [1] * 10, list(np.random.default_rng(8).normal(0, 0.6, 10)), kS=2.0, kT=0.5, T_us=1.5)
    B = np.array([[0.0, 1.0, 3.0, 6.0]])
    ang = rp.sample(s, 21, 6)
    _say("graph replay")
    for prec in (32, 64):
        direct = rp.propagate(s, B, ang, 6, precision=prec, tiled=True, graph=False).cpu().numpy()
        graph = rp.propagate(s, B, ang, 6, precision=prec, tiled=True).cpu().numpy()
        assert np.array_equal(direct, graph)
        small = rp.propagate(s, B, ang, 6, precision=prec, tiled=True, workspace_bytes=6 * 10 ** 6).cpu().numpy()
        assert np.array_equal(direct, small)
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            again = rp.propagate(s, B, ang, 6, precision=prec, tiled=True)
        side.synchronize()
        assert np.array_equal(direct, again.cpu().numpy())


# --------------------------------------------------------------------------- edge cases
def test_empty_inputs_are_no_ops():
    s = workloads.tiny_c1().systems[0]
    ang = rp.sample(s, 1, 0)
    assert ang.shape == (0, 3, 2)
    out = rp.propagate(s, np.zeros((1, 0)), ang, 0)
    assert out.numel() == 0
    out = rp.propagate(s, np.array([[1.0]]), rp.sample(s, 1, 2), 2)   # one field
    assert out.shape == (1, 1, 2)


def test_negative_fields_and_single_step():
    """A negative field reverses the Zeeman term (single-wavepacket yields differ from those at
    +B; only the ensemble yield is even in B) and matches the oracle sample by sample; a
    horizon of one short step does too."""
    s = SpinSystem(2, 1, [1, 2, 1], [0.7, -0.4, 0.3], J_mT=0.3, kS=1.2, kT=0.4, T_us=0.004)
    B = np.array([[-2.0, 2.0]])
    ang = rp.sample(s, 9, 4)
    phi = rp.propagate(s, B, ang, 4).cpu().numpy()[0]
    want = gc.oracle_phi(s, B[0], philox.sample_angles(9, 0, 4, 3))
    assert _rel(phi, want) < 1e-10
    assert rp.plan_field(s, 2.0)["n_steps"] == 1


def test_no_recombination_gives_zero_yield():
    s = SpinSystem(2, 1, [1, 1, 1], [0.8, 0.3, 0.5], kS=0.0, kT=0.0, T_us=2.0)
    phi = rp.propagate(s, np.array([[0.0, 1.0]]), rp.sample(s, 2, 3), 3).cpu().numpy()
    assert np.all(phi == 0.0)


def test_invalid_arguments_raise():
    s = workloads.tiny_c1().systems[0]
    ang = rp.sample(s, 1, 2)
    with pytest.raises(rp.RpError):
        rp.propagate(s, np.array([[np.nan]]), ang, 2)
    with pytest.raises(rp.RpError):
        rp.propagate(SpinSystem(1, 0, [1], [0.5], kS=1.0, kT=1.0, T_us=0.0), np.array([[1.0]]), ang[:, :1].contiguous(), 2)
    with pytest.raises(rp.RpError):
        rp.propagate(s, np.array([[1.0]]), ang, 2, precision=16)


@pytest.mark.parametrize("growth", [1e2, 0.0, 1e30])
def test_strong_dissipation_matches_oracle(growth):
    """|kS - kT| comparable to or larger than the spectral half-width r: the Chebyshev vectors
    can grow on the dissipative strip and the planner bounds the worst-case growth per step.
    At a strict bound and at the default, coherent-state and basis-state (Eq. 14) yields match
    the dense oracle; with no effective bound a call either still matches or reports
    RP_ENOTCONV (never a silently wrong yield)."""
    cases = [
        SpinSystem(1, 0, [1], [0.5], kS=1.0, kT=300.0, T_us=0.05),
        SpinSystem(2, 1, [1, 2, 1], [0.6, -0.3, 0.4], J_mT=0.5, kS=150.0, kT=2.0, T_us=0.08),
        SpinSystem(2, 2, [1, 1, 1, 1], [0.9, 0.2, -0.7, 0.3], kS=20.0, kT=400.0, T_us=0.03),
    ]
    for i, s in enumerate(cases):
        B = np.array([[0.0, 1.0, 6.0]])
        ang = rp.sample(s, 40 + i, 4)
        want = gc.oracle_phi(s, B[0], philox.sample_angles(40 + i, 0, 4, s.N))
        for prec, tol in ((64, 1e-10), (32, 1e-5)):
            for tiled in (False, True):
                _say(f"dissipative case {i} precision {prec} growth {growth} tiled {tiled}")
                try:
                    phi = rp.propagate(s, B, ang, 4, precision=prec, max_growth=growth, tiled=tiled).cpu().numpy()[0]
                except rp.RpError as e:
                    assert growth == 1e30 and e.code == -4, (i, prec, tiled, e)
                    continue
                assert _rel(phi, want) < tol, (i, prec, tiled, _rel(phi, want))
        dig = rp.sample(s, 0, s.Z, basis_mode=2)
        want_b = gc.oracle_phi(s, B[0], philox.enumerate_basis_digits(0, s.Z, s.two_I), basis=True)
        for prec, tol in ((64, 1e-10), (32, 1e-5)):
            _say(f"dissipative case {i} basis states precision {prec} growth {growth}")
            try:
                phi = rp.propagate(s, B, dig, s.Z, init_mode=1, precision=prec, max_growth=growth).cpu().numpy()[0]
            except rp.RpError as e:
                assert growth == 1e30 and e.code == -4, (i, prec, "basis", e)
                continue
            assert _rel(phi, want_b) < tol, (i, prec, "basis", _rel(phi, want_b))


# --------------------------------------------------------------------------- short-iterative Arnoldi
@pytest.mark.parametrize("krylov", [0, 8, 32])
def test_arnoldi_propagator_matches_oracle(krylov):
    """The paper's propagator (RP_FLAG_ARNOLDI): adaptive Krylov steps with the in-step yield
    from the projected singlet Gram matrix give the same per-sample yields as the oracle, for
    spin-1 with exchange, strong triplet dissipation and a state spanning two workgroups."""
    cases = [
        (SpinSystem(2, 1, [1, 2, 1], [0.6, -0.3, 0.4], J_mT=0.5, kS=1.2, kT=0.4, T_us=1.0), False),
        (SpinSystem(1, 0, [1], [0.5], kS=1.0, kT=300.0, T_us=0.05), False),
        (SpinSystem(5, 4, [1] * 9, list(np.random.default_rng(9).normal(0, 0.5, 9)), kS=2.0, kT=0.5, T_us=0.3), True),
    ]
    for i, (s, sparse) in enumerate(cases):
        B = np.array([[0.0, 2.0]])
        ang = rp.sample(s, 60 + i, 3)
        a_h = philox.sample_angles(60 + i, 0, 3, s.N)
        want = gc.oracle_phi_sparse(s, B[0], a_h) if sparse else gc.oracle_phi(s, B[0], a_h)
        for prec, tol in ((64, 1e-10), (32, 1e-5)):
            _say(f"arnoldi case {i} precision {prec} krylov {krylov}")
            phi = rp.propagate(s, B, ang, 3, precision=prec, arnoldi=True, krylov_dim=krylov).cpu().numpy()[0]
            _say("  max relative error", _rel(phi, want))
            assert _rel(phi, want) < tol, (i, prec, krylov, _rel(phi, want))


def test_arnoldi_invalid_krylov_dimension():
    s = workloads.tiny_c1().systems[0]
    ang = rp.sample(s, 1, 2)
    for m in (1, 33, -2):
        with pytest.raises(rp.RpError):
            rp.propagate(s, np.array([[1.0]]), ang, 2, arnoldi=True, krylov_dim=m)


def test_combine_matches_oracle():
    rng = np.random.default_rng(5)
    ma, mb = rng.uniform(0, 1, 37), rng.uniform(0, 1, 37)
    ea, eb = rng.uniform(1e-4, 1e-2, 37), rng.uniform(1e-4, 1e-2, 37)
    ea[3] = 0.0
    eb[7] = 0.0
    t = lambda x: torch.tensor(x, dtype=torch.float64, device="cuda")
    m, e = rp.combine(t(ma), t(ea), t(mb), t(eb))
    wm, we = stats.combine(ma, ea, mb, eb)
    assert np.max(np.abs(m.cpu().numpy() - wm)) < 1e-14 and np.max(np.abs(e.cpu().numpy() - we)) < 1e-14
