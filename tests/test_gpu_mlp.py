"""GPU checks of the control-variate network and estimator against the FP64 oracle.

Tolerances for the network: every hidden-layer product rounds its inputs to BF16
(relative rounding error <= 2^-9 per input).  Against the plain FP64 oracle, layer outputs
carry relative errors of a few 1e-3, so after three hidden layers the outputs are checked at
a relative L2 error of 3e-2 and the gradient at 5e-2.  With the same operand rounding modelled
in the test (the oracle's operand map), every output and every gradient element of every
parameter block agrees to 1e-5 of its own size plus its block's largest element (measured:
2e-7; what is left is FP32 accumulation order).  Elementwise FP32 steps (features, Adam) are
checked at 1e-6."""
import math
import sys

import numpy as np
import pytest

from oracle import coherent, mlp, philox, spin, stats, yields
from paper_1612_09517_amd import cv, rp
from paper_1612_09517_amd.workloads import SpinSystem

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


def _t(x, dt=torch.float32):
    return torch.tensor(np.asarray(x), dtype=dt, device="cuda")


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("layout", [0, 1, 2])
def test_features_match_oracle(layout):
    B = [0.0, 1.5, 4.0]
    ang = philox.sample_angles(5, 0, 37 * (3 if layout == 2 else 1), 6)
    x = rp.mlp_features(_t(ang, torch.float64), B, 19, layout=layout).cpu().numpy()
    if layout == 2:      # row r: direction r, field r % 3
        want = np.concatenate([mlp.features(ang[r:r + 1], [B[r % 3]]) for r in range(111)])
    else:
        want = mlp.features(ang, B)
        if layout == 1:
            want = want.reshape(3, 37, -1).transpose(1, 0, 2).reshape(111, -1)
    assert np.max(np.abs(x - want)) < 1e-6


def test_rotated_features_match_oracle():
    B = [0.0, 1.5, 4.0]
    ang = philox.sample_angles(6, 0, 41, 6)
    x = rp.mlp_features(_t(ang, torch.float64), B, 19, layout=0, rot_seed=987654321).cpu().numpy()
    assert np.max(np.abs(x - mlp.features(ang, B, rot_seed=987654321))) < 1e-6
    x0 = rp.mlp_features(_t(ang, torch.float64), B, 19, layout=0).cpu().numpy()
    assert np.max(np.abs(x - x0)) > 0.1          # the rotation did act


def _net(n_in=19, width=64, depth=3, seed=1):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(n_in, width, depth, rng)
    p += rng.normal(0, 0.02, len(p))
    return p


def test_forward_matches_fp64_oracle():
    n_in, width, depth = 19, 64, 3
    p = _net(n_in, width, depth)
    rng = np.random.default_rng(2)
    x = rng.normal(0, 1, (100, mlp.in_pad(n_in)))
    _say("mlp forward")
    y = rp.mlp_forward(_t(p), _t(x), n_in, width, depth).cpu().numpy()
    want, _ = mlp.forward(p.astype(np.float32).astype(float), x.astype(np.float32).astype(float), n_in, width, depth)
    assert _rel(y, want) < 3e-2


def test_gradient_and_adam_match_oracle():
    n_in, width, depth = 19, 64, 3
    p = _net(n_in, width, depth, seed=4)
    rng = np.random.default_rng(3)
    x = rng.normal(0, 1, (96, mlp.in_pad(n_in)))
    t = rng.normal(0, 1, 96)
    P, Mo, V = _t(p), torch.zeros(len(p), device="cuda"), torch.zeros(len(p), device="cuda")
    G = torch.empty(len(p), device="cuda")
    err = torch.empty(96, device="cuda")
    _say("mlp gradient")
    rp.mlp_train_step(P, Mo, V, 1, _t(x), _t(t), n_in, width, depth, lr=0.0, grad_out=G, sq_err=err)
    p32 = p.astype(np.float32).astype(float)
    loss, g = mlp.loss_and_grad(p32, x.astype(np.float32).astype(float), t, n_in, width, depth)
    assert _rel(G.cpu().numpy(), g) < 5e-2
    assert abs(err.cpu().numpy().mean() - loss) < 5e-2 * loss
    assert np.array_equal(P.cpu().numpy(), p.astype(np.float32))         # lr = 0 leaves parameters alone
    # one real Adam step: parameters follow the oracle's Adam applied to the GPU gradient
    rp.mlp_train_step(P, Mo, V, 1, _t(x), _t(t), n_in, width, depth, lr=1e-3, grad_out=G)
    gg = G.cpu().numpy().astype(float)
    want, _, _ = mlp.adam(p.astype(np.float32).astype(float), np.zeros(len(p)), np.zeros(len(p)), gg, 1, 1e-3)
    assert np.max(np.abs(P.cpu().numpy() - want)) < 1e-6


def _bf16(a):
    """Round to BF16 (nearest, ties to even) through FP32, as the device rounds MFMA operands."""
    u = np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32)).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _blocks(v, n_in, width, depth):
    """Packed parameter vector -> named blocks (W_l, b_l, w_out, b_out)."""
    layers, w, bo = mlp.unpack(v, n_in, width, depth)
    out = {}
    for l, (W, b) in enumerate(layers):
        out[f"W{l}"], out[f"b{l}"] = W, b
    out["w_out"], out["b_out"] = w, np.array([bo])
    return out


def test_forward_and_gradient_elementwise_with_bf16_operands():
    """Elementwise parity of the network with the FP64 oracle when the test rounds the operands
    of every hidden-layer product to BF16 as the device does (everything else FP64 in the
    oracle, FP32 on the device): outputs and every parameter block of the gradient (W_l, b_l,
    output weights and bias) separately, each element within 1e-5 of its own size plus its
    block's largest element.  A sign flip or a wrong block would fail by O(1)."""
    n_in, width, depth = 19, 64, 3
    p = _net(n_in, width, depth, seed=4).astype(np.float32).astype(float)
    rng = np.random.default_rng(3)
    x = rng.normal(0, 1, (96, mlp.in_pad(n_in))).astype(np.float32).astype(float)
    t = rng.normal(0, 1, 96).astype(np.float32).astype(float)
    _say("mlp elementwise with BF16 operands")
    y = rp.mlp_forward(_t(p), _t(x), n_in, width, depth).cpu().numpy()
    want_y, _ = mlp.forward(p, x, n_in, width, depth, q=_bf16)
    dev = np.abs(y - want_y) / (np.abs(want_y) + np.abs(want_y).max())
    _say("  forward: max scaled deviation", dev.max())
    assert dev.max() < 1e-5
    P, Mo, V = _t(p), torch.zeros(len(p), device="cuda"), torch.zeros(len(p), device="cuda")
    G = torch.empty(len(p), device="cuda")
    rp.mlp_train_step(P, Mo, V, 1, _t(x), _t(t), n_in, width, depth, lr=0.0, grad_out=G)
    _, g = mlp.loss_and_grad(p, x, t, n_in, width, depth, q=_bf16)
    got, want = _blocks(G.cpu().numpy(), n_in, width, depth), _blocks(g, n_in, width, depth)
    for name in want:
        a, b = got[name], want[name]
        dev = np.abs(a - b) / (np.abs(b) + np.abs(b).max())
        _say(f"  gradient block {name}: max scaled deviation {dev.max():.2e}")
        assert dev.max() < 1e-5, name


def test_target_standardisation_and_validation_loss():
    """rp_mlp_standardize against its definition (per-field mean and 1/n deviation over the
    first n_fit rows, applied to every row; a constant field divides by 1), and rp_mlp_loss
    against the mean of squared differences between the device forward pass and the targets."""
    rng = np.random.default_rng(12)
    nB, n_rows, n_fit = 5, 23, 17
    phi = rng.uniform(0.2, 0.8, (n_rows, nB))
    phi[:, 3] = 0.5                                    # constant field (exact mean, zero deviation)
    _say("target standardisation")
    t = rp.mlp_standardize(_t(phi.reshape(-1), torch.float64), nB, n_rows, n_fit).cpu().numpy().reshape(n_rows, nB)
    mean, sd = phi[:n_fit].mean(axis=0), phi[:n_fit].std(axis=0)
    sd[sd == 0] = 1.0
    assert np.max(np.abs(t - (phi - mean) / sd)) < 1e-6
    n_in, width, depth = 19, 64, 3
    p = _net(n_in, width, depth, seed=7)
    x = rng.normal(0, 1, (77, mlp.in_pad(n_in)))
    tg = rng.normal(0, 1, 77)
    mse = float(rp.mlp_loss(_t(p), _t(x), _t(tg), n_in, width, depth))
    y = rp.mlp_forward(_t(p), _t(x), n_in, width, depth).cpu().numpy().astype(float)
    assert abs(mse - np.mean((y - tg.astype(np.float32)) ** 2)) < 1e-6 * mse


def test_training_reduces_loss():
    n_in, width, depth = 7, 64, 2
    rng = np.random.default_rng(8)
    x = rng.normal(0, 1, (1024, 16))
    x[:, n_in:] = 0.0
    t = np.sin(x[:, 0]) * x[:, 1] + 0.3 * x[:, 2] ** 2
    p = mlp.init_params(n_in, width, depth, rng)
    P, Mo, V = _t(p), torch.zeros(len(p), device="cuda"), torch.zeros(len(p), device="cuda")
    X, T = _t(x), _t(t)
    err = torch.empty(256, device="cuda")
    _say("mlp training")
    first = None
    for step in range(1, 401):
        i = (step * 256) % 1024
        rp.mlp_train_step(P, Mo, V, step, X[i:i + 256], T[i:i + 256], n_in, width, depth, lr=3e-3, sq_err=err)
        if step == 1:
            first = float(err.mean())
    y = rp.mlp_forward(P, X, n_in, width, depth).cpu().numpy()
    assert np.mean((y - t) ** 2) < first / 10


def test_control_variate_is_unbiased_and_reduces_variance():
    """Trained on yields of stream 1, beta from held-out samples, mu from stream 2: the
    estimate on stream 0 agrees with the Eq. 14 trace within 4 standard errors and its
    standard error is well below the plain Monte Carlo error of the same samples."""
    s = SpinSystem(3, 3, [1] * 6, [0.9, -0.6, 0.35, 0.7, -0.45, 0.2], kS=2.0, kT=0.5, T_us=5.0)
    B = np.array([0.0, 1.0, 2.5, 5.0])
    c = cv.ControlVariate(s, B, seed=77, width=64, depth=3)
    _say("cv: generate")
    a_tr, phi_tr = c.generate_training(512)
    # training yield r: direction r of stream 1 at field r % nB (one call over the system once
    # per field), against the oracle
    d = spin.DenseSystem((3, 3), s.two_I, s.a_mT, kS=s.kS, kT=s.kT)
    ph, at = phi_tr.cpu().numpy(), a_tr.cpu().numpy()
    for r in (0, 1, 2, 3, 5, 2046):
        want = yields.FieldOracle(d, B[r % 4], s.T_us).phi(coherent.initial_wavepacket(d, at[r]))
        assert abs(ph[r] - want) < 1e-5 * want, (r, ph[r], want)
    _say("cv: train")
    c.train(a_tr, phi_tr, epochs=80, batch=256, lr=2e-3)
    c.fit_mu(32768)
    a_ev, phi_ev = c.generate(256, stream=cv.STREAM_EVAL)
    m_cv, e_cv = (t.cpu().numpy() for t in c.estimate(a_ev, phi_ev))
    m_pl, e_pl = (t.cpu().numpy() for t in rp.yield_stats(phi_ev))
    exact = np.array([yields.FieldOracle(d, b, s.T_us).trace_yield() for b in B])
    _say("cv", m_cv, e_cv, "plain", m_pl, e_pl, "exact", exact, "val mse", c.val_mse)
    assert np.all(np.abs(m_cv - exact) < 4 * e_cv + 1e-5)
    assert np.all(np.abs(m_pl - exact) < 4 * e_pl + 1e-5)
    # gain: every field improves, and on average the samples needed for a given error fall >= 4x
    assert np.all(e_cv < 0.75 * e_pl)
    assert np.mean((e_cv / e_pl) ** 2) < 0.25
    # the estimator is the oracle's formula applied to the same numbers
    g = c.g(a_ev).cpu().numpy()
    wm, we = stats.cv_mean_error(phi_ev.cpu().numpy(), g, c.mu.cpu().numpy(), c.beta.cpu().numpy(),
                                 c.mu_err.cpu().numpy())
    assert np.max(np.abs(wm - m_cv)) < 1e-12 and np.max(np.abs(we - e_cv)) < 1e-12
    # combined with the plain mean of the (independent) training yields
    m_cb, e_cb = (t.cpu().numpy() for t in c.estimate(a_ev, phi_ev, with_training=True))
    assert np.all(np.abs(m_cb - exact) < 4 * e_cb + 1e-5)
    assert np.all(e_cb < e_cv)
    tm, te = c.train_mean.cpu().numpy(), c.train_err.cpu().numpy()
    om, oe = stats.combine(m_cv, e_cv, tm, te)
    assert np.max(np.abs(om - m_cb)) < 1e-12 and np.max(np.abs(oe - e_cb)) < 1e-12


def test_control_variate_on_the_cv_workload():
    """The learned control variate on the control-variate workload itself (N = 14 spin-1/2,
    Z = 2^14; every fourth of its 32 fields): trained on 1,024 yields, its estimate agrees
    with an independent strength-2 sign-flip design estimate (4 groups of 16 per field, a
    different seed) within 4 combined standard errors at every field, and needs fewer samples
    than plain Monte Carlo on the same evaluation samples."""
    from paper_1612_09517_amd import workloads
    w = workloads.cv_c5()
    s = w.systems[0]
    B = w.fields_mT[0][::4]
    c = cv.ControlVariate(s, B, seed=w.seed, width=256, depth=3, precision=32)
    _say("cv workload: generate")
    a_tr, phi_tr = c.generate_training(128)
    _say("cv workload: train")
    c.train(a_tr, phi_tr, epochs=60, batch=256, lr=1e-3)
    c.fit_mu(32768)
    a_ev, phi_ev = c.generate(64, stream=cv.STREAM_EVAL)
    m_cv, e_cv = (t.cpu().numpy() for t in c.estimate(a_ev, phi_ev))
    m_pl, e_pl = (t.cpu().numpy() for t in rp.yield_stats(phi_ev))
    R = rp.design_size(s.N, 5)
    ang = rp.sample(s, w.seed + 7, 4 * R, basis_mode=5)
    phi_d = rp.propagate(s, B[None, :], ang, 4 * R, precision=32)[0]
    m_d, e_d = (t.cpu().numpy() for t in rp.yield_stats(rp.group_mean(phi_d, R)))
    _say("cv", m_cv, e_cv, "plain", e_pl, "design", m_d, e_d, "val mse", c.val_mse)
    assert np.all(np.abs(m_cv - m_d) < 4 * np.hypot(e_cv, e_d))
    assert np.all(np.abs(m_pl - m_d) < 4 * np.hypot(e_pl, e_d))
    assert np.mean((e_cv / e_pl) ** 2) < 0.6
