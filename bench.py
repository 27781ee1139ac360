"""Benchmark: singlet-yield field sweep of the 7+7 spin-1/2 radical pair (Z = 2^14).

One step = one pass of the hot path over one batch: sample Mb coherent-state
directions, propagate every (field, sample) wavepacket to T = 20 us with the
exact in-step yield integral, and reduce the per-field mean and standard error.
The batch is all 64 fields (0..10 mT) x Mb samples; each step draws fresh samples.

Prints one JSON line (see the repository notes for the field meanings).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def _oracle_worker(task):
    """One oracle propagation (sparse augmented system) of the sweep workload over part of the
    horizon: (sample index, field, horizon fraction) -> (fraction, seconds)."""
    i, B, frac = task
    from oracle import large, philox
    from paper_1612_09517_amd import workloads
    w = workloads.sweep_c2()
    s = w.systems[0]
    sp = large.SparseSystem((s.n1, s.n2), s.two_I, s.a_mT, J_mT=s.J_mT, kS=s.kS, kT=s.kT, gamma=s.gamma)
    a = philox.sample_angles(w.seed, 10 ** 6 + i, 1, s.N)[0]
    t0 = time.perf_counter()
    large.yield_augmented(sp, B, s.T_us * frac, sp.wavepacket(a), tau=1.0)
    return frac, time.perf_counter() - t0


def cpu_baseline(w, seconds_target=20.0):
    """The CPU oracle (sparse augmented system, scipy expm_multiply) on every host core the box
    gives this GPU: one process per core, each propagating its own wavepacket of the bench
    workload at the sweep's middle field over the same part of the horizon (cost is linear in
    the horizon, so the rate is stated in full propagations).  A one-process probe sizes the
    part so that the parallel run takes about seconds_target."""
    from multiprocessing import get_context
    s = w.systems[0]
    B = float(np.median(w.fields_mT[0]))
    cores = max(1, min(16, os.cpu_count() or 1))
    probe_frac = 0.01
    _, dt = _oracle_worker((0, B, probe_frac))
    frac = min(1.0, probe_frac * seconds_target / max(dt, 1e-3) * 0.8)
    env = dict(OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        with get_context("spawn").Pool(cores) as pool:
            t0 = time.perf_counter()
            res = pool.map(_oracle_worker, [(i + 1, B, frac) for i in range(cores)], chunksize=1)
            wall = time.perf_counter() - t0
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    rate = sum(f for f, _ in res) / wall
    return {"value": rate, "unit": "propagations/s", "cores": cores, "kind": "oracle",
            "sample": f"{cores} wavepackets in {cores} processes (one per core), B={B:.3f} mT, each over "
                      f"{frac * s.T_us:.3g} of {s.T_us} us, {wall:.1f} s wall; rate in full propagations "
                      f"(cost linear in the horizon); host has {os.cpu_count()} cores"}


def term_kernel_digest():
    """SHA-256 of the source that decides the term kernel's memory traffic: the device
    structures (kernels.hpp), the Chebyshev-term kernels of rp.hip and the host code that
    sizes chunks and launches them (TiledRun)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1612_09517_amd", "csrc")
    hip = open(os.path.join(csrc, "rp.hip")).read()
    a = hip.index("// " + "-" * 77 + " Chebyshev term")
    b = hip.index("// " + "-" * 77 + " in-step quadrature")
    c = hip.index("struct TiledRun {")
    d = hip.index("\n};\n", c) + 4
    text = open(os.path.join(csrc, "kernels.hpp")).read() + hip[a:b] + hip[c:d]
    return hashlib.sha256(text.encode()).hexdigest()


def measured_traffic(precision, terms_per_step, elements_per_launch):
    """HBM bytes per term launch from the committed counter summary, or None when the
    term kernel's source has changed since the counters were taken (or for FP64, not measured)."""
    f = os.path.join(ROOT, "profiles", "k_cheb_pair_c2_traffic.json")
    if precision != 32 or not os.path.exists(f):
        return None
    doc = json.load(open(f))
    if term_kernel_digest() != doc.get("term_kernel_sha256"):
        return None
    t = doc["per_launch_type"]
    n_acc3 = (terms_per_step - 2) // 3
    n_plain = terms_per_step - 2 - n_acc3
    per_elem = (t["first"]["total"] + n_plain * t["plain"]["total"] + n_acc3 * t["acc3"]["total"]) / (terms_per_step - 1)
    return per_elem * elements_per_launch


def summarize(path):
    """Per-kernel summary of a rocprofv3 CSV output directory (kernel stats and/or counters)."""
    import csv
    import glob
    from collections import defaultdict
    out = {}
    for f in glob.glob(os.path.join(path, "*kernel_stats.csv")):
        for r in csv.DictReader(open(f)):
            out.setdefault(r["Name"], {}).update(
                {"calls": int(r["Calls"]), "avg_us": float(r["AverageNs"]) / 1e3, "pct": float(r["Percentage"])})
    for f in glob.glob(os.path.join(path, "*counter_collection.csv")):
        acc = defaultdict(list)
        for r in csv.DictReader(open(f)):
            acc[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
        for (k, c), v in acc.items():
            out.setdefault(k, {})[c + "_KiB_avg"] = sum(v) / len(v)
            out[k][c + "_dispatches"] = len(v)
    return out


def cv_headline(args):
    """Sweep wall time to eps <= 1e-3 at every field: FP32 + learned control variate (training
    included) against plain FP64 and plain FP32 Monte Carlo, on the control-variate workload
    (the first N=14 system of the batched set, 32 fields).  Rates and standard deviations are
    measured here; the wall times follow from them as M_needed * fields / rate."""
    import torch
    from paper_1612_09517_amd import cv, rp, workloads
    w = workloads.cv_c5()
    s = w.systems[0]
    B = w.fields_mT[0]
    nB = len(B)
    torch.cuda.set_device(0)
    c = cv.ControlVariate(s, B, seed=w.seed, width=256, depth=3, precision=32)
    n_train = args.cv_train // nB
    sync = torch.cuda.synchronize
    sync()
    t0 = time.perf_counter()

    def say(msg):
        print(json.dumps({"progress": msg, "t_s": round(time.perf_counter() - t0, 1)}), flush=True)

    a_tr, phi_tr = c.generate_training(n_train, progress=lambda d, n: say(f"training yields: field {d}/{n}"))
    sync()
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    val = c.train(a_tr, phi_tr, epochs=args.cv_epochs, batch=512, lr=1e-3, augment=not args.cv_no_augment)
    sync()
    t_train = time.perf_counter() - t0
    say(f"trained: validation mse {val:.4f} (standardised), {len(c.history)} epochs")
    t0 = time.perf_counter()
    c.fit_mu(args.cv_quad)
    sync()
    t_mu = time.perf_counter() - t0
    say("mu fitted")
    Me = args.cv_eval
    t0 = time.perf_counter()
    a_ev = rp.sample(s, w.seed, Me, stream_id=cv.STREAM_EVAL)
    phi_ev = rp.propagate(s, B[None, :], a_ev, Me, precision=32)[0]
    sync()
    rate32 = Me * nB / (time.perf_counter() - t0)
    say(f"evaluation samples done, {rate32:.1f} propagations/s")
    m_cv, e_cv = (x.cpu().numpy() for x in c.estimate(a_ev, phi_ev))
    m_pl, e_pl = (x.cpu().numpy() for x in rp.yield_stats(phi_ev))
    M64 = max(4, Me // 8)
    t0 = time.perf_counter()
    a64 = rp.sample(s, w.seed, M64, first=10 ** 6, stream_id=cv.STREAM_EVAL)
    rp.propagate(s, B[None, :], a64, M64, precision=64)
    sync()
    rate64 = M64 * nB / (time.perf_counter() - t0)
    sig_pl = e_pl * np.sqrt(Me)
    sig_cv = e_cv * np.sqrt(Me)        # includes the (small) contribution of mu's error
    eps = 1e-3
    M_pl = float(np.ceil(np.max((sig_pl / eps) ** 2)))
    M_cv = float(np.ceil(np.max((sig_cv / eps) ** 2)))
    # With the plain mean of the training yields combined in (rp_combine), a field needs
    # sigma_cv^2 (1/eps^2 - 1/err_train^2) evaluation samples.
    e_tr = c.train_err.cpu().numpy()
    M_cb = float(np.ceil(np.max(sig_cv ** 2 * np.maximum(0.0, 1.0 / eps ** 2 - 1.0 / e_tr ** 2))))
    wall64 = M_pl * nB / rate64
    wall32 = M_pl * nB / rate32
    wall_cv_only = t_gen + t_train + t_mu + M_cv * nB / rate32
    wall_cv = t_gen + t_train + t_mu + M_cb * nB / rate32
    m_cb, e_cb = (x.cpu().numpy() for x in c.estimate(a_ev, phi_ev, with_training=True))
    rec = {"metric": "sweep wall time at sigma(Phi_S)<=1e-3: FP32 + learned control variate vs plain FP64 MC",
           "value": wall_cv, "unit": "s", "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
           "dtype": "f32", "config": {"workload": w.name + ": N=14 spin-1/2, Z=16384, 32 fields 0..5 mT",
                                      "kS": s.kS, "kT": s.kT, "T_us": s.T_us, "train_yields": n_train * nB,
                                      "eval_samples": Me, "mu_samples": args.cv_quad, "net": "3x256 GELU, BF16 MFMA",
                                      "augment": not args.cv_no_augment, "epochs_run": len(c.history)},
           "plain_fp64_wall_s": wall64, "plain_fp32_wall_s": wall32, "speedup_vs_fp64": wall64 / wall_cv,
           "cv_without_training_mean_wall_s": wall_cv_only,
           "rate_fp32_props_s": rate32, "rate_fp64_props_s": rate64,
           "train_s": {"generate": t_gen, "fit": t_train, "mu": t_mu}, "val_mse_standardised": val,
           "samples_needed": {"plain": M_pl, "cv": M_cv, "cv_with_training_mean": M_cb},
           "sigma_plain_max": float(sig_pl.max()), "sigma_cv_max": float(sig_cv.max()),
           "variance_ratio_mean": float(np.mean((e_cv / e_pl) ** 2)),
           "cv_minus_plain_over_err": float(np.max(np.abs(m_cv - m_pl) / np.sqrt(e_cv ** 2 + e_pl ** 2))),
           "combined_minus_plain_over_err": float(np.max(np.abs(m_cb - m_pl) / np.sqrt(e_cb ** 2 + e_pl ** 2)))}
    print(json.dumps(rec), flush=True)


def sequential_sweep(nB, eps, initial, draw, stats, say, label):
    """The stopping rule every estimator of the headline shares: each round draws fresh units
    (samples, or design groups) for each field whose standard error is still above eps, as many
    as that field needs, n (err / eps_f)^2 x 1.05 from its current error (at least one more),
    until none is; fields that need the same number share one draw.
    draw(fields, n, first) -> CUDA [len(fields)][n] new units; stats(f, units) -> (mean, err,
    ratio): the estimate, its error, and the ratio of the units' own error to the error they
    must reach (err / eps, or a smaller target when another estimate is combined in).  Returns
    per-field means, errors, unit counts and rounds."""
    import torch
    store = [None] * nB
    done = np.zeros(nB, int)
    need = np.full(nB, initial)
    mean, err = np.zeros(nB), np.full(nB, np.inf)
    rounds = 0
    while True:
        todo = np.nonzero(need > done)[0]
        if todo.size == 0:
            break
        # fields that need the same number of new units share one draw (and one call)
        for n in sorted(set(int(x) for x in need[todo] - done[todo])):
            fields = todo[need[todo] - done[todo] == n]
            new = draw(fields, n, int(done[fields].max()))
            for j, f in enumerate(fields):
                store[f] = new[j] if store[f] is None else torch.cat([store[f], new[j]])
        for f in todo:
            done[f] = store[f].numel()
            m, e, ratio = stats(f, store[f])
            mean[f], err[f] = m, e
            need[f] = done[f] if e <= eps else max(done[f] + 1, int(np.ceil(done[f] * ratio ** 2 * 1.05)))
        rounds += 1
        say(f"{label}: round {rounds}, {int(done.sum())} units, max error {err.max():.2e}")
    return mean, err, done, rounds


def headline_sweeps(args, say):
    """Measured sweeps to eps <= 1e-3 at every field of the control-variate workload (the first
    N=14 system of the batched set: Z = 2^14, 32 fields 0..5 mT, T = 20 us): plain Monte Carlo
    with complex-FP64 wavepackets (the baseline), complex FP32 with the strength-2 sign-flip
    design (groups of 16), and complex FP32 with the learned control variate (training-yield
    generation, training and the mean of the network included) combined with the training
    yields' own plain mean.  Each leg is timed end to end on the GPU with the same sequential
    stopping rule; samples come from separate seeds."""
    import torch
    from paper_1612_09517_amd import cv, rp, workloads
    w = workloads.cv_c5()
    s = w.systems[0]
    B = w.fields_mT[0]
    nB = len(B)
    eps = 1e-3
    sync = torch.cuda.synchronize
    legs = set(args.headline_legs.split(","))
    out = {"workload": f"{w.systems[0].name}: N=14 spin-1/2 (7+7), Z=16384, {nB} fields {B[0]:g}..{B[-1]:g} mT, "
                       f"T={s.T_us:g} us, kS={s.kS:.4f}, kT={s.kT:.4f} /us",
           "eps": eps, "rule": "a pilot of 64 wavepackets per field (design: 4 groups of 16; control variate: "
                               "16 evaluation samples after the training yields), then rounds of fresh units for the "
                               "fields whose standard error is above eps, n (err/eps)^2 x 1.05 each, until every "
                               "field is at or below eps"}

    def propagate_fields(fields, ang, n, prec):
        parts = []
        for c0 in range(0, len(fields), 16):
            fs = fields[c0:c0 + 16]
            parts.append(rp.propagate(s, B[fs][None, :], ang, n, precision=prec)[0])
        return torch.cat(parts)

    def plain_stats(f, u):
        m, e = rp.yield_stats(u[None, :])
        return float(m[0]), float(e[0]), float(e[0]) / eps

    means = {}
    if "fp64" in legs:
        sync()
        t0 = time.perf_counter()
        props = [0]

        def draw64(fields, n, first):
            props[0] += n * len(fields)
            return propagate_fields(fields, rp.sample(s, w.seed + 1, n, first=first), n, 64)

        m, e, done, rounds = sequential_sweep(nB, eps, 64, draw64, plain_stats, say, "plain FP64")
        sync()
        wall = time.perf_counter() - t0
        means["plain_fp64"] = (m, e)
        out["plain_fp64"] = {"wall_s": wall, "propagations": props[0], "rate_props_s": props[0] / wall,
                             "samples_per_field_max": int(done.max()), "rounds": rounds, "err_max": float(e.max())}
    if "design" in legs:
        mode = 5
        R = rp.design_size(s.N, mode)
        sync()
        t0 = time.perf_counter()
        props = [0]

        def draw_design(fields, G, first):
            props[0] += G * R * len(fields)
            ang = rp.sample(s, w.seed + 2, G * R, first=first * R, basis_mode=mode)
            return rp.group_mean(propagate_fields(fields, ang, G * R, 32), R)

        # the same pilot as plain Monte Carlo: 64 wavepackets per field (4 groups of 16)
        m, e, done, rounds = sequential_sweep(nB, eps, max(2, 64 // R), draw_design, plain_stats, say,
                                              "FP32 design")
        sync()
        wall = time.perf_counter() - t0
        means["design_fp32"] = (m, e)
        out["design_fp32"] = {"wall_s": wall, "propagations": props[0], "rate_props_s": props[0] / wall,
                              "design": f"rp_sample mode {mode}, {R} samples per group (orthogonal array of strength 2)",
                              "groups_per_field_max": int(done.max()), "rounds": rounds, "err_max": float(e.max())}
    if "cv" in legs:
        sync()
        t0 = time.perf_counter()
        c = cv.ControlVariate(s, B, seed=w.seed, width=256, depth=3, precision=32)
        a_tr, phi_tr = c.generate_training(args.cv_train // nB)
        sync()
        t_gen = time.perf_counter() - t0
        say(f"control variate: {args.cv_train // nB * nB} training yields in {t_gen:.1f} s")
        val = c.train(a_tr, phi_tr, epochs=args.cv_epochs, batch=512, lr=1e-3, augment=True)
        sync()
        t_fit = time.perf_counter() - t0 - t_gen
        c.fit_mu(args.cv_quad)
        tr_m, tr_e = c.train_mean.cpu().numpy(), c.train_err.cpu().numpy()
        say(f"control variate: trained (validation mse {val:.3f}), mu fitted")
        props = [args.cv_train // nB * nB]
        gs = [None] * nB

        def draw_cv(fields, n, first):
            props[0] += n * len(fields)
            ang = rp.sample(s, w.seed, n, first=first, stream_id=cv.STREAM_EVAL)
            phi = propagate_fields(fields, ang, n, 32)
            g = c.g(ang)[fields]
            for j, f in enumerate(fields):
                gs[f] = g[j] if gs[f] is None else torch.cat([gs[f], g[j]])
            return phi

        def cv_stats(f, u):
            m, e = rp.yield_stats(u[None, :], gs[f][None, :], c.mu[f:f + 1], c.beta[f:f + 1], c.mu_err[f:f + 1])
            mc, ec = rp.combine(m, e, c.train_mean[f:f + 1], c.train_err[f:f + 1])
            # combined with the training mean, the control-variate estimate itself must reach
            # (1/eps^2 - 1/err_train^2)^(-1/2)
            tgt = np.inf if tr_e[f] <= eps else (1.0 / eps ** 2 - 1.0 / tr_e[f] ** 2) ** -0.5
            return float(mc[0]), float(ec[0]), float(e[0]) / tgt

        m, e, done, rounds = sequential_sweep(nB, eps, 16, draw_cv, cv_stats, say, "FP32 control variate")
        sync()
        wall = time.perf_counter() - t0
        means["cv_fp32"] = (m, e)
        out["cv_fp32"] = {"wall_s": wall, "propagations": props[0],
                          "train": {"yields": args.cv_train // nB * nB, "generate_s": t_gen, "fit_s": t_fit,
                                    "epochs_run": len(c.history), "val_mse_standardised": val,
                                    "mu_samples": args.cv_quad, "net": "3x256 GELU, BF16 MFMA, FP32 master weights"},
                          "eval_samples_per_field_max": int(done.max()), "rounds": rounds,
                          "err_max": float(e.max())}
    if "plain_fp64" in means:
        m64, e64 = means["plain_fp64"]
        for k in ("design_fp32", "cv_fp32"):
            if k in means:
                m, e = means[k]
                out[k]["speedup_vs_plain_fp64"] = out["plain_fp64"]["wall_s"] / out[k]["wall_s"]
                out[k]["max_dev_from_plain_fp64_over_err"] = float(np.max(np.abs(m - m64) / np.sqrt(e ** 2 + e64 ** 2)))
    return out


def other_workload(args):
    """Throughput of the other workloads (one JSON line each): the tiny Z=8 system, a strided
    subset of the 256 uneven systems (one call: small systems in the LDS-resident launches,
    larger ones tiled), a subset of the large spin-1 system, and the paper's Table I model."""
    import torch
    from paper_1612_09517_amd import rp, workloads
    torch.cuda.set_device(0)
    name = args.workload
    if name == "tiny":
        w = workloads.tiny_c1()
        systems, B, M = w.systems, w.fields_mT, w.M
    elif name == "batched":
        w = workloads.batched_c3()
        sel = [i for i in range(0, len(w.systems), args.stride) if w.systems[i].N <= args.max_n]
        systems = [w.systems[i] for i in sel]
        B, M = w.fields_mT[sel], args.samples_per_step
    elif name == "large":
        w = workloads.large_c4(n_fields=args.fields)
        systems, B, M = w.systems, w.fields_mT, args.samples_per_step
    elif name == "paper":
        w = workloads.paper_model(n_fields=args.fields)
        systems, B, M = w.systems, w.fields_mT, args.samples_per_step
    else:
        raise SystemExit("unknown workload " + name)
    R = max(rp.design_size(s.N, args.sampler) for s in systems)
    if M % R:
        raise SystemExit(f"--samples-per-step must be a multiple of the design size {R}")
    angs = [rp.sample(s, w.seed + i, M, basis_mode=args.sampler) for i, s in enumerate(systems)]
    cat = torch.cat([a.reshape(-1) for a in angs])
    for _ in range(args.warmup):
        rp.propagate(systems, B, cat, M, precision=args.precision, workspace_bytes=int(args.workspace_gb * 2 ** 30),
                     xcd=args.xcd)
    torch.cuda.synchronize()
    # Long single-system sweeps run a few fields per call and report each call.
    group = args.field_group if (args.field_group > 0 and len(systems) == 1) else B.shape[1]
    t0 = time.perf_counter()
    for _ in range(args.steps):
        parts = []
        for f0 in range(0, B.shape[1], group):
            parts.append(rp.propagate(systems, B[:, f0:f0 + group], cat, M, precision=args.precision,
                                      workspace_bytes=int(args.workspace_gb * 2 ** 30), xcd=args.xcd))
            if group < B.shape[1]:
                torch.cuda.synchronize()
                print(json.dumps({"progress": f"fields {f0 + len(B[0, f0:f0 + group])}/{B.shape[1]}",
                                  "t_s": round(time.perf_counter() - t0, 1)}), flush=True)
        phi = torch.cat(parts, dim=1)
        # sign-flip designs: the group means are the independent units
        mean, err = rp.yield_stats(rp.group_mean(phi.reshape(-1, M), R) if R > 1 else phi.reshape(-1, M))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    prof = None
    if name in ("large", "paper") and not args.no_profile_call:
        # one extra profiled call (tiled kernels) for the term-kernel bandwidth
        rp.propagate(systems, B, cat, M, precision=args.precision, workspace_bytes=int(args.workspace_gb * 2 ** 30),
                     profile=True, xcd=args.xcd)
        p = rp.profile_last()
        prof = {"term_ms": p["term_ms"], "quad_ms": p["quad_ms"], "total_ms": p["total_ms"],
                "term_GBps": p["elements"] * p["bytes_per_element"] / (p["term_ms"] * 1e-3) / 1e9,
                "terms_per_step": p["terms_per_step"]}
    props = len(systems) * B.shape[1] * M
    Zs = [s.Z for s in systems]
    rec = {"metric": "propagations per second", "value": props / dt, "unit": "propagations/s",
           "higher_is_better": True, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": dt * 1e3, "dtype": "f32" if args.precision == 32 else "f64", "data": "synthetic",
           "config": {"workload": w.name, "systems": len(systems), "fields": int(B.shape[1]), "samples": M,
                      "Z_min": min(Zs), "Z_max": max(Zs), "sampler": args.sampler, "design_size": R},
           "phi_mean_first_system": [round(float(x), 6) for x in mean[:B.shape[1]].cpu().numpy()],
           "phi_err_first_system": [round(float(x), 6) for x in err[:B.shape[1]].cpu().numpy()],
           "fields_first_system": [round(float(x), 4) for x in B[0]], "profile": prof}
    print(json.dumps(rec), flush=True)


def trace_vs_mc(args):
    """Deterministic trace (Eq. 14: all Z basis states |S, M>) against the Monte Carlo estimate
    (Eq. 18: M = 200 coherent states) on one MI355X: wall times, their ratio (the paper quotes
    only the count ratio Z/M), and the Monte Carlo error against the exact trace."""
    import torch
    from paper_1612_09517_amd import rp, workloads
    torch.cuda.set_device(0)
    w = workloads.batched_c3()
    s = next(x for x in w.systems if x.N == args.trace_n)
    B = w.fields_mT[0][:: max(1, w.fields_mT.shape[1] // 8)][None, :]
    dig = rp.sample(s, 0, s.Z, basis_mode=2)
    ang = rp.sample(s, w.seed, 200)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    tr, t_tr = timed(lambda: rp.propagate(s, B, dig, s.Z, init_mode=1, precision=args.precision))
    mc, t_mc = timed(lambda: rp.propagate(s, B, ang, 200, precision=args.precision))
    trace = tr[0].mean(dim=1)
    mean, err = rp.yield_stats(mc[0])
    z = ((mean - trace).abs() / err).cpu().numpy()
    print(json.dumps({"metric": "deterministic trace vs Monte Carlo wall time", "system": s.name, "Z": s.Z,
                      "fields": int(B.shape[1]), "M": 200, "trace_s": t_tr, "mc_s": t_mc,
                      "wall_ratio": t_tr / t_mc, "count_ratio": s.Z / 200,
                      "max_abs_dev_over_eps": float(z.max()), "dtype": f"f{args.precision}"}), flush=True)


def design_headline(args):
    """Sweep wall time to eps <= 1e-3 at every field with coherent states in a sign-flip design
    (rp_sample mode 5 by default: strength-2 orthogonal array, 16 samples per group for N = 14)
    in complex FP32, measured end to end: groups are added to the fields whose standard error
    (over group means) is above eps until none is, starting from --design-groups groups.
    Plain FP64 and plain FP32 Monte Carlo wall times follow from measured rates and the
    per-sample deviation of a plain pilot, as M_needed * fields / rate.  The workload of --cv,
    or with --design-workload sweep the bench sweep (64 fields 0..10 mT)."""
    import torch
    from paper_1612_09517_amd import rp, workloads
    w = workloads.sweep_c2() if args.design_workload == "sweep" else workloads.cv_c5()
    s = w.systems[0]
    B = w.fields_mT[0]
    nB = len(B)
    torch.cuda.set_device(0)
    sync = torch.cuda.synchronize
    eps = 1e-3
    mode = args.design_mode
    R = rp.design_size(s.N, mode)
    t00 = time.perf_counter()

    def say(msg):
        print(json.dumps({"progress": msg, "t_s": round(time.perf_counter() - t00, 1)}), flush=True)

    # group means per field, grown until every field's error is below eps
    sync()
    t0 = time.perf_counter()
    gm = [None] * nB                     # per field: CUDA tensor of its group means
    mean_d, err_d = np.zeros(nB), np.full(nB, np.inf)
    need = np.full(nB, args.design_groups)
    done = np.zeros(nB, int)
    props = 0
    rounds = 0
    while True:
        todo = np.nonzero(need > done)[0]
        if todo.size == 0:
            break
        G = int(np.max(need[todo] - done[todo]))
        first = int(done[todo].max()) * R   # fresh groups for every field in this round
        a = rp.sample(s, w.seed, G * R, first=first, basis_mode=mode)
        parts = []
        for c0 in range(0, todo.size, 16):          # 16 fields per call, with progress
            fs = todo[c0:c0 + 16]
            parts.append(rp.group_mean(rp.propagate(s, B[fs][None, :], a, G * R, precision=32)[0], R))
            say(f"round {rounds + 1}: fields {c0 + fs.size}/{todo.size}")
        g = torch.cat(parts)
        props += G * R * todo.size
        for j, f in enumerate(todo):
            gm[f] = g[j] if gm[f] is None else torch.cat([gm[f], g[j]])
            done[f] = gm[f].numel()
            m, e = rp.yield_stats(gm[f][None, :])
            mean_d[f], err_d[f] = float(m[0]), float(e[0])
        need = np.where(err_d > eps, np.ceil(done * (err_d / eps) ** 2 * 1.05).astype(int), done)
        rounds += 1
        say(f"round {rounds}: {props} propagations, max error {err_d.max():.2e}")
    sync()
    wall_design = time.perf_counter() - t0
    # plain pilot (FP32) and the FP64 rate
    Me = args.cv_eval
    t0 = time.perf_counter()
    a_ev = rp.sample(s, w.seed + 1, Me)
    phi_ev = torch.cat([rp.propagate(s, B[None, c0:c0 + 16], a_ev, Me, precision=32)[0]
                        for c0 in range(0, nB, 16)])
    sync()
    rate32 = Me * nB / (time.perf_counter() - t0)
    m_pl, e_pl = (x.cpu().numpy() for x in rp.yield_stats(phi_ev))
    say(f"plain pilot done, {rate32:.1f} propagations/s")
    M64 = max(4, Me // 8)
    t0 = time.perf_counter()
    rp.propagate(s, B[None, :], rp.sample(s, w.seed + 2, M64), M64, precision=64)
    sync()
    rate64 = M64 * nB / (time.perf_counter() - t0)
    sig_pl = e_pl * np.sqrt(Me)
    M_pl = float(np.ceil(np.max((sig_pl / eps) ** 2)))
    wall64 = M_pl * nB / rate64
    wall32 = M_pl * nB / rate32
    # variance of the mean from n samples: plain sigma^2 / n, design err^2 G R / n
    vr = sig_pl ** 2 / (err_d ** 2 * done * R)
    rec = {"metric": "sweep wall time at sigma(Phi_S)<=1e-3: FP32 + sign-flip design vs plain FP64 MC",
           "value": wall_design, "unit": "s", "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
           "dtype": "f32", "config": {"workload": w.name + f": N=14 spin-1/2, Z=16384, {nB} fields "
                                                   f"{B[0]:g}..{B[-1]:g} mT, T={s.T_us:g} us",
                                      "design_mode": mode, "samples_per_group": R,
                                      "initial_groups": args.design_groups, "plain_pilot_samples": Me},
           "plain_fp64_wall_s": wall64, "plain_fp32_wall_s": wall32, "speedup_vs_fp64": wall64 / wall_design,
           "speedup_vs_fp32": wall32 / wall_design,
           "rate_fp32_props_s": rate32, "rate_fp64_props_s": rate64, "design_propagations": props,
           "design_rounds": rounds, "groups_min": int(done.min()), "groups_max": int(done.max()),
           "samples_needed": {"plain": M_pl, "design_max": int(done.max()) * R},
           "design_err_max": float(err_d.max()), "sigma_plain_max": float(sig_pl.max()),
           "variance_reduction_at_equal_samples": {"min": float(vr.min()), "median": float(np.median(vr)),
                                                   "max": float(vr.max())},
           "design_minus_plain_over_err": float(np.max(np.abs(mean_d - m_pl) / np.sqrt(err_d ** 2 + e_pl ** 2)))}
    print(json.dumps(rec), flush=True)


def sampling_variance(args):
    """Monte Carlo samplers at equal cost on the sweep system: coherent states (Eq. 15), random
    J_z eigenstates (Sec. V, last paragraph), and coherent states in sign-flip designs
    (antithetic pairs, orthogonal arrays of strength 3 and 2: the uniform measure of Eq. 17 is
    invariant under n -> -n).  Reports the per-sample standard deviation and, for every
    sampler, the variance of its estimate of the mean with M propagations (design groups as
    the independent units)."""
    import torch
    from paper_1612_09517_amd import rp, workloads
    torch.cuda.set_device(0)
    if args.sampling_system == "paper":
        w = workloads.paper_model()
        B = np.array([[1.0, 3.5]])
    else:
        w = workloads.sweep_c2()
        B = np.array([[0.0, 2.5, 10.0]])
    s = w.systems[0]
    modes = {"coherent": 0, "jz": 1, "antithetic": 3, "oa3": 4, "oa2": 5}
    chosen = [(n, modes[n]) for n in args.samplers.split(",")]
    Rmax = max(rp.design_size(s.N, m) for _, m in chosen)
    M = -(-args.samples_per_step // Rmax) * Rmax      # whole design groups
    out = {}
    for name, mode in chosen:
        t0 = time.time()
        ang = rp.sample(s, w.seed, M, basis_mode=mode)
        phi = rp.propagate(s, B, ang, M, init_mode=1 if mode == 1 else 0, precision=args.precision)[0]
        R = rp.design_size(s.N, mode)
        units = rp.group_mean(phi, R) if R > 1 else phi
        mean, err = rp.yield_stats(units)
        _, err1 = rp.yield_stats(phi)
        torch.cuda.synchronize()
        out[name] = {"mean": mean.cpu().numpy(), "est_var": (err ** 2).cpu().numpy(),
                     "per_sample_sigma": (err1 * np.sqrt(M)).cpu().numpy(), "group": R,
                     "units": M // R}
        print(f"sampler {name}: {M} propagations x {B.shape[1]} fields in {time.time() - t0:.1f} s",
              file=sys.stderr, flush=True)
    c = out[chosen[0][0]]
    rec = {"metric": "Monte Carlo samplers at equal cost (variance of the mean estimate)", "system": s.name,
           "reference_sampler": chosen[0][0],
           "fields_mT": B[0].tolist(), "M": M, "dtype": f"f{args.precision}"}
    for name, v in out.items():
        rec[name] = {"group": v["group"], "independent_units": v["units"],
                     "per_sample_sigma": v["per_sample_sigma"].tolist(),
                     "mean": v["mean"].tolist(), "stderr": np.sqrt(v["est_var"]).tolist(),
                     "variance_reduction_vs_reference": (c["est_var"] / v["est_var"]).tolist(),
                     "mean_diff_over_eps": (np.abs(v["mean"] - c["mean"]) /
                                            np.sqrt(v["est_var"] + c["est_var"])).tolist()}
    print(json.dumps(rec), flush=True)


def arnoldi_ablation(args):
    """The paper's short-iterative Arnoldi propagator (RP_FLAG_ARNOLDI, Krylov dimension 16)
    against the Chebyshev series on the sweep system (horizon cut to 2 us), and on the Sec. IV
    model (strong dissipation, horizon 0.1 us): wall time, operator applications per
    wavepacket and the largest relative difference of the yields, at equal seeded inputs."""
    import dataclasses
    import torch
    from paper_1612_09517_amd import rp, workloads
    torch.cuda.set_device(0)
    for w, T, B in ((workloads.sweep_c2(), 2.0, [0.0, 5.0, 10.0]), (workloads.paper_model(), 0.1, [0.5, 3.5])):
        s = dataclasses.replace(w.systems[0], T_us=T)
        Bf = np.array([B])
        M = args.samples_per_step
        ang = rp.sample(s, w.seed, M)
        res = {}
        for name, kw in (("chebyshev", {}), ("arnoldi", {"arnoldi": True})):
            rp.propagate(s, Bf[:, :1], ang[:1].contiguous(), 1, precision=args.precision, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            phi = rp.propagate(s, Bf, ang, M, precision=args.precision, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            res[name] = (phi[0].cpu().numpy(), dt)
        rp.propagate(s, Bf, ang, M, precision=args.precision, arnoldi=True, profile=True)
        p = rp.profile_last()
        jobs = Bf.shape[1] * M
        cheb_terms = sum(rp.plan_field(s, b, precision=args.precision)["n_terms"] *
                         rp.plan_field(s, b, precision=args.precision)["n_steps"] for b in B) * M / jobs
        diff = np.abs(res["arnoldi"][0] - res["chebyshev"][0]) / np.abs(res["chebyshev"][0])
        print(json.dumps({"metric": "Arnoldi vs Chebyshev propagator", "system": s.name, "T_us": T, "fields_mT": B,
                          "samples": M, "dtype": f"f{args.precision}",
                          "chebyshev_s": res["chebyshev"][1], "arnoldi_s": res["arnoldi"][1],
                          "time_ratio": res["arnoldi"][1] / res["chebyshev"][1],
                          "chebyshev_terms_per_job": cheb_terms,
                          "arnoldi_applications_per_job": p["terms_per_step"] / jobs,
                          "arnoldi_steps_per_job": p["quad_launches"] / jobs,
                          "max_rel_diff": float(diff.max())}), flush=True)


def histogram(args):
    """Distribution of single-wavepacket yields of the Sec. IV model at three fields (the
    paper's Fig. 4 workload: 1000 samples per field): mean, sigma (Eq. 23), quantiles and a
    20-bin histogram per field; the paper bounds sigma by 1/2."""
    import torch
    from paper_1612_09517_amd import rp, workloads
    torch.cuda.set_device(0)
    w = workloads.paper_model()
    s = w.systems[0]
    M = args.samples_per_step
    t0 = time.perf_counter()
    out = []
    for B in (0.0, 3.5, 10.0):
        parts = []
        for m0 in range(0, M, 250):
            m = min(250, M - m0)
            ang = rp.sample(s, w.seed, m, first=m0)
            parts.append(rp.propagate(s, np.array([[B]]), ang, m, precision=args.precision)[0, 0].cpu().numpy())
            print(json.dumps({"progress": f"B={B} samples {m0 + m}/{M}", "t_s": round(time.perf_counter() - t0, 1)}),
                  flush=True)
        phi = np.concatenate(parts)
        h, edges = np.histogram(phi, bins=20, range=(0.0, 1.0))
        out.append({"B_mT": B, "mean": float(phi.mean()), "sigma": float(phi.std(ddof=1)),
                    "eps": float(phi.std(ddof=1) / np.sqrt(M)), "min": float(phi.min()), "max": float(phi.max()),
                    "quantiles_5_25_50_75_95": [float(q) for q in np.quantile(phi, [0.05, 0.25, 0.5, 0.75, 0.95])],
                    "histogram_0_to_1_20_bins": h.tolist()})
    print(json.dumps({"metric": "single-wavepacket yield distribution, Sec. IV model", "samples": M,
                      "dtype": f"f{args.precision}", "wall_s": time.perf_counter() - t0, "fields": out}), flush=True)


def batched_classes(args):
    """The batched workload (256 uneven systems) by size class, on a horizon cut to args.class_t
    us (the cost of a propagation is linear in its horizon; the full workload is about 6.6 h at
    70 % of the HBM peak): for every N = 8..18 the first args.per_class systems of that size,
    every eighth of their 32 fields and enough samples (at least args.samples_per_step) for
    about 2^21 nuclear states per call, one call per class; then
    all of them in one call (the LDS-resident launches plus one job queue of unequal Z).  Rates
    are in wavepacket-microseconds per second and, divided by each system's own horizon, in
    propagations per second at the workload's horizons; the tiled classes also report the term
    kernel's algorithmic GB/s from a profiled call."""
    import dataclasses
    import torch
    from paper_1612_09517_amd import rp, workloads
    torch.cuda.set_device(0)
    w = workloads.batched_c3()
    M = args.samples_per_step
    fsel = list(range(0, w.fields_mT.shape[1], 8))
    chosen, classes = [], []
    for N in range(8, 19):
        idx = [i for i, x in enumerate(w.systems) if x.N == N][:args.per_class]
        chosen += idx
        classes.append((N, idx))
    t00 = time.perf_counter()

    def run(idx, profile=False):
        full = [w.systems[i] for i in idx]
        systems = [dataclasses.replace(x, T_us=min(x.T_us, args.class_t)) for x in full]
        B = w.fields_mT[idx][:, fsel]
        # samples so that a class holds about 2^21 nuclear states in all (a full job queue)
        M = max(args.samples_per_step, -(-(1 << 21) // (sum(x.Z for x in systems) * B.shape[1])))
        cat = torch.cat([rp.sample(x, w.seed, M).reshape(-1) for x in systems])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rp.propagate(systems, B, cat, M, precision=args.precision, xcd=args.xcd)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        jobs = len(idx) * B.shape[1] * M
        wp_us = sum(x.T_us for x in systems) * B.shape[1] * M
        full_props = sum(x.T_us / y.T_us for x, y in zip(systems, full)) * B.shape[1] * M
        out = {"systems": len(idx), "samples": M, "jobs": jobs, "horizon_us": [round(x.T_us, 3) for x in systems],
               "wall_s": dt,
               "wavepacket_us_per_s": wp_us / dt, "propagations_per_s_at_own_horizon": full_props / dt}
        if profile:
            rp.propagate(systems, B, cat, M, precision=args.precision, profile=True, xcd=args.xcd)
            p = rp.profile_last()
            gbs = p["elements"] * p["bytes_per_element"] / (p["term_ms"] * 1e-3) / 1e9
            out.update({"term_GBps": gbs, "term_frac_of_8TBps": gbs / PEAK_HBM_GBS,
                        "term_time_frac": p["term_ms"] / p["total_ms"], "quad_time_frac": p["quad_ms"] / p["total_ms"]})
        return out

    rec = {"metric": "batched workload by size class", "dtype": f"f{args.precision}", "min_samples": args.samples_per_step,
           "fields": [float(x) for x in w.fields_mT[0][fsel]], "per_class": args.per_class,
           "horizon_cut_us": args.class_t, "classes": {}}
    for N, idx in classes:
        rec["classes"][f"N={N} Z={2 ** N}"] = run(idx, profile=2 ** N > (1024 if args.precision == 32 else 512))
        print(json.dumps({"progress": f"class N={N} done", "t_s": round(time.perf_counter() - t00, 1)}),
              file=sys.stderr, flush=True)
    rec["all_in_one_call"] = run(chosen)
    print(json.dumps(rec), flush=True)


def mlp_timing(args):
    """The control-variate network's kernels on their own: one Adam training step (forward,
    backward, update) and one forward pass of the 43 -> 3 x 256 -> 1 network on a batch of 512
    rows, averaged over 200 calls, with the MFMA work they do."""
    import torch
    from paper_1612_09517_amd import rp
    torch.cuda.set_device(0)
    n_in, width, depth, rows = 43, 256, 3, 512
    rng = np.random.default_rng(0)
    P = torch.tensor(rng.normal(0, 0.05, rp.mlp_param_count(n_in, width, depth)).astype(np.float32), device="cuda")
    Mo, V = torch.zeros_like(P), torch.zeros_like(P)
    x = rp.mlp_features(torch.tensor(rng.uniform(-1, 1, (rows, 14, 2)), device="cuda"), [1.0], n_in)
    t = torch.tensor(rng.normal(0, 1, rows).astype(np.float32), device="cuda")
    ws = rp.mlp_workspace(n_in, width, depth, rows)
    pad = rp.mlp_in_pad(n_in)
    flops_fwd = 2 * rows * (pad * width + (depth - 1) * width * width)
    out = {}
    for name, fn, fl in (("train_step", lambda i: rp.mlp_train_step(P, Mo, V, i + 1, x, t, n_in, width, depth, lr=1e-4,
                                                                     workspace=ws), 3 * flops_fwd),
                         ("forward", lambda i: rp.mlp_forward(P, x, n_in, width, depth, workspace=ws), flops_fwd)):
        for i in range(10):
            fn(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(200):
            fn(i)
        torch.cuda.synchronize()
        us = (time.perf_counter() - t0) / 200 * 1e6
        out[name] = {"us_per_call": us, "gemm_TFLOPs": fl / (us * 1e-6) / 1e12}
    print(json.dumps({"metric": "control-variate network kernels", "rows": rows, "net": f"{n_in}->{depth}x{width}->1",
                      **out}), flush=True)


def convergence(args):
    """The Sec. IV model's field sweep at M = 100, 200 and 400 (the convergence study of Fig. 2:
    M = 100 and M = 200 against a well converged M = 400), from three disjoint sets of seeded
    samples (0..99, 100..299, 300..699).  One call computes the samples args.sample_range a:b
    for every field (complex FP32) and saves the yields [fields][b - a] to args.out (.npy);
    with args.combine it reads the saved files and prints the three curves with their errors
    (Eq. 23) and the deviations of M = 100 and 200 from M = 400."""
    from paper_1612_09517_amd import workloads
    w = workloads.paper_model(n_fields=args.fields)
    s = w.systems[0]
    B = w.fields_mT
    if args.combine:
        parts = [np.load(f) for f in args.combine.split(",")]
        phi = np.concatenate(parts, axis=1)
        sets = {"M100": phi[:, :100], "M200": phi[:, 100:300], "M400": phi[:, 300:700]}
        out = {}
        for k, v in sets.items():
            out[k] = {"mean": v.mean(axis=1).tolist(), "eps": (v.std(axis=1, ddof=1) / np.sqrt(v.shape[1])).tolist()}
        ref = np.array(out["M400"]["mean"])
        for k in ("M100", "M200"):
            d = np.array(out[k]["mean"]) - ref
            e = np.hypot(np.array(out[k]["eps"]), np.array(out["M400"]["eps"]))
            out[k]["max_abs_dev_from_M400"] = float(np.abs(d).max())
            out[k]["max_dev_over_err"] = float(np.max(np.abs(d) / e))
        print(json.dumps({"metric": "Fig. 2 convergence study, Sec. IV model", "fields_mT": B[0].tolist(), **out}),
              flush=True)
        return
    import torch
    from paper_1612_09517_amd import rp
    torch.cuda.set_device(0)
    a, b = (int(x) for x in args.sample_range.split(":"))
    t0 = time.perf_counter()
    parts = []
    for m0 in range(a, b, args.samples_per_step):
        m = min(args.samples_per_step, b - m0)
        ang = rp.sample(s, w.seed, m, first=m0)
        parts.append(rp.propagate(s, B, ang, m, precision=args.precision)[0].cpu().numpy())
        print(json.dumps({"progress": f"samples {m0 + m - a}/{b - a}", "t_s": round(time.perf_counter() - t0, 1)}),
              flush=True)
    phi = np.concatenate(parts, axis=1)
    np.save(args.out, phi)
    print(json.dumps({"saved": args.out, "shape": list(phi.shape), "wall_s": time.perf_counter() - t0,
                      "propagations_per_s": phi.size / (time.perf_counter() - t0)}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--samples-per-step", type=int, default=4)
    ap.add_argument("--profile-steps", type=int, default=2,
                    help="extra steps with HIP events around the term launches (roofline)")
    ap.add_argument("--no-headline", action="store_true",
                    help="skip the measured sweeps to eps <= 1e-3 (plain FP64, FP32 + design, FP32 + control variate)")
    ap.add_argument("--headline-legs", default="fp64,design,cv",
                    help="which measured sweeps to run (comma-separated subset of fp64,design,cv)")
    ap.add_argument("--fields", type=int, default=64)
    ap.add_argument("--precision", type=int, default=32, choices=[32, 64])
    ap.add_argument("--rdt", type=float, default=0.0)
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuner (r*dt, XCD order, tile kernel, path, axis order by timed probes) "
                         "and time the library defaults")
    ap.add_argument("--workspace-gb", type=float, default=0.0,
                    help="device workspace cap per call (bounds how many wavepackets run together)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="only run the streaming probes over buffers of this many GiB (ceilings; calibrates counters)")
    ap.add_argument("--workload", default="sweep",
                    choices=["sweep", "tiny", "batched", "large", "paper", "trace", "sampling", "arnoldi",
                             "histogram", "convergence", "batched-classes", "mlp"])
    ap.add_argument("--trace-n", type=int, default=10, help="trace workload: nuclei of the batched system used")
    ap.add_argument("--field-group", type=int, default=0,
                    help="large/paper workloads: fields per call, with a progress line after each (0: all)")
    ap.add_argument("--no-profile-call", action="store_true",
                    help="large/paper workloads: skip the extra profiled call")
    ap.add_argument("--stride", type=int, default=8, help="batched workload: take every stride-th system")
    ap.add_argument("--max-n", type=int, default=12, help="batched workload: only systems with at most this many nuclei")
    ap.add_argument("--per-class", type=int, default=2, help="batched-classes workload: systems per size class")
    ap.add_argument("--class-t", type=float, default=1.0, help="batched-classes workload: horizon cut (us)")
    ap.add_argument("--xcd", default=None, choices=["local", "spread"],
                    help="batched-classes and other workloads: force the XCD workgroup order")
    ap.add_argument("--cv", action="store_true",
                    help="headline comparison: FP32 + learned control variate vs plain FP64 sweep wall time")
    ap.add_argument("--cv-train", type=int, default=3072, help="training yields (one direction each)")
    ap.add_argument("--cv-epochs", type=int, default=200)
    ap.add_argument("--cv-no-augment", action="store_true", help="train without the field-axis rotations")
    ap.add_argument("--cv-quad", type=int, default=65536, help="samples for the mean of the network")
    ap.add_argument("--cv-eval", type=int, default=128, help="evaluation samples (pilot)")
    ap.add_argument("--sampling-system", default="sweep", choices=["sweep", "paper"],
                    help="sampling workload: the sweep system (0, 2.5, 10 mT) or the Sec. IV model (1, 3.5 mT)")
    ap.add_argument("--samplers", default="coherent,jz,antithetic,oa3,oa2",
                    help="sampling workload: comma-separated samplers, the first is the reference")
    ap.add_argument("--sampler", type=int, default=0, choices=[0, 3, 4, 5],
                    help="tiny/batched/large/paper workloads: rp_sample mode of the directions (0 plain; "
                         "3-5 sign-flip designs, errors from group means)")
    ap.add_argument("--design", action="store_true",
                    help="sweep to eps <= 1e-3 with sign-flip design sampling (FP32) against plain FP64")
    ap.add_argument("--design-mode", type=int, default=5, choices=[3, 4, 5], help="rp_sample design mode")
    ap.add_argument("--design-groups", type=int, default=8, help="design groups per field to start with")
    ap.add_argument("--design-workload", default="cv", choices=["cv", "sweep"],
                    help="--design on the control-variate workload (32 fields) or the bench sweep (64 fields)")
    ap.add_argument("--sample-range", default="0:100", help="convergence workload: samples a:b of this call")
    ap.add_argument("--out", default="convergence.npy", help="convergence workload: where to save the yields")
    ap.add_argument("--combine", default="", help="convergence workload: comma-separated saved files to combine")
    ap.add_argument("--summarize", default="",
                    help="print a per-kernel summary of a rocprofv3 CSV directory and exit")
    args = ap.parse_args()
    if args.summarize:
        for k, v in sorted(summarize(args.summarize).items(), key=lambda kv: -kv[1].get("pct", 0)):
            print(json.dumps({"kernel": k, **v}))
        return
    if args.design:
        design_headline(args)
        return
    if args.cv:
        cv_headline(args)
        return
    if args.workload == "trace":
        trace_vs_mc(args)
        return
    if args.workload == "sampling":
        sampling_variance(args)
        return
    if args.workload == "arnoldi":
        arnoldi_ablation(args)
        return
    if args.workload == "histogram":
        histogram(args)
        return
    if args.workload == "convergence":
        convergence(args)
        return
    if args.workload == "batched-classes":
        batched_classes(args)
        return
    if args.workload == "mlp":
        mlp_timing(args)
        return
    if args.workload != "sweep":
        other_workload(args)
        return
    if args.copy_probe > 0:
        # hand-written 16-byte streaming kernels (rp_probe_stream): GB/s per pattern; under
        # rocprofv3 --pmc the copy launches (k_stream<0>, GiB read and written) calibrate the counters
        from paper_1612_09517_amd import rp
        n = int(args.copy_probe * 2 ** 30)
        print(json.dumps({"probe_bytes": n, "GBps": rp.probe_stream(n, reps=5)}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU only (--gpus 1); a multi-GPU sweep would "
                                   "shard jobs across GPUs with one final all-reduce of per-field sums"}))
        sys.exit(2)

    import torch
    from paper_1612_09517_amd import rp, workloads

    w = workloads.sweep_c2(n_fields=args.fields)
    s = w.systems[0]
    Mb = args.samples_per_step
    B = w.fields_mT
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t_start = time.perf_counter()

    def say(msg):
        print(json.dumps({"progress": msg, "t_s": round(time.perf_counter() - t_start, 1)}), file=sys.stderr,
              flush=True)

    tuned = {"rdt": args.rdt, "xcd": None}
    t_tune = 0.0
    if not args.no_autotune:
        import tempfile
        from paper_1612_09517_amd import autotune
        t0 = time.perf_counter()
        with tempfile.TemporaryDirectory() as td:     # probe afresh on this GPU
            tuned = autotune.tune(s, B[0], precision=args.precision, cache=os.path.join(td, "tune.json"))
        t_tune = time.perf_counter() - t0
        say(f"autotuned in {t_tune:.1f} s: {tuned}")

    def step(i, profile=False):
        ang = rp.sample(s, w.seed, Mb, first=i * Mb)
        phi = rp.propagate(s, B, ang, Mb, precision=args.precision, profile=profile,
                           workspace_bytes=int(args.workspace_gb * 2 ** 30), **tuned)
        mean, err = rp.yield_stats(phi[0])
        return phi, mean, err

    # Throughput: the production path (captured step graphs, no events), K timed steps.
    for i in range(args.warmup):
        step(1000 + i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    props = args.steps * Mb * B.shape[1]
    value = props / elapsed if args.steps else 0.0
    say(f"throughput: {value:.1f} propagations/s")
    # Roofline: one more step with HIP events around the term launches (on the call's stream).
    prof = {"term_ms": 0.0, "term_launches": 0.0, "elements": 0.0, "quad_ms": 0.0, "total_ms": 0.0}
    for i in range(args.profile_steps):
        step(args.steps + i, profile=True)
        p = rp.profile_last()
        for k in prof:
            prof[k] += p[k]
        bpe = p["bytes_per_element"]
        nterms = p["terms_per_step"]
    achieved = prof["elements"] * bpe / (prof["term_ms"] * 1e-3) / 1e9
    ceil = rp.probe_stream(1 << 30, reps=5)
    say(f"streaming ceilings (GB/s): {ceil}")
    rec = {
        "metric": "sweep wall time at sigma(Phi_S)<=1e-3 vs plain FP64 MC; H.psi HBM GB/s vs peak",
        "value": value,
        "unit": "propagations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3 if args.steps else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == 32 else "f64",
        "data": "synthetic",
        "config": {"workload": "c2_7+7_Z16384: 7+7 spin-1/2, a~U(-1,1) mT, kS=2, kT=0.5 /us, T=20 us, "
                               f"{B.shape[1]} fields 0..10 mT x {Mb} samples per step",
                   "Z": s.Z, "dim": s.dim, "fields": int(B.shape[1]), "samples_per_step": Mb,
                   "precision": f"complex-FP{args.precision} state, FP64 coefficients and reductions",
                   "launch": {**{k: v for k, v in tuned.items() if v is not None},
                              "autotuned": not args.no_autotune, "autotune_s": round(t_tune, 2),
                              "graphs": True}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS,
                     "traffic": measured_traffic(args.precision, int(nterms),
                                                 prof["elements"] / max(prof["term_launches"], 1)),
                     "algorithmic_bytes_per_launch": prof["elements"] * bpe / max(prof["term_launches"], 1),
                     "kernel": ("k_cheb_pair (Chebyshev term on index pairs"
                                if args.precision == 32 and not tuned.get("term_scalar") else
                                "k_cheb_tile (Chebyshev term") + "; three launch variants)",
                     "avg_launch_us": prof["term_ms"] * 1e3 / max(prof["term_launches"], 1),
                     "bytes_per_element_term": bpe, "terms_per_step": nterms,
                     "profiled_steps": args.profile_steps,
                     "measured_ceilings_GBps": {k: round(v, 1) for k, v in ceil.items()},
                     "frac_of_read2_write1": achieved / ceil["read2_write1"],
                     "term_time_frac": prof["term_ms"] / max(prof["total_ms"], 1e-9),
                     "quad_time_frac": prof["quad_ms"] / max(prof["total_ms"], 1e-9)},
    }
    if not args.no_headline:
        rec["sweep_to_eps"] = headline_sweeps(args, say)
    if not args.no_cpu_baseline:
        say("cpu baseline")
        rec["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
