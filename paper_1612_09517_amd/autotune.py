"""Launch-parameter autotuner for rp_propagate, with an on-disk cache.

For a system shape it times short probes of the real call -- the same system with a horizon
shortened to 12 Chebyshev steps of the candidate's own length at the highest field, three of
its fields and as many samples as fill the job queue -- and keeps the candidate with the lowest
time per simulated microsecond per wavepacket.  The candidates are
searched one dimension at a time, starting from the library's defaults:

1. the step length r*dt (RDT);
2. the workgroup order: each wavepacket's tiles on one XCD, or every XCD on few wavepackets;
3. the tile kernel: two nuclear indices per thread with 16-byte accesses, or one index per
   thread (complex FP32 with at least 8 leading spin-1/2 nuclei; otherwise only one exists);
4. the path of a small state (at most 1024 complex-FP32 or 512 FP64 nuclear states): the whole
   propagation in one workgroup's LDS, or the tiled kernels;
5. the axis order of a system that mixes spins: spin-1/2 nuclei on the fastest axes (tile
   kernels), or the higher spins there (mixed-radix kernel).

Results are cached as JSON keyed by GPU name, precision and system shape (spins per radical,
exchange, rate difference and the rounded spectral width), so later calls reuse them without
probing.  The returned dict holds keyword arguments of rp.propagate.
"""
import dataclasses
import json
import os
import time

import numpy as np

from . import rp

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "rpmc", "autotune.json")
RDT = (60.0, 80.0, 100.0, 120.0, 130.0, 140.0, 150.0, 160.0)
XCD = ("local", "spread")
RESIDENT_MAX = {32: 1024, 64: 512}


def _key(system, precision, r_max):
    import torch
    gpu = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    spins = (tuple(sorted(system.two_I[:system.n1])), tuple(sorted(system.two_I[system.n1:])))
    return (f"{gpu}|fp{precision}|{spins}|J={system.J_mT != 0}|dk={abs(system.kS - system.kT):.2g}"
            f"|r~{r_max:.2g}|v4")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def probe_horizon(system, rdt, r_max, steps=12):
    """Horizon of a probe for step length `rdt`: `steps` whole steps at the highest field (whose
    spectral half-width is r_max), or the system's own horizon if that is shorter."""
    return min(system.T_us, steps * rdt / r_max)


def dimensions(system, precision):
    """The categorical dimensions that apply to this system, with their candidate values (the
    library default first)."""
    dims = [("xcd", XCD)]
    leading_half = 0
    for t in sorted(system.two_I):
        if t != 1:
            break
        leading_half += 1
    if precision == 32 and leading_half >= 8:
        dims.append(("term_scalar", (False, True)))
    if system.Z <= RESIDENT_MAX[precision]:
        dims.append(("tiled", (False, True)))
    if len(set(system.two_I)) > 1:
        dims.append(("axes_high_first", (False, True)))
    return dims


def tune(system, fields_mT, precision=32, samples=8, cache=None, force=False, seed=12345, repeats=3):
    """Best rp.propagate keyword arguments for `system` over `fields_mT`: 'rdt', 'xcd' and, where
    they apply, 'term_scalar', 'tiled' and 'axes_high_first'.  Probes only on a cache miss.

    A probe is sized like production work: at least `samples` samples, and enough wavepackets
    (about 2^21 nuclear states in all, at most 256) to fill the job queue's slots as a sweep
    does, over a horizon of 12 of the candidate's steps at the highest field, so that rounding
    the step counts up costs every r*dt the same."""
    import torch
    cache = cache or os.environ.get("RPMC_AUTOTUNE_CACHE", DEFAULT_CACHE)
    B = np.asarray(fields_mT, np.float64).reshape(-1)
    r_max = max(rp.plan_field(system, float(b), precision=precision)["r"] for b in (B.min(), B.max()))
    key = _key(system, precision, r_max)
    db = _load(cache)
    if key in db and not force:
        return dict(db[key]["best"])
    Bp = np.unique(np.quantile(B, [0.0, 0.5, 1.0]))[None, :]
    jobs = int(np.clip((1 << 21) // max(system.Z, 1), 8, 256))
    samples = max(samples, -(-jobs // Bp.shape[1]))
    ang = rp.sample(system, seed, samples)
    results = []

    def timed(cand):
        # Each candidate's horizon is a whole number (12) of its own steps at the highest
        # field, so that rounding the step count up costs every candidate the same.
        T_probe = probe_horizon(system, cand["rdt"], r_max)
        probe = dataclasses.replace(system, T_us=T_probe)
        kw = dict(precision=precision, **cand)
        rp.propagate(probe, Bp, ang, samples, **kw)
        torch.cuda.synchronize()
        best = np.inf
        for _ in range(repeats):
            t0 = time.perf_counter()
            rp.propagate(probe, Bp, ang, samples, **kw)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        v = best / (T_probe * samples * Bp.shape[1])
        results.append({**cand, "s_per_us_job": v})
        return v

    cur = {"rdt": 100.0, "xcd": None}
    for name, values in dimensions(system, precision):
        cur[name] = values[0]
    cur["xcd"] = "local" if 4 * system.Z * (4 if precision == 32 else 8) * 2 <= (32 << 20) else "spread"
    scores = {rdt: timed({**cur, "rdt": rdt}) for rdt in RDT}
    cur["rdt"] = min(scores, key=scores.get)
    best_v = scores[cur["rdt"]]
    for name, values in dimensions(system, precision):
        for v in values:
            if v == cur[name]:
                continue
            t = timed({**cur, name: v})
            if t < best_v:
                best_v, cur[name] = t, v
    db[key] = {"best": cur, "probes": results}
    os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
    tmp = cache + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1)
    os.replace(tmp, cache)
    return dict(cur)
