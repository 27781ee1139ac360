"""Launch-parameter autotuner for rp_propagate, with an on-disk cache.

For a system shape it times short probes of the real call -- the same system with a horizon
shortened to a few Chebyshev steps at its highest field, a few fields and samples -- over the
candidate step lengths r*dt and workgroup orders (one XCD per wavepacket, or all XCDs on
few wavepackets), and keeps the one with the lowest time per simulated microsecond per
wavepacket.  Results are cached as JSON keyed by GPU name, precision and system shape
(spins per radical and the rounded spectral width), so later calls reuse them without
probing.
"""
import dataclasses
import json
import os
import time

import numpy as np

from . import rp

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "rpmc", "autotune.json")
RDT = (60.0, 80.0, 100.0, 120.0, 160.0)
XCD = ("local", "spread")


def _key(system, precision, r_max):
    import torch
    gpu = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    spins = (tuple(sorted(system.two_I[:system.n1])), tuple(sorted(system.two_I[system.n1:])))
    return f"{gpu}|fp{precision}|{spins}|J={system.J_mT != 0}|dk={abs(system.kS - system.kT):.2g}|r~{r_max:.2g}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(system, fields_mT, precision=32, samples=8, cache=None, force=False, seed=12345):
    """Best {'rdt', 'xcd'} for propagating `system` over `fields_mT`; probes only on a cache miss."""
    import torch
    cache = cache or os.environ.get("RPMC_AUTOTUNE_CACHE", DEFAULT_CACHE)
    B = np.asarray(fields_mT, np.float64).reshape(-1)
    r_max = max(rp.plan_field(system, float(b), precision=precision)["r"] for b in (B.min(), B.max()))
    key = _key(system, precision, r_max)
    db = _load(cache)
    if key in db and not force:
        return dict(db[key]["best"])
    # Probe: horizon of about six steps at r*dt = 80 for the highest field.
    T_probe = min(system.T_us, 6 * 80.0 / r_max)
    probe = dataclasses.replace(system, T_us=T_probe)
    Bp = np.unique(np.quantile(B, [0.0, 0.5, 1.0]))[None, :]
    ang = rp.sample(probe, seed, samples)
    results = []
    for rdt in RDT:
        for xcd in XCD:
            kw = dict(precision=precision, rdt=rdt, xcd=xcd, tiled=True)
            rp.propagate(probe, Bp, ang, samples, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rp.propagate(probe, Bp, ang, samples, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            results.append({"rdt": rdt, "xcd": xcd, "s_per_us_job": dt / (T_probe * samples * Bp.shape[1])})
    best = min(results, key=lambda r: r["s_per_us_job"])
    db[key] = {"best": {"rdt": best["rdt"], "xcd": best["xcd"]}, "probes": results}
    os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
    tmp = cache + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1)
    os.replace(tmp, cache)
    return dict(db[key]["best"])
