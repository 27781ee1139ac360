"""Writes batched_golden.json: exact single-wavepacket yields for a subset of the batched
workload of 256 uneven systems (N ~ U{8..18} spin-1/2, a ~ N(0, 0.7) mT, kS, kT log-uniform on
[0.1, 5] /us): the first system of every size N = 8..18 (Z = 2^8 .. 2^18), at the first and
last of its 32 fields (0 and 5 mT), samples 0 and 1 of its seeded directions.  Systems with
N <= 12 keep their own horizon T = min(10 / min(kS, kT), 20) us; the larger ones are cut to
T = 0.5 us (about ten Chebyshev steps) so that the oracle finishes.  Source: the oracle's sparse
augmented-system route only.  Run from the repository root:

    python tests/golden/make_batched_golden.py [--procs 6]
"""
import argparse
import json
import os
import sys
import time
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import large, philox                       # noqa: E402
from paper_1612_09517_amd import workloads             # noqa: E402

SAMPLES = [0, 1]
FIELD_INDEX = [0, 31]
T_CUT = 0.5


def subset():
    """(index in the batched set, horizon) of the first system of every N."""
    w = workloads.batched_c3()
    first = {}
    for i, s in enumerate(w.systems):
        first.setdefault(s.N, i)
    return [(first[N], w.systems[first[N]].T_us if N <= 12 else T_CUT) for N in sorted(first)]


def one(task):
    idx, T, B, i = task
    w = workloads.batched_c3()
    s = w.systems[idx]
    sp = large.SparseSystem((s.n1, s.n2), s.two_I, s.a_mT, J_mT=s.J_mT, kS=s.kS, kT=s.kT, gamma=s.gamma)
    ang = philox.sample_angles(w.seed, 0, max(SAMPLES) + 1, s.N)
    t0 = time.time()
    phi, _ = large.yield_augmented(sp, B, T, sp.wavepacket(ang[i]), tau=1.0)
    print(f"system {idx} (N={s.N}) T={T} B={B!r} sample={i} phi={phi!r} ({time.time() - t0:.0f} s)", flush=True)
    return idx, B, i, phi


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=6)
    args = ap.parse_args()
    w = workloads.batched_c3()
    sub = subset()
    tasks = []
    for idx, T in reversed(sub):
        for k in FIELD_INDEX:
            for i in SAMPLES:
                tasks.append((idx, T, float(w.fields_mT[idx][k]), i))
    with Pool(args.procs) as pool:
        res = pool.map(one, tasks, chunksize=1)
    out = {"workload": w.name, "seed": w.seed, "stream": 0, "samples": SAMPLES,
           "systems": [{"index": idx, "N": w.systems[idx].N, "T_us": T,
                        "fields_mT": [float(w.fields_mT[idx][k]) for k in FIELD_INDEX]} for idx, T in sub],
           "phi": {f"{idx}:{B}:{i}": phi for idx, B, i, phi in res},
           "source": "oracle.large.yield_augmented (scipy expm_multiply), tau = 1 us"}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "batched_golden.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
