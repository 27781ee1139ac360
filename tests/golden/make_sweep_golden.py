"""Writes sweep_golden.json: exact single-wavepacket yields of the 7+7 spin-1/2 sweep
workload (Z = 2^14, T = 20 us) for 8 of its 64 fields (every ninth, 0 and 10 mT included; the
10 mT field has the most Chebyshev steps) x samples 0..3, from the oracle's sparse
augmented-system route only (one process per yield).  Run from the repository root:

    python tests/golden/make_sweep_golden.py [--procs 6]
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

FIELD_INDEX = [0, 9, 18, 27, 36, 45, 54, 63]
SAMPLES = [0, 1, 2, 3]


def one(task):
    B, i = task
    w = workloads.sweep_c2()
    s = w.systems[0]
    sp = large.SparseSystem((s.n1, s.n2), s.two_I, s.a_mT, J_mT=s.J_mT, kS=s.kS, kT=s.kT, gamma=s.gamma)
    ang = philox.sample_angles(w.seed, 0, max(SAMPLES) + 1, s.N)
    t0 = time.time()
    phi, _ = large.yield_augmented(sp, B, s.T_us, sp.wavepacket(ang[i]), tau=1.0)
    print(f"B={B!r} sample={i} phi={phi!r} ({time.time() - t0:.0f} s)", flush=True)
    return B, i, phi


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=6)
    args = ap.parse_args()
    w = workloads.sweep_c2()
    s = w.systems[0]
    fields = [float(w.fields_mT[0][k]) for k in FIELD_INDEX]
    tasks = [(B, i) for B in reversed(fields) for i in SAMPLES]
    with Pool(args.procs) as pool:
        res = pool.map(one, tasks, chunksize=1)
    out = {"workload": w.name, "seed": w.seed, "stream": 0, "T_us": s.T_us, "fields_mT": fields,
           "samples": SAMPLES, "phi": {f"{B}:{i}": phi for B, i, phi in res},
           "source": "oracle.large.yield_augmented (scipy expm_multiply), tau = 1 us"}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "sweep_golden.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
