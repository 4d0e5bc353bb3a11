"""Writes the stored expected values under tests/golden/ that come from the
oracle (not from the paper): the SHA-256 of the arrival times of the 3D
512x512x256 layered model (the benchmark's timed solve), computed by the CPU
oracle's sequential fast marching.  Calls only `oracle` and the seeded input
generators.

    python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "layered_512x512x256_seed2.json")


def times_sha256(t) -> str:
    import numpy as np
    return hashlib.sha256(np.ascontiguousarray(t, dtype="<f8").tobytes()).hexdigest()


def layered_golden() -> dict:
    import oracle
    import workloads as W
    p = W.layered_3d(512, 512, 256, h=10.0, seed=2)
    t = oracle.fmm(p.field, p.h, p.src)
    return {"workload": "3D 512x512x256 layered+noise speed, h=10 m, seed 2, source at the surface centre",
            "input_sha256_16": p.sha256(), "times_sha256": times_sha256(t),
            "times_max": float(t.max()), "made_by": "tests/golden/make_golden.py (oracle.fmm)"}


if __name__ == "__main__":
    g = layered_golden()
    with open(OUT, "w") as f:
        json.dump(g, f, indent=1)
        f.write("\n")
    print(json.dumps(g))
