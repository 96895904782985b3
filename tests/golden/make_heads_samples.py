"""Writes the oracle's heads (SuperLU per shift, contour sum) for the full-size 3D
workloads that the GPU parity tests compare against element by element:

    c3_heads.npz       64x64x32 workload: all 25 sources x 48 receivers x both times
    c5_32c_heads.npz   the 32^3 problem of the six-grid batch: 16 sources x 32 receivers x both times

Calls only oracle/ and workloads/ (the seeded inputs).  The 64x64x32 operator takes
24 factorisations of about 1.5 minutes each on one core (a few minutes on 8 cores).

    python tests/golden/make_heads_samples.py [c3] [c5_32c]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

SAMPLES = {"c3": ("C3", "c3_heads.npz"), "c5_32c": ("C5_32c", "c5_32c_heads.npz")}

if __name__ == "__main__":
    import workloads as wl
    from oracle.heads import heads_problem

    which = sys.argv[1:] or list(SAMPLES)
    for key in which:
        name, fname = SAMPLES[key]
        p = wl.make_problem(name)
        t0 = time.time()
        phi = heads_problem(p, workers=min(8, os.cpu_count() or 1))
        np.savez_compressed(os.path.join(HERE, fname), heads=phi, sources=p.sources, receivers=p.receivers,
                            times=p.times, nz=p.nz_contour)
        print(f"wrote {fname} {phi.shape} ({time.time() - t0:.0f} s)", flush=True)
