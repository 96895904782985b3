"""Writes c3_adjoint_sample.npz: the oracle's sensitivities (discrete adjoint, SuperLU per
shift) of the full 64x64x32 workload for its first source and first two receivers, at
4096 seeded cells, with each (source, receiver, time) map's largest magnitude and 2-norm.
Calls only oracle/ and workloads/ (the seeded inputs).  About 24 factorisations of the
131,072-cell operator: several minutes on 8 cores.

    python tests/golden/make_c3_adjoint_sample.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

if __name__ == "__main__":
    import workloads as wl
    from oracle.jacobian import jacobian

    p = wl.make_problem("C3")
    src, rec = p.sources[:1], p.receivers[:2]
    t0 = time.time()
    JK, JS = jacobian(p.n, p.h, p.kappa, p.S, src, rec, p.times, p.nz_contour, q=p.q, bc=p.bc,
                      workers=min(8, os.cpu_count() or 1), ndim=p.ndim)
    cells = np.sort(np.random.default_rng(3030).choice(p.N, size=4096, replace=False))
    np.savez_compressed(os.path.join(HERE, "c3_adjoint_sample.npz"), cells=cells,
                        dlnK=JK[..., cells], dlnS=JS[..., cells],
                        dlnK_max=np.abs(JK).max(axis=-1), dlnS_max=np.abs(JS).max(axis=-1),
                        dlnK_norm=np.linalg.norm(JK, axis=-1), dlnS_norm=np.linalg.norm(JS, axis=-1),
                        sources=src, receivers=rec)
    print(f"wrote c3_adjoint_sample.npz ({time.time() - t0:.0f} s)")
