#!/usr/bin/env python3
"""Write the oracle's reference rows of the large single geometry.

Sphere of radius 8 wavelengths (icosphere of frequency 96: 184 320
triangles, 276 480 RWG functions, 7-level octree with quarter-wavelength
leaves), 16 right-hand sides with real and imaginary parts i.i.d. N(0,1)
(seed 4), op C (the BI block of eqs. 43-46).  The sample is 2 000 RWG rows
drawn without replacement by numpy's PCG64 with seed 40; both halves of each
row (J-tested and M-tested) are stored.

Output `sphere_r8_rows_2000.npz`:
  rows   (2000,) int32, sorted RWG indices;
  near   (4000, 16) complex64: the part of pairs whose leaf boxes are adjacent;
  level2 ... level6 (4000, 16) complex64: the part of pairs that are first
         well separated at that octree level (the pairs the MLFMA translates
         there);
  rows [0, 2000) of each array are the J-tested rows, [2000, 4000) the
  M-tested rows, in the order of `rows`.
Complex64 storage keeps the file small; its rounding (6e-8 relative) is far
below the 1e-3 tolerance the values are used at.

Only the oracle and the seeded input generators are called.  Runs about
15 minutes on 8 cores.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth   # noqa: E402

OUT = os.path.join(HERE, "sphere_r8_rows_2000.npz")
NROWS, NRHS, X_SEED, ROW_SEED = 2000, 16, 4, 40


def sample_rows(n_rwg):
    return np.sort(np.random.default_rng(ROW_SEED).choice(n_rwg, NROWS, replace=False)).astype(np.int32)


def main():
    v, t, spec = synth.workload("sphere_r8")
    N = 3 * len(t) // 2
    x = synth.gaussian_coeffs(2 * N, NRHS, X_SEED)
    rows = sample_rows(N)
    out = {"rows": rows}
    t0 = time.time()
    chunk = 100
    parts = []
    for c in range(0, NROWS, chunk):
        r = rows[c:c + chunk]
        y = oracle.matvec(v, t, 2 * np.pi, x, op=oracle.OP_C, rows=r, leaf=spec["leaf"], classes=True)
        parts.append(y)
        print("rows %d-%d done, %.0f s" % (c, c + len(r), time.time() - t0), flush=True)
    ncls = parts[0].shape[0]
    for cls in [0] + list(range(2, ncls)):
        j = np.concatenate([p[cls][:p.shape[1] // 2] for p in parts])
        m = np.concatenate([p[cls][p.shape[1] // 2:] for p in parts])
        out["near" if cls == 0 else "level%d" % cls] = np.concatenate([j, m]).astype(np.complex64)
    np.savez(OUT, **out)
    print("wrote %s (%.0f s, %d threads)" % (OUT, time.time() - t0, oracle.threads()), flush=True)


if __name__ == "__main__":
    main()
