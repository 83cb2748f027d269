"""Writes the stored expected values used by the full-size parity tests and
by the benchmark's accuracy checks.

Calls only the CPU oracle (oracle/) and the seeded generators.
- bump_grid1024_s2_ich.npz: the exact field of the 1024^2 bump grid from
  vertex 0 (several minutes of single-core ICH, too long for a test), every
  vertex, with the run's window counts and the mean edge length (the floor
  of the relative error);
- icosphere7_ich.npz: the exact fields of the bumpy icosphere with 327,680
  faces from two seeded vertices, with the mean edge length.

    python tests/golden/make_golden.py [bump_grid|icosphere]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_1305_1293_amd import meshgen as G  # noqa: E402


def icosphere():
    m = G.config_mesh(2)
    srcs = np.random.default_rng(7).choice(m.nv, size=2, replace=False).astype(np.int64)
    dist = np.stack([O.ich(m, [int(s)])[0] for s in srcs])
    hbar = float(O.lengths(m).mean())
    np.savez_compressed(os.path.join(HERE, "icosphere7_ich.npz"), dist=dist, sources=srcs, nv=m.nv, nf=m.nf,
                        mean_edge=hbar)
    print("wrote", dist.shape, "distances from", srcs.tolist())


def bump_grid():
    m = G.config_mesh(3)
    s = m.meta["source"]
    t = time.time()
    d, st = O.ich(m, [s])
    el = time.time() - t
    hbar = float(O.lengths(m).mean())
    np.savez_compressed(os.path.join(HERE, "bump_grid1024_s2_ich.npz"), dist=d, source=s, nv=m.nv, nf=m.nf,
                        mean_edge=hbar, created=st["created"], processed=st["processed"], ich_seconds=el)
    print("wrote", m.nv, "distances; ich seconds", round(el, 1), st)


def main():
    O.build()
    which = sys.argv[1:] or ["bump_grid", "icosphere"]
    if "bump_grid" in which:
        bump_grid()
    if "icosphere" in which:
        icosphere()


if __name__ == "__main__":
    main()
