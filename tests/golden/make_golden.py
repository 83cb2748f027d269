"""Writes the stored expected values used by the full-size parity tests.

Calls only the CPU oracle (oracle/) and the seeded generators. The exact
field of the 1024^2 bump grid from vertex 0 takes several minutes of
single-core ICH, too long for a test, so it is stored once, every vertex,
with the run's window counts and the mean edge length (the floor of the
relative error):

    python tests/golden/make_golden.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_1305_1293_amd import meshgen as G  # noqa: E402


def main():
    O.build()
    m = G.config_mesh(3)
    s = m.meta["source"]
    t = time.time()
    d, st = O.ich(m, [s])
    el = time.time() - t
    hbar = float(O.lengths(m).mean())
    np.savez_compressed(os.path.join(HERE, "bump_grid1024_s2_ich.npz"), dist=d, source=s, nv=m.nv, nf=m.nf,
                        mean_edge=hbar, created=st["created"], processed=st["processed"], ich_seconds=el)
    print("wrote", m.nv, "distances; ich seconds", round(el, 1), st)


if __name__ == "__main__":
    main()
