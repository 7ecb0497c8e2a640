"""Write the oracle's smooth sum of the batched 256x256-box workload at its
4,096 sampled targets x 16 densities (tests/golden/c3_sample_smooth.npy).

The direct sum over 4,194,304 nodes at 4,096 targets and 16 densities takes
minutes on a host, so the GPU parity test and the benchmark read the stored
values and add the correction rows (a cheap oracle call) for whichever
correction matrix they use.  The values come only from the CPU oracle
(oracle/direct.c) on the seeded inputs of vp_workloads; the parity test
re-evaluates a subset of the rows live and checks that the file still
matches.

Run from the repository root:  python tests/golden/make_c3_reference.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import direct  # noqa: E402
from vp_workloads import generators as gen  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "c3_sample_smooth.npy")


def main():
    wl = gen.config3()
    t0 = time.perf_counter()
    ref = direct.smooth(wl.x, wl.y, wl.w, wl.f, tidx=wl.sample)
    dt = time.perf_counter() - t0
    assert ref.shape == (wl.nbatch, wl.sample.size)
    np.save(OUT, ref)
    print(f"wrote {OUT}: {ref.shape} in {dt:.0f} s on {direct.num_threads()} threads")


if __name__ == "__main__":
    main()
