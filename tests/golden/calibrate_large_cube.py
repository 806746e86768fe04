"""Find the displacement amplitude of the 100^3 large_cube workload for which
30% of the Gauss points are plastic at the trial state (f_tr > 0).

Calls only the CPU oracle (trial yield test) and the seeded input generator.
Prints the amplitude; its value is stored as synth.LARGE_CUBE_AMPLITUDE.
Run:  python tests/golden/calibrate_large_cube.py
"""
import os
import sys

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", ".."))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2606_17390_amd import synth  # noqa: E402


def plastic_fraction(p, amp):
    flag = oracle.trial_yield(p.X, p.conn, p.prm, amp * p.meta["shape"], p.hist_n)
    return float(flag.mean())


def main(target=0.30, n=100):
    p = synth.large_cube(n=n, amplitude=1.0)
    lo, hi = 0.0, 0.05
    for _ in range(30):
        mid = 0.5 * (lo + hi)
        f = plastic_fraction(p, mid)
        print(f"amplitude {mid:.10g}  plastic fraction {f:.5f}", flush=True)
        if f < target:
            lo = mid
        else:
            hi = mid
        if abs(f - target) < 0.001:
            break
    print("AMPLITUDE", mid)


if __name__ == "__main__":
    main()
