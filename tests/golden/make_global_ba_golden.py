"""Write the float64 oracle's result for the 1000-keyframe global BA.

    python tests/golden/make_global_ba_golden.py

Calls only the oracle (and the seeded scene generator).  Output:
tests/golden/global_ba_oracle.npz with the final poses [1000,7], inverse
depths [96000] and the per-iteration cost.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ba64  # noqa: E402
from scenes import make_config  # noqa: E402


def main():
    s = make_config(2)
    t0 = time.time()
    P, D, rep = ba64.solve_scene(s)
    print(f"oracle global BA: {time.time() - t0:.1f}s cost {rep.cost} invalid {rep.n_invalid}", flush=True)
    np.savez_compressed(os.path.join(HERE, "global_ba_oracle.npz"), poses=P, inv_depth=D,
                        cost=np.array(rep.cost), n_invalid=np.array(rep.n_invalid))


if __name__ == "__main__":
    main()
