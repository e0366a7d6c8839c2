"""Write oracle values of 64 sampled rows of the dense operator applied to a
seeded density, for the N = 32768 near-grazing Wood workload
(tests/golden/rows_grazing32768.json).

Calls only the CPU oracle (dense direct operator rows); rows are computed in
parallel worker processes.  The rows are 0, N-1 and 62 seeded random rows; the
density is workloads.random_density(N, 5).
Usage: python tests/golden/gen_rows_grazing32768.py
"""
import json
import os
import sys
import time
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import dense  # noqa: E402

N = 32768
_DISC = None
_MU = None


def _init():
    global _DISC, _MU
    _DISC = dense.Discretization(W.config_grazing_wood(N))
    _MU = W.random_density(N, 5)


def _row(r):
    return r, complex(dense.operator_rows(_DISC, np.array([r]))[0] @ _MU)


def main(procs=8):
    rng = np.random.default_rng(W.SEED_BASE + 64)
    rows = sorted(set([0, N - 1] + [int(v) for v in rng.choice(np.arange(1, N - 1), 62, replace=False)]))
    t0 = time.time()
    with Pool(procs, initializer=_init) as pool:
        vals = dict(pool.map(_row, rows))
    wl = W.config_grazing_wood(N)
    disc = dense.Discretization(wl)
    out = {
        "workload": wl.name, "N": N,
        "n_a": int(disc.n_a), "density": "workloads.random_density(N, 5)", "rows": rows,
        "y_re": [vals[r].real for r in rows], "y_im": [vals[r].imag for r in rows],
        "oracle_seconds": time.time() - t0, "oracle_processes": procs,
        "source": "tests/golden/gen_rows_grazing32768.py (CPU oracle: dense operator rows)",
    }
    with open(os.path.join(HERE, "rows_grazing32768.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print("rows", len(rows), "%.1fs" % out["oracle_seconds"])


if __name__ == "__main__":
    main()
