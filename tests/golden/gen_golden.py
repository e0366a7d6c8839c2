"""Write oracle reference efficiencies for the random-surface workloads at a
reduced node count (tests/golden/*.json).

Calls only the CPU oracle (dense direct operator, LU solve, Rayleigh
efficiencies); the operator rows are assembled in parallel worker processes.
Usage: python tests/golden/gen_golden.py [name ...]
  names: grazing4096, wood30_4096, grazing8192, grazing16384
The two larger grazing cases pin the benched N = 32768 workload's efficiencies
at node counts where the oracle itself has converged; the N = 16384 file also
records its distance to the N = 8192 result (self-convergence in N).
Environment: GOLDEN_PROCS (worker processes, default 8).
"""
import json
import math
import os
import sys
import time
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import dense, rayleigh  # noqa: E402

CASES = {
    "grazing4096": lambda: W.config_grazing_wood(4096),
    "wood30_4096": lambda: W.config_random_double_wood(4096),
    "grazing8192": lambda: W.config_grazing_wood(8192),
    "grazing16384": lambda: W.config_grazing_wood(16384),
}
# a finer-N case records its distance to the coarser one
COARSER = {"grazing16384": "grazing8192", "grazing8192": "grazing4096"}

_DISC = None


def _init(name):
    global _DISC
    _DISC = dense.Discretization(CASES[name]())


def _rows(r):
    return r, dense.operator_rows(_DISC, np.arange(r[0], r[1]))


def run(name, procs=8, block=16):
    wl = CASES[name]()
    disc = dense.Discretization(wl)
    t0 = time.time()
    M = np.empty((disc.N, disc.N), dtype=np.complex128)
    ranges = [(s, min(disc.N, s + block)) for s in range(0, disc.N, block)]
    with Pool(procs, initializer=_init, initargs=(name,)) as pool:
        for r, blk in pool.imap_unordered(_rows, ranges):
            M[r[0]:r[1]] = blk
    t_asm = time.time() - t0
    t1 = time.time()
    mu = np.linalg.solve(M, dense.rhs(disc))
    t_lu = time.time() - t1
    n, e, eps = rayleigh.efficiencies(disc, mu)
    out = {
        "workload": wl.name, "N": disc.N, "d": disc.d, "k": disc.k, "theta_deg": wl.theta_deg, "j": disc.j,
        "h": disc.h, "A_periods": disc.A, "c": disc.c, "n_a": disc.n_a, "gamma_frac": wl.gamma_frac,
        "eta": disc.eta, "U_eta": [int(u) for u in disc.U_eta], "orders": [int(v) for v in n],
        "efficiencies": [float(v) for v in e], "energy_error": float(eps),
        "oracle_assembly_seconds": t_asm, "oracle_lu_seconds": t_lu, "oracle_processes": procs,
        "source": "tests/golden/gen_golden.py (CPU oracle: dense operator, LU, Rayleigh efficiencies)",
    }
    coarse = COARSER.get(name)
    if coarse and os.path.exists(os.path.join(HERE, coarse + ".json")):
        with open(os.path.join(HERE, coarse + ".json")) as fh:
            G = json.load(fh)
        ec = dict(zip(G["orders"], G["efficiencies"]))
        out["self_convergence"] = {
            "coarser": coarse, "coarser_N": G["N"],
            "max_abs_efficiency_diff": max(abs(ec[int(o)] - float(v)) for o, v in zip(n, e)),
            "coarser_energy_error": G["energy_error"]}
    out["command"] = "python tests/golden/gen_golden.py " + name
    with open(os.path.join(HERE, name + ".json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(name, "N", disc.N, "assembly %.1fs" % t_asm, "eps %.3e" % eps, flush=True)


if __name__ == "__main__":
    for nm in (sys.argv[1:] or list(CASES)):
        run(nm, procs=int(os.environ.get("GOLDEN_PROCS", "8")))
