"""Benchmark: GMRES solves/s and matvec Munknowns/s on the near-grazing Wood
workload (Gaussian random surface, d = 100 wavelengths, rms 1 wavelength,
89 degree incidence, k on a Wood anomaly, N = 32768, j = 8, A = 40 periods).

One step = one pass of the whole path: set_surface (Algorithm 2), GMRES solve
with the forward map (Algorithms 1 and 3) and the efficiencies.  Inputs are
synthetic (seeded surface coefficients).  Prints one JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode accel|dense]
                       [--N 32768] [--no-cpu-baseline]
       python bench.py --copy-probe   (one 256 MiB device copy, the reference
                                       kernel for scaling HBM traffic counters)
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BATCH = 8  # densities of the batched forward-map figure
METRIC = "GMRES solves/s and matvec Munknowns/s at N=32768, efficiency err ≤1e-6"
HBM_PEAK_GBS = 8000.0
TIMING_EVERY = 8


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", choices=["accel", "dense"], default=os.environ.get("SESM_BENCH_MODE", "accel"))
    ap.add_argument("--N", type=int, default=32768)
    # relative residual; the accelerated map is linear only up to its rounding
    # (~1e-12 relative), which puts the attainable true residual of this
    # workload near 4e-9, so the tolerance sits above that
    ap.add_argument("--tol", type=float, default=1e-8)
    # the other members of the Bloch class have |mu| / |b| ~ 600 (against ~120
    # for the benched incidence) and a true-residual floor near 2e-8
    ap.add_argument("--batch-tol", type=float, default=5e-8)
    ap.add_argument("--max-iter", type=int, default=3000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched-solve", action="store_true")  # e.g. under counter collection (many dispatches)
    # near-field work items per launch of the single-density forward map:
    # "auto" lets the library's tuner time candidate splits; otherwise the
    # thousandths of the items in the first launch, the merge + FFT launch and
    # the y-convolution launch (the inverse FFT takes the rest).  The default is
    # a split the tuner settles near on this workload: fixed, so the kernel
    # shapes (and the counter-measured traffic) are the same from run to run.
    ap.add_argument("--near-split", default="595,110,125")
    ap.add_argument("--no-mixed", action="store_true")  # skip the extra solves (mixed precision, hybrid tables, field)
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--workload", choices=["grazing", "c4", "c5"], default="grazing")
    ap.add_argument("--c4-angles", type=int, default=64)
    ap.add_argument("--c4-N", type=int, default=16384)
    ap.add_argument("--c4-max-iter", type=int, default=1000)
    return ap.parse_args()


def copy_probe():
    """One plain device copy of 256 MiB (after two warm-up copies): a kernel of
    known traffic (256 MiB read, 256 MiB written) for scaling FETCH_SIZE and
    WRITE_SIZE counter readings."""
    import torch
    n = (256 << 20) // 16
    a = torch.zeros(n, dtype=torch.complex128, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": 256 << 20, "copy_probe_bytes_written": 256 << 20, "launches": 3}))


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_local_apply_traffic_grazing_wood_N32768.md")


def library_sources_sha256():
    """Hash of the library sources (HIP files, internal headers, the C header)."""
    import glob
    import hashlib
    csrc = os.path.join(ROOT, "paper_1707_04950_amd", "csrc")
    files = sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.h")))
    files.append(os.path.join(ROOT, "include", "sesm.h"))
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, near_items=None):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when there is none for this kernel, the library changed since, or the
    near-field work items were split over the launches differently."""
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    fields = dict(l.strip().split(": ", 1) for l in text.splitlines() if l.strip().count(": ") == 1 and
                  l.strip().split(": ", 1)[0] in ("traffic_kernel", "traffic_bytes_per_launch", "library_sources_sha256",
                                                  "near_items_per_launch"))
    if fields.get("traffic_kernel") != kernel or fields.get("library_sources_sha256") != library_sources_sha256():
        return None
    if "near_items_per_launch" in fields and near_items is not None and \
            [int(v) for v in fields["near_items_per_launch"].split(",")] != list(near_items):
        return None
    return float(fields["traffic_bytes_per_launch"])


def cpu_baseline(wl, N, target_s=15.0):
    """Time the oracle (as is) on a bounded sample: dense operator rows of the
    same workload, assembled and applied on the host."""
    import numpy as np
    from oracle import dense
    import workloads as W
    disc = dense.Discretization(wl, N=N)
    mu = W.random_density(N, 1)
    rows_done, t0 = 0, time.perf_counter()
    r = 0
    while time.perf_counter() - t0 < target_s and rows_done < N:
        dense.matvec_rows(disc, mu, [r])
        rows_done += 1
        r = (r + 997) % N
    dt = time.perf_counter() - t0
    per_row = dt / rows_done
    return {
        "value": 1.0 / (per_row * N),
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": "%d dense operator rows of the N=%d workload in %.1f s; a solve needs all N rows "
                  "(assembly dominates), GMRES time not added" % (rows_done, N, dt),
        "matvec_munknowns_per_s": rows_done / dt / 1e6,
    }


GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")


def efficiency_vs_oracle(n, e):
    """max |e_n - e_n^oracle| against the finest stored oracle solution of the
    benched workload (dense operator, LU), with the oracle's own energy error
    and its distance to the next coarser N; None if no such file exists."""
    import numpy as np
    for name in ("grazing16384", "grazing8192"):
        path = os.path.join(GOLDEN_DIR, name + ".json")
        if not os.path.exists(path):
            continue
        with open(path) as fh:
            G = json.load(fh)
        if list(map(int, n)) != G["orders"]:
            return {"oracle": name, "error": "order sets differ"}
        return {"value": float(np.max(np.abs(np.asarray(e) - np.asarray(G["efficiencies"])))), "oracle": name,
                "oracle_N": G["N"], "oracle_energy_error": G["energy_error"],
                "oracle_self_convergence": (G.get("self_convergence") or {}).get("max_abs_efficiency_diff")}
    return None


def bench_c5(args):
    """Adjoint gradient of the specular efficiency with respect to the 256
    cosine and 256 sine coefficients of the deep-corrugation profile (dense
    mode, N = 8192): set-up, direct solve, adjoint solve and shape gradient,
    timed; checked against central finite differences (step 1e-6, and
    Richardson-extrapolated steps 1e-3 / 5e-4) of the library's own solves for
    the largest entries, outside the timed region."""
    import numpy as np
    import torch

    import paper_1707_04950_amd as lib
    import workloads as W

    wl = W.config_c5(8192)
    s = lib.Solver(0)
    N = wl.N
    n_a = max(8, int(math.floor(0.8 * min(wl.L, wl.d) / wl.dx)))
    kw = dict(d=wl.d, k=wl.k, alpha=wl.alpha, j=wl.j, A=wl.A, N=N, h=wl.h, c=wl.c, n_a=n_a,
              gamma_frac=wl.gamma_frac, eta=wl.eta, L=wl.L, mode=lib.MODE_DENSE)
    a0, b0 = np.array(wl.a_coef), np.array(wl.b_coef)

    def J_of(a, b, w):
        s.set_surface(a, b, **kw)
        mu, _ = s.solve(tol=1e-11, max_iter=3000, allow_noconv=True)
        return s.objective_adjoint_rhs(mu, w)[0]

    def gradient():
        t0 = time.perf_counter()
        s.set_surface(a0, b0, adjoint=1, **kw)  # the derivative matrices in the same pass as the operator
        mu, info = s.solve(tol=1e-11, max_iter=3000, allow_noconv=True)
        n, e, eps = s.efficiencies(mu)
        w = np.zeros(len(n))
        w[list(n).index(0)] = 1.0
        J, rhs = s.objective_adjoint_rhs(mu, w)
        t1 = time.perf_counter()
        nu, info2 = s.solve(b=rhs, tol=1e-12, max_iter=3000, adjoint=True, allow_noconv=True)
        ga, gb = s.shape_gradient(mu, nu, w, 256)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return dict(t_forward=t1 - t0, t_adjoint=t2 - t1, J=J, eps=eps, iters=info["iters"],
                    res=info["rel_residual"], adj_iters=info2["iters"], ga=ga, gb=gb, w=w)

    gradient()  # warm-up
    steps = max(1, args.steps)
    t0 = time.perf_counter()
    recs = [gradient() for _ in range(steps)]
    total = time.perf_counter() - t0
    r = recs[-1]
    scale = max(np.max(np.abs(r["ga"])), np.max(np.abs(r["gb"])))
    checks = []
    for kind, g in (("a", r["ga"]), ("b", r["gb"])):
        for m in list(np.argsort(-np.abs(g[1:]))[:2] + 1):
            fd = []
            for hh in (1e-6, 1e-3, 5e-4):
                ap, bp, am, bm = a0.copy(), b0.copy(), a0.copy(), b0.copy()
                (ap if kind == "a" else bp)[m] += hh
                (am if kind == "a" else bm)[m] -= hh
                fd.append((J_of(ap, bp, r["w"]) - J_of(am, bm, r["w"])) / (2 * hh))
            rich = (4 * fd[2] - fd[1]) / 3
            checks.append({"coef": "%s_%d" % (kind, m), "adjoint": float(g[m]), "fd_step_1e-6": fd[0],
                           "fd_richardson": rich, "rel_err_fd_1e-6": abs(fd[0] - g[m]) / scale,
                           "rel_err_richardson": abs(rich - g[m]) / scale})
    out = {
        "metric": "adjoint gradients/s: d(specular efficiency)/d(512 profile coefficients), deep corrugation N=8192",
        "value": steps / total,
        "unit": "gradients/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "N": N, "d_over_lambda": wl.d, "depth_pp": 10.0, "coefficients": 256,
                   "theta_deg": wl.theta_deg, "j": wl.j, "h": wl.h, "A_periods": wl.A, "mode": "dense"},
        "phase_s": {"setup_forward_solve": float(np.mean([x["t_forward"] for x in recs])),
                    "adjoint_solve_and_gradient": float(np.mean([x["t_adjoint"] for x in recs]))},
        "specular_efficiency": r["J"], "energy_balance_error": r["eps"], "iters": r["iters"],
        "rel_residual": r["res"], "adjoint_iters": r["adj_iters"],
        "gradient_max_abs": scale, "finite_difference_checks": checks,
    }
    s.close()
    print(json.dumps(out))


def bench_c4(args):
    """Many incidences (C4): a Gaussian random surface of period 50, N = 16384,
    64 incidence angles uniform in [0, 85] degrees at each of 4 wavenumbers
    (d/lambda = 50, 50.5, 51, 51.5).  Each wavenumber is one surface with one
    incidence set: the alpha-independent operator parts are built once, every
    member gets its own lattice-sum spectra, and the 64 systems are solved in
    lockstep (batched forward maps, one launch per stage and group).  The
    baseline solves the same 256 problems one at a time (set_surface at the
    angle, solve, efficiencies).  Prints one JSON line."""
    import numpy as np
    import torch

    import paper_1707_04950_amd as lib
    import workloads as W
    s = lib.Solver(0)
    angles = W.c4_angles(args.c4_angles)
    nk = len(W.C4_D_OVER_LAMBDA)

    def setup(wl, theta=0.0, mixed=False, mfma=False):
        n_a = max(8, int(math.floor(0.8 * min(wl.L, wl.d) / wl.dx)))
        w = wl.with_(theta_deg=theta)
        s.set_surface(np.asarray(w.a_coef), np.asarray(w.b_coef), w.d, w.k, w.alpha, w.j, w.A, w.N, h=w.h, c=w.c,
                      n_a=n_a, gamma_frac=w.gamma_frac, eta=w.eta, mode=lib.MODE_ACCEL, L=w.L, mixed=int(mixed),
                      batch_mfma=int(mfma))

    def batched(ik, mixed=False, mfma=False):
        wl = W.config_c4(ik, args.c4_N)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        setup(wl, mixed=mixed, mfma=mfma)
        s.set_incidences([wl.k * math.sin(math.radians(t)) for t in angles])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        X, infos = s.solve_incidences(tol=args.tol, max_iter=args.c4_max_iter, allow_noconv=True, mixed=mixed)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        effs = [s.efficiencies_incidence(r, X[r].contiguous()) for r in range(len(angles))]
        t3 = time.perf_counter()
        return dict(setup=t1 - t0, solve=t2 - t1, eff=t3 - t2, iters=[i["iters"] for i in infos],
                    steps=[i["residual_restarts"] for i in infos],
                    conv=[i["converged"] for i in infos], e=[e for _, e, _ in effs], eps=[p for _, _, p in effs])

    def single(ik):
        wl = W.config_c4(ik, args.c4_N)
        out = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for th in angles:
            setup(wl, th)
            mu, info = s.solve(tol=args.tol, max_iter=args.c4_max_iter, allow_noconv=True)
            out.append((s.efficiencies(mu)[1], info["iters"], info["converged"]))
        torch.cuda.synchronize()
        return time.perf_counter() - t0, out

    batched(0)  # warm-up: tuner, pools, code objects
    batched(0, mixed=True)
    batched(0, mfma=True)
    single(0)
    recs = [batched(ik) for ik in range(nk)]
    t_batch = sum(r["setup"] + r["solve"] + r["eff"] for r in recs)
    frecs = [batched(ik, mfma=True) for ik in range(nk)]
    t_mfma = sum(r["setup"] + r["solve"] + r["eff"] for r in frecs)
    dmf = max(float(np.max(np.abs(np.asarray(em) - np.asarray(eb)))) for r, m in zip(recs, frecs)
              for eb, em in zip(r["e"], m["e"]))
    mrecs = [batched(ik, mixed=True) for ik in range(nk)]
    t_mixed = sum(r["setup"] + r["solve"] + r["eff"] for r in mrecs)
    dmix = max(float(np.max(np.abs(np.asarray(em) - np.asarray(eb)))) for r, m in zip(recs, mrecs)
               for eb, em in zip(r["e"], m["e"]))
    sing = [single(ik) for ik in range(nk)]
    t_single = sum(t for t, _ in sing)
    n_solves = nk * len(angles)
    diff = max(float(np.max(np.abs(np.asarray(eb) - np.asarray(es)))) for r, (_, o) in zip(recs, sing)
               for eb, (es, _, _) in zip(r["e"], o))
    out = {
        "metric": "incidence sweep solves/s (C4: 64 angles x 4 wavenumbers, N=%d)" % args.c4_N,
        "value": n_solves / t_batch, "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "gauss-d50-rms0.5 incidence sweep", "N": args.c4_N, "angles": len(angles),
                   "d_over_lambda": list(W.C4_D_OVER_LAMBDA), "gmres_tol": args.tol},
        "single_solves_per_s": n_solves / t_single, "speedup_vs_single": t_single / t_batch,
        "phase_s": {"setup": sum(r["setup"] for r in recs), "solve": sum(r["solve"] for r in recs),
                    "eff": sum(r["eff"] for r in recs)},
        "iters_min_median_max": [int(min(min(r["iters"]) for r in recs)),
                                 int(np.median([i for r in recs for i in r["iters"]])),
                                 int(max(max(r["iters"]) for r in recs))],
        "all_converged": all(all(r["conv"]) for r in recs) and all(c for _, o in sing for _, _, c in o),
        "max_energy_balance_error": max(abs(p) for r in recs for p in r["eps"]),
        "max_efficiency_diff_batched_vs_single": diff,
        "matrix_cores_batched": {
            "solves_per_s": n_solves / t_mfma, "speedup_vs_single": t_single / t_mfma,
            "speedup_vs_vector_batched": t_batch / t_mfma, "solve_s": sum(r["solve"] for r in frecs),
            "all_converged": all(all(r["conv"]) for r in frecs), "max_efficiency_diff_vs_vector_batched": dmf},
        "mixed_precision_batched": {
            "solves_per_s": n_solves / t_mixed, "speedup_vs_fp64_batched": t_batch / t_mixed,
            "solve_s": sum(r["solve"] for r in mrecs),
            "iters_min_median_max": [int(min(min(r["iters"]) for r in mrecs)),
                                     int(np.median([i for r in mrecs for i in r["iters"]])),
                                     int(max(max(r["iters"]) for r in mrecs))],
            "refinement_steps_max": int(max(max(r["steps"]) for r in mrecs)),
            "all_converged": all(all(r["conv"]) for r in mrecs),
            "max_efficiency_diff_vs_fp64": dmix,
            "max_energy_balance_error": max(abs(p) for r in mrecs for p in r["eps"])},
    }
    s.close()
    print(json.dumps(out))


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.workload == "c5":
        if args.gpus != 1:
            print("bench.py: the solver runs on a single GPU; --gpus %d is not supported" % args.gpus, file=sys.stderr)
            sys.exit(2)
        bench_c5(args)
        return
    if args.workload == "c4":
        if args.gpus != 1:
            print("bench.py: the solver runs on a single GPU; --gpus %d is not supported" % args.gpus, file=sys.stderr)
            sys.exit(2)
        bench_c4(args)
        return
    if args.gpus != 1:
        print("bench.py: the solver runs on a single GPU; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1707_04950_amd as lib
    import workloads as W

    wl = W.config_grazing_wood(args.N)
    mode = lib.MODE_ACCEL if args.mode == "accel" else lib.MODE_DENSE
    s = lib.Solver(0)
    n_a = max(8, int(math.floor(0.8 * min(wl.L, wl.d) / wl.dx)))  # a = n_a dx just below the cell side

    if args.near_split == "auto":
        split_kw = {"near_split": 0}
    else:
        split_kw = {"near_split": 1, "split_permille": tuple(int(v) for v in args.near_split.split(","))}

    def setup(**kw):
        s.set_surface(np.asarray(wl.a_coef), np.asarray(wl.b_coef), wl.d, wl.k, wl.alpha, wl.j, wl.A, args.N,
                      h=wl.h, c=wl.c, n_a=n_a, gamma_frac=wl.gamma_frac, eta=wl.eta, mode=mode, L=wl.L,
                      **(kw or split_kw))

    def step():
        t0 = time.perf_counter()
        setup()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        mu, info = s.solve(tol=args.tol, max_iter=args.max_iter, allow_noconv=True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        n, e, eps = s.efficiencies(mu)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        return dict(setup=t1 - t0, solve=t2 - t1, eff=t3 - t2, iters=info["iters"], res=info["rel_residual"],
                    est=info["est_residual"], conv=info["converged"], eps=eps, n_orders=len(n), n=n, e=e,
                    mism=info["column_mismatches"])

    split_info = {"near_items": None, "near_tuned_us": None}
    # Warmup.  The last warmup step times every kernel class (HIP events on each
    # kernel's own stream) to find the class with the largest total time.
    all_mask = (1 << lib.KT_COUNT) - 1
    ranking = None
    for w in range(args.warmup):
        if w == args.warmup - 1:
            s.timing_enable(all_mask)
        step()
        if w == args.warmup - 1:
            ranking = s.timing_read()
            s.timing_enable(0)
            if mode == lib.MODE_ACCEL:
                inf = s.info()
                split_info = {"near_items": inf["near_items"], "near_tuned_us": inf["near_tuned_us"]}
    if ranking:  # records come in class order
        dom = max(ranking, key=lambda n: ranking[n]["total_ms"])
        dom_id = list(ranking).index(dom)
    else:  # no warmup: the operator's main HBM stream
        dom_id = lib.KT_GEMV if mode == lib.MODE_DENSE else lib.KT_LOCAL
        dom = "k_gemv_rows" if mode == lib.MODE_DENSE else "k_local_apply"

    # Timed region: every TIMING_EVERY-th launch of the dominant kernel class is
    # bracketed by events (a sparse sample keeps the brackets' cost out of the step time).
    s.timing_enable(1 << dom_id, TIMING_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    ms_per_step = 1e3 * total / args.steps
    kst = s.timing_read()[dom]
    s.timing_enable(0)

    # steady-state forward map: events on the library's stream (torch's current stream)
    mu = torch.from_numpy(W.random_density(args.N, 1)).cuda()
    y = torch.empty_like(mu)
    reps = 30
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def time_matvec():
        # steady state: the median of three rounds of `reps` maps after a warm-up
        # (the first round after the solves runs a few per cent slow)
        for _ in range(10):
            s.matvec(mu, y)
        rounds = []
        for _ in range(3):
            ev0.record()
            for _ in range(reps):
                s.matvec(mu, y)
            ev1.record()
            torch.cuda.synchronize()
            rounds.append(ev0.elapsed_time(ev1) / 1e3 / reps)
        return sorted(rounds)[1]

    mv_s = time_matvec()
    y_fixed = y.clone()
    auto_split = None
    if mode == lib.MODE_ACCEL and args.near_split != "auto":
        # the tuner's own pick for comparison (a surface set up with near_split = 0)
        setup(near_split=0)
        inf = s.info()
        auto_split = {"near_items_per_launch": inf["near_items"], "ms": time_matvec() * 1e3,
                      "same_result": bool(torch.equal(y, y_fixed))}
        setup()

    # batched forward maps (one operator, BATCH densities: groups of four share
    # the near-field and projection pass); same events, same stream
    batch = None
    if args.mode == "accel":
        mub = torch.from_numpy(np.stack([W.random_density(args.N, 100 + r) for r in range(BATCH)])).cuda()
        yb = torch.empty_like(mub)
        for _ in range(3):
            s.matvec_batch(mub, yb)
        ev0.record()
        for _ in range(reps // 3):
            s.matvec_batch(mub, yb)
        ev1.record()
        torch.cuda.synchronize()
        bt_s = ev0.elapsed_time(ev1) / 1e3 / (reps // 3)
        y1 = torch.empty_like(mu)
        s.matvec(mub[BATCH - 1].contiguous(), y1)
        torch.cuda.synchronize()
        batch = {"nrhs": BATCH, "ms_per_batch": bt_s * 1e3, "munknowns_per_s": BATCH * args.N / bt_s / 1e6,
                 "speedup_vs_single": mv_s * BATCH / bt_s,
                 "last_row_equals_single": bool(torch.equal(yb[BATCH - 1], y1))}

    # batched solve: the incidences alpha + 2 pi p / d, p = 0, -1, ..., of the
    # workload's Bloch class (one operator) in one lockstep GMRES, against the
    # single solve of the timed steps (same tolerance, unrestarted)
    bsolve = None
    if args.mode == "accel" and not args.no_batched_solve:
        B = torch.stack([s.rhs_bloch(-p) for p in range(BATCH)])
        s.solve_batch(B, tol=args.batch_tol, max_iter=args.max_iter, allow_noconv=True)  # warm-up (work space pooled)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xb, infos = s.solve_batch(B, tol=args.batch_tol, max_iter=args.max_iter, allow_noconv=True)
        torch.cuda.synchronize()
        bs_s = time.perf_counter() - t0
        # the single solves of the same eight systems at the same tolerance
        single_s = 0.0
        for p in range(BATCH):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xp, _ = s.solve(B[p].contiguous(), tol=args.batch_tol, max_iter=args.max_iter, allow_noconv=True)
            torch.cuda.synchronize()
            single_s += time.perf_counter() - t0
            if p == 0:
                x1 = xp
        single_s /= BATCH
        bsolve = {"nrhs": BATCH, "incidences": "alpha + 2 pi p / d, p = 0..-%d" % (BATCH - 1), "tol": args.batch_tol,
                  "single_solve_ms_mean": single_s * 1e3,
                  "ms_per_batch": bs_s * 1e3, "solves_per_s": BATCH / bs_s,
                  "speedup_vs_single_solve": single_s * BATCH / bs_s,
                  "iters": [i["iters"] for i in infos], "all_converged": all(i["converged"] for i in infos),
                  "column_mismatches": int(sum(i["column_mismatches"] for i in infos)),
                  "member0_equals_single": bool(torch.equal(xb[0], x1))}
        # the same batch with the near field of the eight densities on the matrix cores
        setup(batch_mfma=1, **split_kw)
        s.solve_batch(B, tol=args.batch_tol, max_iter=args.max_iter, allow_noconv=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xm, infm = s.solve_batch(B, tol=args.batch_tol, max_iter=args.max_iter, allow_noconv=True)
        torch.cuda.synchronize()
        bm_s = time.perf_counter() - t0
        ybm = torch.empty_like(mub)
        s.matvec_batch(mub, ybm)
        for _ in range(3):
            s.matvec_batch(mub, ybm)
        ev0.record()
        for _ in range(reps // 3):
            s.matvec_batch(mub, ybm)
        ev1.record()
        torch.cuda.synchronize()
        bsolve["matrix_cores"] = {
            "ms_per_batch": bm_s * 1e3, "solves_per_s": BATCH / bm_s, "speedup_vs_single_solve": single_s * BATCH / bm_s,
            "forward_map_ms_per_8": ev0.elapsed_time(ev1) / (reps // 3),
            "iters": [i["iters"] for i in infm], "all_converged": all(i["converged"] for i in infm),
            "max_rel_diff_vs_vector_solutions": float((xm - xb).abs().max() / xb.abs().max())}
        setup()

    # mixed precision (FP32 EqSources operators and Krylov basis under FP64
    # refinement) on the same workload, outside the timed region: a surface
    # set up with the FP32 operators, one warm-up and one timed solve
    mixed = None
    if args.mode == "accel" and not args.no_mixed:
        s.set_surface(np.asarray(wl.a_coef), np.asarray(wl.b_coef), wl.d, wl.k, wl.alpha, wl.j, wl.A, args.N,
                      h=wl.h, c=wl.c, n_a=n_a, gamma_frac=wl.gamma_frac, eta=wl.eta, mode=mode, L=wl.L, mixed=1)
        s.solve(tol=args.tol, max_iter=args.max_iter, allow_noconv=True, mixed=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mu_m, inf_m = s.solve(tol=args.tol, max_iter=args.max_iter, allow_noconv=True, mixed=True)
        torch.cuda.synchronize()
        t_m = time.perf_counter() - t0
        n_m, e_m, eps_m = s.efficiencies(mu_m)
        cmp_m = efficiency_vs_oracle(n_m, e_m)
        mixed = {"solve_ms": t_m * 1e3, "fp64_solve_ms": float(np.mean([r["solve"] for r in recs])) * 1e3,
                 "speedup_vs_fp64": float(np.mean([r["solve"] for r in recs])) / t_m, "iters": inf_m["iters"],
                 "refinement_steps": inf_m["residual_restarts"], "converged": inf_m["converged"],
                 "rel_residual": inf_m["rel_residual"],
                 "max_efficiency_diff_vs_fp64": float(np.max(np.abs(e_m - recs[-1]["e"]))),
                 "efficiency_err_vs_oracle": cmp_m["value"] if cmp_m else None, "energy_balance_error": eps_m}

    # efficiencies against the oracle's (dense LU of the same workload at the
    # largest N it was run at; stored by tests/golden/gen_golden.py), outside
    # the timed region
    oracle_cmp = efficiency_vs_oracle(recs[-1]["n"], recs[-1]["e"])

    # hybrid spatial/spectral kernel tables (the same workload set up with
    # table = 1), and the scattered field off the surface, outside the timed region
    hybrid = field_rec = None
    if args.mode == "accel" and not args.no_mixed:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        setup(table=1, **split_kw)
        torch.cuda.synchronize()
        t_set = time.perf_counter() - t0
        t0 = time.perf_counter()
        mu_h, inf_h = s.solve(tol=args.tol, max_iter=args.max_iter, allow_noconv=True)
        torch.cuda.synchronize()
        t_sol = time.perf_counter() - t0
        n_h, e_h, eps_h = s.efficiencies(mu_h)
        cmp_h = efficiency_vs_oracle(n_h, e_h)
        hybrid = {"setup_ms": t_set * 1e3, "windowed_setup_ms": float(np.mean([r["setup"] for r in recs])) * 1e3,
                  "spectral_rows": s.info()["spectral_rows"], "solve_ms": t_sol * 1e3, "iters": inf_h["iters"],
                  "converged": inf_h["converged"], "efficiency_err_vs_oracle": cmp_h["value"] if cmp_h else None,
                  "max_efficiency_diff_vs_windowed": float(np.max(np.abs(e_h - recs[-1]["e"]))),
                  "energy_balance_error": eps_h}
        setup()
        mu_f, _ = s.solve(tol=args.tol, max_iter=args.max_iter, allow_noconv=True)
        inf = s.info()
        ytop = inf["y0"] + inf["n_y"] * inf["L"]
        rng = np.random.default_rng(3)
        npts = 16384
        field_rec = {"points": npts}
        for name, yy in (("grid_ms", ytop - rng.uniform(0.01, 0.4, npts)), ("rayleigh_ms", ytop + 0.5 + rng.uniform(0, 2, npts))):
            xx = rng.uniform(0, wl.d, npts)
            s.field(mu_f, xx[:16], yy[:16])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.field(mu_f, xx, yy)
            torch.cuda.synchronize()
            field_rec[name] = (time.perf_counter() - t0) * 1e3

    # the whole forward map against the HBM roof: algorithmic bytes of its five
    # launches (per launch, from the fully timed warm-up step) over the
    # steady-state forward-map time
    fmap = None
    if ranking and args.mode == "accel":
        fb = sum(ranking[k]["bytes"] / ranking[k]["launches"] for k in
                 ("k_local_apply", "k_merge_fft", "k_fft_rows", "k_yconv", "k_cells_far") if ranking[k]["launches"])
        fmap = {"bytes": fb, "ms": mv_s * 1e3, "GBps": fb / mv_s / 1e9, "frac_of_hbm_peak": fb / mv_s / 1e9 / HBM_PEAK_GBS,
                "near_split": args.near_split, "near_items_per_launch": split_info["near_items"],
                "tuned_split": auto_split}

    n_launch = max(kst["launches"], 1)
    avg_s = kst["total_ms"] / 1e3 / n_launch
    roof = {"kernel": dom, "bound": "hbm", "achieved": kst["bytes"] / n_launch / avg_s / 1e9, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "bytes_per_launch": kst["bytes"] / n_launch, "avg_launch_us": avg_s * 1e6,
            "launches": kst["launches"], "sampled_every": TIMING_EVERY}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(dom, split_info["near_items"])
    kernels = None
    if ranking:
        kernels = {n: {"launches": r["launches"], "total_ms": round(r["total_ms"], 3),
                       "avg_us": round(1e3 * r["total_ms"] / r["launches"], 2),
                       "GBps": round(r["bytes"] / (r["total_ms"] / 1e3) / 1e9, 1)}
                   for n, r in ranking.items() if r["launches"]}

    out = {
        "metric": METRIC,
        "value": args.steps / total,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "N": args.N, "d_over_lambda": wl.d * wl.k / (2 * math.pi),
                   "theta_deg": wl.theta_deg, "j": wl.j, "h": wl.h, "A_periods": wl.A, "mode": args.mode,
                   "gmres_tol": args.tol},
        "matvec_munknowns_per_s": args.N / mv_s / 1e6,
        "matvec_ms": mv_s * 1e3,
        "forward_map": fmap,
        "batched_matvec": batch,
        "batched_solve": bsolve,
        "gmres_iters": recs[-1]["iters"],
        "gmres_rel_residual": recs[-1]["res"],
        "gmres_rel_residual_estimate": recs[-1]["est"],
        "all_steps_converged": all(r["conv"] for r in recs),
        "efficiency_err_vs_oracle": oracle_cmp,
        "mixed_precision_solve": mixed,
        "hybrid_table": hybrid,
        "off_surface_field": field_rec,
        "energy_balance_error": max((r["eps"] for r in recs), key=abs),
        # every step solves the same problem: its efficiencies must agree bit for bit
        "steps_identical": all(np.array_equal(r["e"], recs[0]["e"]) for r in recs),
        "hessenberg_column_mismatches": int(sum(r["mism"] for r in recs)),
        "phase_s": {k: float(np.mean([r[k] for r in recs])) for k in ("setup", "solve", "eff")},
        "roofline": roof,
        "kernels_warmup_step": kernels,
    }
    s.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.N)
    print(json.dumps(out))
    if not out["all_steps_converged"]:
        print("bench.py: a timed solve missed the tolerance (true residual %.3e > %.1e)" % (recs[-1]["res"], args.tol),
              file=sys.stderr)
        sys.exit(3)


if __name__ == "__main__":
    main()
