"""Helpers for the GPU tests: marshal a workloads.Workload into the library."""
import numpy as np

import paper_1707_04950_amd as lib


def set_surface(solver, wl, disc, mode=lib.MODE_DENSE, **kw):
    """Configure `solver` with exactly the discretisation parameters the
    oracle's Discretization `disc` uses."""
    solver.set_surface(np.asarray(wl.a_coef), np.asarray(wl.b_coef), wl.d, wl.k, wl.alpha, wl.j, wl.A,
                       disc.N, h=wl.h, c=wl.c, n_a=disc.n_a, gamma_frac=wl.gamma_frac, eta=wl.eta,
                       mode=mode, L=wl.L, **kw)


def to_dev(torch, v):
    return torch.from_numpy(np.ascontiguousarray(v, dtype=np.complex128)).cuda()


def to_host(t):
    return t.detach().cpu().numpy()
