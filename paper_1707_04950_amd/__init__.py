"""Python binding of libsesm (C ABI in include/sesm.h).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch provides device memory (complex128 CUDA tensors) and the stream.
Importing this module does not load the library; the first Solver() does, and
raises if libsesm.so has not been built (python -m paper_1707_04950_amd.build).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsesm.so")

SESM_OK = 0
SESM_EINVAL = -1
SESM_ENOSURF = -2
SESM_ENOMEM = -3
SESM_EHIP = -4
SESM_ERESONANT = -5
SESM_ENOCONV = -6
MODE_DENSE = 0
MODE_ACCEL = 1


class Profile(ctypes.Structure):
    _fields_ = [("n_modes", ctypes.c_int32), ("a", ctypes.POINTER(ctypes.c_double)),
                ("b", ctypes.POINTER(ctypes.c_double))]


class Params(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("h", ctypes.c_double), ("c_window", ctypes.c_double),
                ("n_a", ctypes.c_int32), ("gamma_frac", ctypes.c_double), ("eta", ctypes.c_double),
                ("mode", ctypes.c_int32), ("L_cell", ctypes.c_double), ("n_side", ctypes.c_int32),
                ("n_ext", ctypes.c_int32), ("n_coll", ctypes.c_int32), ("n_plw", ctypes.c_int32),
                ("near_ring", ctypes.c_int32), ("near_split", ctypes.c_int32),
                ("split_permille", ctypes.c_int32 * 3), ("mixed", ctypes.c_int32), ("table", ctypes.c_int32), ("batch_mfma", ctypes.c_int32),
                ("adjoint", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("rel_residual", ctypes.c_double), ("converged", ctypes.c_int32),
                ("column_mismatches", ctypes.c_int32), ("est_residual", ctypes.c_double),
                ("residual_restarts", ctypes.c_int32), ("reserved_i", ctypes.c_int32)]


SOLVE_X0 = 1  # sesm_solve flag: mu holds the initial guess on entry
SOLVE_MIXED = 2  # mixed precision: FP64 refinement around FP32-basis inner solves
SOLVE_ADJOINT = 4  # the conjugate-transpose system (dense mode)


def _info_dict(i):
    return {"iters": i.iters, "rel_residual": i.rel_residual, "converged": bool(i.converged),
            "column_mismatches": i.column_mismatches, "est_residual": i.est_residual,
            "residual_restarts": i.residual_restarts}


# kernel classes of sesm_timing_enable (bit i of the mask selects class i)
KT_LOCAL, KT_MERGE, KT_FFT, KT_YCONV, KT_CELLS, KT_DOTS, KT_UPDATE, KT_GEMV = range(8)
KT_COUNT = 8
SESM_MAX_BATCH = 64  # right-hand sides per solve_batch call


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class SurfaceInfo(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("n_a", ctypes.c_int32), ("dx", ctypes.c_double),
                ("a", ctypes.c_double), ("gamma", ctypes.c_double), ("h", ctypes.c_double),
                ("A_len", ctypes.c_double), ("mode", ctypes.c_int32), ("n_eta", ctypes.c_int32),
                ("U_eta", ctypes.c_int32 * 16), ("n_first", ctypes.c_int32), ("n_count", ctypes.c_int32),
                ("n_x", ctypes.c_int32), ("n_y", ctypes.c_int32), ("n_cells_occupied", ctypes.c_int32),
                ("stencil_rows", ctypes.c_int32), ("L", ctypes.c_double), ("y0", ctypes.c_double),
                ("delta", ctypes.c_double), ("near_entries", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("near_items", ctypes.c_int32 * 4), ("near_tuned_us", ctypes.c_double),
                ("spectral_rows", ctypes.c_int32 * 2)]


_lib = None
_P = ctypes.c_void_p
_I = ctypes.c_int32
_D = ctypes.c_double


def load_library(path=LIB_PATH):
    """Load libsesm.so and declare the C signatures (no GPU work)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libsesm.so is not built (%s); run `python -m paper_1707_04950_amd.build`" % path)
    lib = ctypes.CDLL(path)
    sig = {
        "sesm_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, _P]),
        "sesm_destroy": (ctypes.c_int, [_P]),
        "sesm_set_surface": (ctypes.c_int, [_P, ctypes.POINTER(Profile), _D, _D, _D, _I, _D,
                                            ctypes.POINTER(Params)]),
        "sesm_matvec": (ctypes.c_int, [_P, _P, _P]),
        "sesm_matvec_batch": (ctypes.c_int, [_P, _I, _P, ctypes.c_int64, _P, ctypes.c_int64]),
        "sesm_rhs": (ctypes.c_int, [_P, _P]),
        "sesm_rhs_bloch": (ctypes.c_int, [_P, _I, _P]),
        "sesm_solve": (ctypes.c_int, [_P, _P, _P, _D, _I, _I, _I, ctypes.POINTER(SolveInfo)]),
        "sesm_solve_batch": (ctypes.c_int, [_P, _I, _P, ctypes.c_int64, _P, ctypes.c_int64, _D, _I, _I, _P]),
        "sesm_efficiencies": (ctypes.c_int, [_P, _P, ctypes.POINTER(_I), ctypes.POINTER(_I),
                                             ctypes.POINTER(_D), _I, ctypes.POINTER(_D)]),
        "sesm_rayleigh": (ctypes.c_int, [_P, _P, ctypes.POINTER(_I), _I, _P]),
        "sesm_get_info": (ctypes.c_int, [_P, ctypes.POINTER(SurfaceInfo)]),
        "sesm_last_error": (ctypes.c_char_p, [_P]),
        "sesm_diag_hankel": (ctypes.c_int, [_P, _P, _I, _P, _P]),
        "sesm_diag_cexp": (ctypes.c_int, [_P, _P, _I, _P]),
        "sesm_diag_accel": (ctypes.c_int, [_P, _P, _I, _P, ctypes.c_int64]),
        "sesm_diag_near": (ctypes.c_int, [_P, _P, _P]),
        "sesm_timing_enable": (ctypes.c_int, [_P, ctypes.c_uint32, _I]),
        "sesm_diag_fft": (ctypes.c_int, [_P, _I, _I, _P, _P, _I]),
        "sesm_timing_read": (ctypes.c_int, [_P, _P, _I]),
        "sesm_set_incidences": (ctypes.c_int, [_P, _I, ctypes.POINTER(_D)]),
        "sesm_rhs_incidence": (ctypes.c_int, [_P, _I, _P]),
        "sesm_matvec_incidences": (ctypes.c_int, [_P, _I, _I, _P, ctypes.c_int64, _P, ctypes.c_int64]),
        "sesm_solve_incidences": (ctypes.c_int, [_P, _I, _I, _P, ctypes.c_int64, _P, ctypes.c_int64, _D, _I, _I, _P]),
        "sesm_efficiencies_incidence": (ctypes.c_int, [_P, _I, _P, ctypes.POINTER(_I), ctypes.POINTER(_I),
                                                       ctypes.POINTER(_D), _I, ctypes.POINTER(_D)]),
        "sesm_field": (ctypes.c_int, [_P, _P, _I, _P, _P]),
        "sesm_matvec_adjoint": (ctypes.c_int, [_P, _P, _P]),
        "sesm_objective_adjoint_rhs": (ctypes.c_int, [_P, _P, ctypes.POINTER(_D), _I, _P, ctypes.POINTER(_D)]),
        "sesm_shape_gradient": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(_D), _I, _I, ctypes.POINTER(_D),
                                               ctypes.POINTER(_D)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class SesmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("sesm error %d: %s" % (code, msg))
        self.code = code


def _ptr(t, n=None):
    """Pointer of a contiguous complex128 CUDA tensor holding at least n
    elements (the library reads or writes n elements through it)."""
    import torch
    if t.dtype != torch.complex128:
        raise ValueError("expected a complex128 tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if n is not None and t.numel() < n:
        raise ValueError("tensor holds %d elements, the library needs %d" % (t.numel(), n))
    if not t.is_cuda:
        raise ValueError("expected a CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _ptr_rows(t, n, rows=None):
    """Pointer of a 2-D complex128 CUDA tensor whose rows have unit stride:
    row r (r < rows) is read or written as n elements at data_ptr + r stride(0),
    so the rows must be at least n long and stride(0) >= n (no overlap)."""
    import torch
    if t.dtype != torch.complex128 or t.dim() != 2:
        raise ValueError("expected a 2-D complex128 tensor")
    rows = t.shape[0] if rows is None else rows
    if t.shape[1] < n:
        raise ValueError("rows hold %d elements, the library needs %d" % (t.shape[1], n))
    if t.shape[0] < rows:
        raise ValueError("tensor has %d rows, the call needs %d" % (t.shape[0], rows))
    if t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError("expected unit stride along rows")
    if rows > 1 and t.stride(0) < n:
        raise ValueError("row stride %d is below the row length %d" % (t.stride(0), n))
    # the rows' span must lie inside the tensor's storage
    end = t.storage_offset() + (rows - 1) * t.stride(0) + n if rows > 0 else 0
    if end > t.untyped_storage().nbytes() // t.element_size():
        raise ValueError("rows extend past the tensor's storage")
    if not t.is_cuda:
        raise ValueError("expected a CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """One library context on a GPU (one stream)."""

    def __init__(self, device=0, stream=None):
        import torch
        self._torch = torch
        self.lib = load_library()
        self.device = torch.device("cuda", device)
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.stream = st
        h = _P()
        rc = self.lib.sesm_create(ctypes.byref(h), device, ctypes.c_void_p(st.cuda_stream))
        if rc != 0:
            raise SesmError(rc, "sesm_create failed")
        self.h = h
        self.N = None

    def close(self):
        if getattr(self, "h", None):
            self.lib.sesm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=()):
        if rc != 0 and rc not in allow:
            raise SesmError(rc, self.lib.sesm_last_error(self.h).decode())
        return rc

    def set_surface(self, a_coef, b_coef, d, k, alpha, j, A, N, h=0.0, c=0.0, n_a=0, gamma_frac=0.0,
                    eta=0.0, mode=MODE_DENSE, L=0.0, n_side=0, n_ext=0, n_coll=0, n_plw=0, near_ring=0,
                    near_split=0, split_permille=(0, 0, 0), mixed=0, table=0, batch_mfma=0, adjoint=0):
        a = np.ascontiguousarray(a_coef, dtype=np.float64)
        b = np.zeros_like(a)
        bb = np.asarray(b_coef, dtype=np.float64)
        b[: min(len(a), len(bb))] = bb[: len(a)]
        self._a, self._b = a, b  # keep alive during the call
        prof = Profile(len(a) - 1, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                       b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        prm = Params(N=N, h=h, c_window=c, n_a=n_a, gamma_frac=gamma_frac, eta=eta, mode=mode, L_cell=L,
                     n_side=n_side, n_ext=n_ext, n_coll=n_coll, n_plw=n_plw, near_ring=near_ring,
                     near_split=near_split, split_permille=(ctypes.c_int32 * 3)(*split_permille), mixed=int(mixed),
                     table=int(table), batch_mfma=int(batch_mfma), adjoint=int(adjoint))
        self._check(self.lib.sesm_set_surface(self.h, ctypes.byref(prof), d, k, alpha, j, A, ctypes.byref(prm)))
        self.N = N

    def info(self):
        inf = SurfaceInfo()
        self._check(self.lib.sesm_get_info(self.h, ctypes.byref(inf)))
        out = {f: getattr(inf, f) for f, _ in SurfaceInfo._fields_}
        out["U_eta"] = list(inf.U_eta)[: inf.n_eta]
        out["near_items"] = list(inf.near_items)
        out["spectral_rows"] = list(inf.spectral_rows)
        return out

    def empty(self):
        if os.environ.get("SESM_POISON_ALLOC", "0") not in ("", "0"):  # outputs start as NaN too
            return self._torch.full((self.N,), complex("nan+nanj"), dtype=self._torch.complex128,
                                    device=self.device)
        return self._torch.empty(self.N, dtype=self._torch.complex128, device=self.device)

    def matvec(self, mu, out=None):
        out = self.empty() if out is None else out
        self._check(self.lib.sesm_matvec(self.h, _ptr(mu, self.N), _ptr(out, self.N)))
        return out

    def matvec_batch(self, mu, out=None):
        """Forward maps of the rows of mu (nrhs x >= N, complex128 on the device,
        unit stride along a row) into the rows of out (allocated if None)."""
        if mu.dim() != 2 or mu.shape[1] < self.N:
            raise ValueError("mu must be a (nrhs, >= N) tensor")
        if out is None:
            out = self._torch.empty((mu.shape[0], self.N), dtype=self._torch.complex128, device=self.device)
            if os.environ.get("SESM_POISON_ALLOC", "0") not in ("", "0"):
                out.fill_(complex("nan+nanj"))
        if out.dim() != 2 or out.shape[0] != mu.shape[0] or out.shape[1] < self.N:
            raise ValueError("out must be a (nrhs, >= N) tensor")
        n = int(mu.shape[0])
        self._check(self.lib.sesm_matvec_batch(self.h, n, _ptr_rows(mu, self.N), int(mu.stride(0)),
                                               _ptr_rows(out, self.N, n), int(out.stride(0))))
        return out

    def rhs(self, out=None):
        out = self.empty() if out is None else out
        self._check(self.lib.sesm_rhs(self.h, _ptr(out, self.N)))
        return out

    def rhs_bloch(self, p, out=None):
        """Right-hand side of the incidence alpha + 2 pi p / d (same operator)."""
        out = self.empty() if out is None else out
        self._check(self.lib.sesm_rhs_bloch(self.h, int(p), _ptr(out, self.N)))
        return out

    def solve(self, b=None, tol=1e-10, max_iter=1000, restart=0, out=None, allow_noconv=False, x0=None,
              mixed=False, adjoint=False):
        """GMRES solve; x0 (a device tensor of N) is the initial guess and is
        overwritten with the solution (warm start); otherwise the iteration
        starts from zero and the solution goes to out (allocated if None).
        mixed: FP64 refinement around FP32-basis inner solves (surface set up
        with mixed=1).  adjoint: the conjugate-transpose system (dense mode,
        b required)."""
        flags = (SOLVE_MIXED if mixed else 0) | (SOLVE_ADJOINT if adjoint else 0)
        if x0 is not None:
            if out is not None and out is not x0:
                raise ValueError("with x0 the solution overwrites x0; do not pass out")
            out, flags = x0, flags | SOLVE_X0
        out = self.empty() if out is None else out
        inf = SolveInfo()
        bp = _ptr(b, self.N) if b is not None else None
        rc = self.lib.sesm_solve(self.h, bp, _ptr(out, self.N), tol, max_iter, restart, flags, ctypes.byref(inf))
        self._check(rc, allow=(SESM_ENOCONV,) if allow_noconv else ())
        return out, _info_dict(inf)

    def solve_batch(self, b, tol=1e-10, max_iter=1000, out=None, allow_noconv=False, x0=None, mixed=False):
        """Unrestarted GMRES for the rows of b (nrhs x >= N, complex128 on the
        device) in lockstep; returns the solutions (rows of out) and one info
        dict per row.  x0 (nrhs x >= N): initial guesses, overwritten with the
        solutions (warm start)."""
        if b.dim() != 2 or b.shape[1] < self.N:
            raise ValueError("b must be a (nrhs, >= N) tensor")
        n = int(b.shape[0])
        flags = SOLVE_MIXED if mixed else 0
        if x0 is not None:
            if out is not None and out is not x0:
                raise ValueError("with x0 the solutions overwrite x0; do not pass out")
            out, flags = x0, flags | SOLVE_X0
        if out is None:
            out = self._torch.empty((n, self.N), dtype=self._torch.complex128, device=self.device)
            if os.environ.get("SESM_POISON_ALLOC", "0") not in ("", "0"):
                out.fill_(complex("nan+nanj"))
        if out.dim() != 2 or out.shape[0] != n or out.shape[1] < self.N:
            raise ValueError("out must be a (nrhs, >= N) tensor")
        infs = (SolveInfo * max(n, 1))()
        rc = self.lib.sesm_solve_batch(self.h, n, _ptr_rows(b, self.N), int(b.stride(0)), _ptr_rows(out, self.N, n),
                                       int(out.stride(0)), tol, max_iter, flags, ctypes.cast(infs, ctypes.c_void_p))
        self._check(rc, allow=(SESM_ENOCONV,) if allow_noconv else ())
        return out, [_info_dict(i) for i in infs[:n]]

    def efficiencies(self, mu):
        cap = 4096
        e = np.zeros(cap)
        n0, nc = _I(), _I()
        eps = _D()
        self._check(self.lib.sesm_efficiencies(self.h, _ptr(mu, self.N), ctypes.byref(n0), ctypes.byref(nc),
                                               e.ctypes.data_as(ctypes.POINTER(_D)), cap, ctypes.byref(eps)))
        return np.arange(n0.value, n0.value + nc.value), e[: nc.value].copy(), eps.value

    # ---- incidence sets (several alpha on one surface and wavenumber)
    def set_incidences(self, alphas):
        a = np.ascontiguousarray(alphas, dtype=np.float64)
        self._check(self.lib.sesm_set_incidences(self.h, len(a), a.ctypes.data_as(ctypes.POINTER(_D))))
        self.n_inc = len(a)

    def rhs_incidence(self, r, out=None):
        out = self.empty() if out is None else out
        self._check(self.lib.sesm_rhs_incidence(self.h, int(r), _ptr(out, self.N)))
        return out

    def matvec_incidences(self, mu, r0=0, out=None):
        """Forward maps of the rows of mu, row i with the operator of member r0 + i."""
        if mu.dim() != 2 or mu.shape[1] < self.N:
            raise ValueError("mu must be a (nrhs, >= N) tensor")
        n = int(mu.shape[0])
        if out is None:
            out = self._torch.empty((n, self.N), dtype=self._torch.complex128, device=self.device)
        self._check(self.lib.sesm_matvec_incidences(self.h, int(r0), n, _ptr_rows(mu, self.N), int(mu.stride(0)),
                                                    _ptr_rows(out, self.N, n), int(out.stride(0))))
        return out

    def solve_incidences(self, r0=0, n=None, b=None, tol=1e-10, max_iter=1000, out=None, allow_noconv=False,
                         x0=None, mixed=False):
        """Lockstep GMRES for members r0 .. r0 + n - 1 (their incident fields when b is None)."""
        n = (self.n_inc - r0) if n is None else int(n)
        flags = SOLVE_MIXED if mixed else 0
        if x0 is not None:
            out, flags = x0, flags | SOLVE_X0
        if out is None:
            out = self._torch.empty((n, self.N), dtype=self._torch.complex128, device=self.device)
        if out.dim() != 2 or out.shape[0] != n or out.shape[1] < self.N:
            raise ValueError("out must be a (n, >= N) tensor")
        bp, ldb = None, self.N
        if b is not None:
            if b.dim() != 2 or b.shape[0] != n:
                raise ValueError("b must be a (n, >= N) tensor")
            bp, ldb = _ptr_rows(b, self.N), int(b.stride(0))
        infs = (SolveInfo * max(n, 1))()
        rc = self.lib.sesm_solve_incidences(self.h, int(r0), n, bp, ldb, _ptr_rows(out, self.N, n), int(out.stride(0)),
                                            tol, max_iter, flags, ctypes.cast(infs, ctypes.c_void_p))
        self._check(rc, allow=(SESM_ENOCONV,) if allow_noconv else ())
        return out, [_info_dict(i) for i in infs[:n]]

    def efficiencies_incidence(self, r, mu):
        cap = 4096
        e = np.zeros(cap)
        n0, nc = _I(), _I()
        eps = _D()
        self._check(self.lib.sesm_efficiencies_incidence(self.h, int(r), _ptr(mu, self.N), ctypes.byref(n0),
                                                         ctypes.byref(nc), e.ctypes.data_as(ctypes.POINTER(_D)), cap,
                                                         ctypes.byref(eps)))
        return np.arange(n0.value, n0.value + nc.value), e[: nc.value].copy(), eps.value

    def field(self, mu, x, y, out=None):
        """Scattered field at the points (x[t], y[t]) (host arrays or sequences)."""
        xy = np.ascontiguousarray(np.stack([np.asarray(x, dtype=np.float64).ravel(),
                                            np.asarray(y, dtype=np.float64).ravel()], 1))
        n = xy.shape[0]
        dxy = self._torch.from_numpy(xy.reshape(-1)).to(self.device)
        out = self._torch.empty(n, dtype=self._torch.complex128, device=self.device) if out is None else out
        if n:
            self._check(self.lib.sesm_field(self.h, _ptr(mu, self.N), n, ctypes.c_void_p(dxy.data_ptr()),
                                            _ptr(out, n)))
        return out

    def matvec_adjoint(self, mu, out=None):
        out = self.empty() if out is None else out
        self._check(self.lib.sesm_matvec_adjoint(self.h, _ptr(mu, self.N), _ptr(out, self.N)))
        return out

    def objective_adjoint_rhs(self, mu, weights):
        """(J, rhs): J = sum_n w_n e_n over the propagating orders, rhs the
        right-hand side of the adjoint solve."""
        w = np.ascontiguousarray(weights, dtype=np.float64)
        rhs = self.empty()
        J = _D()
        self._check(self.lib.sesm_objective_adjoint_rhs(self.h, _ptr(mu, self.N), w.ctypes.data_as(ctypes.POINTER(_D)),
                                                        len(w), _ptr(rhs, self.N), ctypes.byref(J)))
        return J.value, rhs

    def shape_gradient(self, mu, nu, weights, n_modes):
        """dJ/da_m, dJ/db_m (m = 0..n_modes) from the direct and adjoint densities."""
        w = np.ascontiguousarray(weights, dtype=np.float64)
        ga = np.zeros(n_modes + 1)
        gb = np.zeros(n_modes + 1)
        self._check(self.lib.sesm_shape_gradient(self.h, _ptr(mu, self.N), _ptr(nu, self.N),
                                                 w.ctypes.data_as(ctypes.POINTER(_D)), len(w), int(n_modes),
                                                 ga.ctypes.data_as(ctypes.POINTER(_D)),
                                                 gb.ctypes.data_as(ctypes.POINTER(_D))))
        return ga, gb

    def rayleigh(self, mu, orders):
        o = np.ascontiguousarray(orders, dtype=np.int32)
        B = np.zeros(len(o), dtype=np.complex128)
        self._check(self.lib.sesm_rayleigh(self.h, _ptr(mu, self.N), o.ctypes.data_as(ctypes.POINTER(_I)), len(o),
                                           ctypes.c_void_p(B.ctypes.data)))
        return B

    def diag_accel(self, mu, which, length):
        out = self._torch.empty(length, dtype=self._torch.complex128, device=self.device)
        self._check(self.lib.sesm_diag_accel(self.h, _ptr(mu, self.N), which, _ptr(out, length), length))
        return out

    def diag_near(self, mu, out=None):
        out = self.empty() if out is None else out
        self._check(self.lib.sesm_diag_near(self.h, _ptr(mu, self.N), _ptr(out, self.N)))
        return out

    def timing_enable(self, mask, every=1):
        """Time every `every`-th launch of the kernel classes in `mask` (bit i = class KT_*); clears counters."""
        self._check(self.lib.sesm_timing_enable(self.h, int(mask), int(every)))

    def timing_read(self):
        """Per-class records {name: dict(launches, total_ms, bytes)} since timing_enable."""
        arr = (KernelStat * KT_COUNT)()
        self._check(self.lib.sesm_timing_read(self.h, ctypes.cast(arr, ctypes.c_void_p), KT_COUNT))
        return {r.name.decode(): {"launches": int(r.launches), "total_ms": float(r.total_ms), "bytes": float(r.bytes)}
                for r in arr}

    def diag_fft(self, x, sign=-1):
        """The library's own FFT along the last axis of a 2-D complex tensor (rows x n)."""
        torch = self._torch
        x = x.to(device=self.device, dtype=torch.complex128).contiguous()
        rows, n = x.shape
        out = torch.empty_like(x)
        self._check(self.lib.sesm_diag_fft(self.h, n, rows, _ptr(x), _ptr(out), sign))
        return out

    def diag_cexp(self, t):
        torch = self._torch
        t = t.to(device=self.device, dtype=torch.float64).contiguous()
        out = torch.empty(t.numel(), dtype=torch.complex128, device=self.device)
        self._check(self.lib.sesm_diag_cexp(self.h, ctypes.c_void_p(t.data_ptr()), t.numel(), _ptr(out)))
        return out

    def diag_hankel(self, x):
        torch = self._torch
        x = x.to(device=self.device, dtype=torch.float64).contiguous()
        h0 = torch.empty(x.numel(), dtype=torch.complex128, device=self.device)
        h1 = torch.empty_like(h0)
        self._check(self.lib.sesm_diag_hankel(self.h, ctypes.c_void_p(x.data_ptr()), x.numel(), _ptr(h0), _ptr(h1)))
        return h0, h1


def efficiency_objective(solver, a_coef, b_coef, weights, surface, tol=1e-10, max_iter=1000):
    """J = sum_n w_n e_n of the surface with Fourier coefficients (a_coef,
    b_coef) (torch tensors, float64, on the host; b_coef[0] unused) as a
    differentiable function: a torch.autograd.Function whose forward sets up
    the surface on `solver` (dense mode; `surface`: the other set_surface
    keywords, d, k, alpha, j, A, N and discretisation parameters), solves and
    forms J, and whose backward solves the adjoint system and takes the shape
    gradient on the device."""
    import torch

    class _Objective(torch.autograd.Function):
        @staticmethod
        def forward(fctx, a, b):
            kw = dict(surface)
            kw["mode"] = MODE_DENSE
            # a gradient to come: the derivative matrices with the operator, in one pass
            kw.setdefault("adjoint", int(a.requires_grad or b.requires_grad))
            solver.set_surface(a.detach().cpu().numpy(), b.detach().cpu().numpy(), **kw)
            mu, info = solver.solve(tol=tol, max_iter=max_iter)
            J, _ = solver.objective_adjoint_rhs(mu, weights)
            fctx.mu = mu
            fctx.n_modes = a.shape[0] - 1
            return torch.tensor(J, dtype=torch.float64)

        @staticmethod
        def backward(fctx, gJ):
            J, rhs = solver.objective_adjoint_rhs(fctx.mu, weights)
            nu, info = solver.solve(b=rhs, tol=tol, max_iter=max_iter, adjoint=True)
            ga, gb = solver.shape_gradient(fctx.mu, nu, weights, fctx.n_modes)
            g = float(gJ)
            return torch.from_numpy(g * ga), torch.from_numpy(g * gb)

    return _Objective.apply(a_coef, b_coef)
