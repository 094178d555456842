"""ctypes binding of libhelm (include/helm.h).

Argument marshalling only: every numerical step runs in the library's HIP kernels.  torch
provides device memory (tensors passed by data_ptr()) and the current HIP stream.  Loading
fails loudly if libhelm.so has not been built; there is no fallback path.
"""
import atexit
import ctypes
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhelm.so")

HELM_OK, HELM_ENOTCONV, HELM_EINVAL, HELM_ENOMEM, HELM_ESINGULAR, HELM_EHIP = 0, 1, -1, -2, -3, -4
HELM_C64, HELM_C128 = 0, 1
HELM_LINE_LDU, HELM_LINE_ND = 0, 1


class helm_grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int)]


class helm_pml(ctypes.Structure):
    _fields_ = [("b", ctypes.c_int), ("C", ctypes.c_double), ("p", ctypes.c_int), ("fronts", ctypes.c_int),
                ("fronts_inner", ctypes.c_int), ("C_moving", ctypes.c_double)]


class helm_stats(ctypes.Structure):
    _fields_ = [("setup_ms", ctypes.c_double), ("apply_launches", ctypes.c_longlong),
                ("apply_rhs", ctypes.c_longlong), ("apply_ms", ctypes.c_double),
                ("apply_bytes_per_rhs", ctypes.c_double), ("matvec_launches", ctypes.c_longlong),
                ("matvec_rhs", ctypes.c_longlong), ("matvec_ms", ctypes.c_double),
                ("matvec_bytes_per_rhs", ctypes.c_double), ("kernel_launches", ctypes.c_longlong),
                ("kernel_rhs", ctypes.c_longlong), ("kernel_ms", ctypes.c_double),
                ("kernel_bytes", ctypes.c_double), ("kernel_flops", ctypes.c_double),
                ("nd_setup_ms", ctypes.c_double)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_SIGS = {
    "helm_setup": (_I, [ctypes.POINTER(helm_grid), _P, _D, ctypes.POINTER(helm_pml), _I, _I, _P,
                        ctypes.POINTER(_P)]),
    "helm_apply": (_I, [_P, _P, _P, _I, _P]),
    "helm_apply_adjoint": (_I, [_P, _P, _P, _I, _P]),
    "helm_apply_static": (_I, [_P, _P, _P, _I, _I, _P]),
    "helm_matvec": (_I, [_P, _P, _P, _I, _I, _P]),
    "helm_solve": (_I, [_P, _P, _P, _I, _D, _I, _I, _I, ctypes.POINTER(_I), ctypes.POINTER(_D), _P]),
    "helm_grad_c": (_I, [_P, _P, _P, _I, _P, _P]),
    "helm_misfit": (_I, [_P, _P, _P, _I, _I, ctypes.POINTER(_D), _P, _P]),
    "helm_set_medium": (_I, [_P, _P, _P]),
    "helm_update_medium": (_I, [_P, _P, _P, _P, _P]),
    "helm_info": (_I, [_P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "helm_workspace_bytes": (_I, [_P, _I, _I, _I, ctypes.POINTER(ctypes.c_size_t),
                                  ctypes.POINTER(ctypes.c_size_t)]),
    "helm_pool_trim": (None, []),
    "helm_pool_stats": (None, [ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
    "helm_plan_bytes": (_I, [ctypes.POINTER(helm_grid), ctypes.POINTER(helm_pml), _I, _I,
                             ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "helm_line_factors": (_I, [_P, _I, _I, _P, ctypes.POINTER(_I), ctypes.POINTER(_I), _P]),
    "helm_line_solve": (_I, [_P, _I, _I, _P, _P, _I, _I, _P]),
    "helm_set_launch": (_I, [_P, _I]),
    "helm_set_line_solver": (_I, [_P, _I, _P]),
    "helm_sweep_shape": (_I, [_P, _I, ctypes.POINTER(_I), ctypes.c_char_p, _I]),
    "helm_set_exchange_test": (_I, [_P, _I, ctypes.c_uint]),
    "helm_get_stats": (_I, [_P, ctypes.POINTER(helm_stats)]),
    "helm_autotune": (_I, [_P, _I, ctypes.c_char_p, ctypes.POINTER(_I), ctypes.POINTER(_D), _P]),
    "helm_reset_stats": (_I, [_P]),
    "helm_destroy": (None, [_P]),
    "helm_error_string": (ctypes.c_char_p, [_I]),
    "helm_last_error": (ctypes.c_char_p, []),
}

_lib = None
# handles not yet destroyed: closed (and the device pool released) by an exit handler that
# runs before the interpreter tears down, so no HIP call reaches the runtime after a
# profiler or the runtime itself has begun finalising
_live = weakref.WeakSet()


@atexit.register
def _close_all():
    for H in list(_live):
        try:
            H.close()
        except Exception:
            pass
    if _lib is not None:
        _lib.helm_pool_trim()


def lib():
    """The loaded libhelm (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1502_07266_amd.build` (no fallback path exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class HelmError(RuntimeError):
    def __init__(self, code, where):
        L = lib()
        msg = f"{where}: {L.helm_error_string(code).decode()} ({L.helm_last_error().decode()})"
        super().__init__(msg)
        self.code = code


def _check(rc, where):
    if rc < 0:
        raise HelmError(rc, where)
    return rc


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def plan_bytes(n, b, C, p, slab_layers=1, prec=HELM_C64, fronts=1, fronts_inner=1):
    """Device bytes of a setup, computed on the host: (bytes, n_lines, max_block)."""
    nb, nl, mb = ctypes.c_size_t(), _I(), _I()
    pml = helm_pml(b, C, p, fronts, fronts_inner)
    _check(lib().helm_plan_bytes(ctypes.byref(helm_grid(n)), ctypes.byref(pml),
                                 slab_layers, prec, ctypes.byref(nb), ctypes.byref(nl),
                                 ctypes.byref(mb)), "helm_plan_bytes")
    return nb.value, nl.value, mb.value


def pool_stats():
    """(bytes cached by the library's device memory pool, bytes in use)."""
    c, l = ctypes.c_size_t(), ctypes.c_size_t()
    lib().helm_pool_stats(ctypes.byref(c), ctypes.byref(l))
    return c.value, l.value


def pool_trim():
    """Release the pool's cached device memory to the HIP runtime."""
    lib().helm_pool_trim()


class Helm:
    """One setup of the recursive sweeping preconditioner on the current GPU.

    c: float64 CUDA tensor of shape (n, n, n), indexed [k, j, i] (x1 fastest).  All vector
    arguments are complex128 CUDA tensors of shape (R, n, n, n) or (n, n, n).  fronts: 1 for
    the outer sweep from x3 = 0 (Algorithm 6), 2 for two fronts meeting in a middle slab;
    fronts_inner: the same for the inner sweep over x2 (Algorithm 4); C_moving: the constant
    of the auxiliary problems' moving PML (0: C).
    """

    def __init__(self, c, omega, b, C, p, slab_layers=1, prec="c64", fronts=1, fronts_inner=1,
                 C_moving=0.0):
        import torch
        if not (isinstance(c, torch.Tensor) and c.is_cuda and c.dtype == torch.float64):
            raise TypeError("c must be a float64 CUDA tensor")
        c = c.contiguous()
        n = c.shape[0]
        if tuple(c.shape) != (n, n, n):
            raise ValueError("c must have shape (n, n, n)")
        self.n, self.omega, self.b, self.C, self.p, self.d = n, float(omega), b, float(C), p, slab_layers
        self.fronts, self.fronts_inner = fronts, fronts_inner
        self.prec = HELM_C64 if prec in ("c64", HELM_C64) else HELM_C128
        h = ctypes.c_void_p()
        _check(lib().helm_setup(ctypes.byref(helm_grid(n)), _ptr(c), self.omega,
                                ctypes.byref(helm_pml(b, self.C, p, fronts, fronts_inner, float(C_moving))),
                                slab_layers, self.prec,
                                _stream(), ctypes.byref(h)), "helm_setup")
        self._h = h
        _live.add(self)

    # ------------------------------------------------------------------ helpers
    def _batch(self, x):
        import torch
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.complex128):
            raise TypeError("vectors must be complex128 CUDA tensors")
        x = x.contiguous()
        if x.dim() == 3:
            x = x.unsqueeze(0)
        if tuple(x.shape[1:]) != (self.n,) * 3:
            raise ValueError("vectors must have shape (R, n, n, n)")
        return x

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("handle was destroyed")
        return self._h

    # ------------------------------------------------------------------ operations
    def apply(self, r, adjoint=False):
        """z = M^{-1} r (or M^{-H} r)."""
        import torch
        r = self._batch(r)
        z = torch.empty_like(r)
        fn = lib().helm_apply_adjoint if adjoint else lib().helm_apply
        _check(fn(self.handle, _ptr(r), _ptr(z), r.shape[0], _stream()), "helm_apply")
        return z

    def apply_static(self, r, adjoint=False):
        """z = M^{-1} r (or M^{-H} r) with the library's static scratch: no allocation in the
        library (z is allocated here by torch)."""
        import torch
        r = self._batch(r)
        z = torch.empty_like(r)
        _check(lib().helm_apply_static(self.handle, _ptr(r), _ptr(z), r.shape[0], int(adjoint), _stream()),
               "helm_apply_static")
        return z

    def matvec(self, u, adjoint=False):
        import torch
        u = self._batch(u)
        y = torch.empty_like(u)
        _check(lib().helm_matvec(self.handle, _ptr(u), _ptr(y), u.shape[0], int(adjoint), _stream()),
               "helm_matvec")
        return y

    def solve(self, f, tol=1e-6, restart=50, maxit=500, adjoint=False, x0=None):
        """FGMRES solve; returns (u, iters[R], relres[R], status)."""
        import torch
        f = self._batch(f)
        u = torch.zeros_like(f) if x0 is None else self._batch(x0).clone()
        R = f.shape[0]
        its = (_I * R)()
        rel = (_D * R)()
        rc = _check(lib().helm_solve(self.handle, _ptr(f), _ptr(u), R, float(tol), int(restart),
                                     int(maxit), int(adjoint), its, rel, _stream()), "helm_solve")
        return u, np.array(its[:]), np.array(rel[:]), rc

    def misfit(self, u, d, plane_k, want_source=True):
        """(J, adjoint source g = P^T (P u - d)) for receivers on x3-layer plane_k."""
        import torch
        u = self._batch(u)
        d = d.contiguous()
        g = torch.empty_like(u) if want_source else None
        J = _D()
        _check(lib().helm_misfit(self.handle, _ptr(u), _ptr(d), u.shape[0], int(plane_k),
                                 ctypes.byref(J), _ptr(g) if g is not None else None, _stream()),
               "helm_misfit")
        return J.value, g

    def grad_c(self, u, lam):
        import torch
        u = self._batch(u)
        lam = self._batch(lam)
        g = torch.empty((self.n,) * 3, dtype=torch.float64, device=u.device)
        _check(lib().helm_grad_c(self.handle, _ptr(u), _ptr(lam), u.shape[0], _ptr(g), _stream()),
               "helm_grad_c")
        return g

    def set_medium(self, c):
        c = c.contiguous()
        _check(lib().helm_set_medium(self.handle, _ptr(c), _stream()), "helm_set_medium")

    def update_medium(self, c, box):
        """Local update after a change of c inside box = (i0, i1, j0, j1, k0, k1) (1-based,
        inclusive): re-factors the lines whose windows meet the box; returns their count."""
        c = c.contiguous()
        b = (ctypes.c_int * 6)(*[int(v) for v in box])
        nr = _I()
        _check(lib().helm_update_medium(self.handle, _ptr(c), b, ctypes.byref(nr), _stream()),
               "helm_update_medium")
        return nr.value

    def info(self):
        fb, nl, mb = ctypes.c_size_t(), _I(), _I()
        _check(lib().helm_info(self.handle, ctypes.byref(fb), ctypes.byref(nl), ctypes.byref(mb)),
               "helm_info")
        return {"factor_bytes": fb.value, "n_lines": nl.value, "max_block": mb.value}

    def workspace_bytes(self, R, restart=50, maxit=500):
        """{"solve": bytes a solve may take at most, "apply": bytes of an apply's scratch}."""
        sb, ab = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().helm_workspace_bytes(self.handle, int(R), int(restart), int(maxit), ctypes.byref(sb),
                                          ctypes.byref(ab)), "helm_workspace_bytes")
        return {"solve": sb.value, "apply": ab.value}

    def line_factors(self, zg, yg):
        """The block inverses T_1..T_n of line (zg, yg): tensor (n, B, B)."""
        import torch
        B = _I()
        _check(lib().helm_line_factors(self.handle, zg, yg, None, ctypes.byref(B), None, _stream()),
               "helm_line_factors")
        dt = torch.complex64 if self.prec == HELM_C64 else torch.complex128
        out = torch.empty((self.n, B.value, B.value), dtype=dt, device="cuda")
        _check(lib().helm_line_factors(self.handle, zg, yg, _ptr(out), None, None, _stream()),
               "helm_line_factors")
        return out

    def line_order(self, zg, yg):
        """The oracle's name of line (zg, yg)'s elimination order: "two-sided" (both ends
        towards block n/2) or "up" (x1 order, middle block n - 1)."""
        m = _I()
        _check(lib().helm_line_factors(self.handle, zg, yg, None, None, ctypes.byref(m), _stream()),
               "helm_line_factors")
        return "up" if m.value == self.n - 1 else "two-sided"

    def line_solve(self, zg, yg, r, adjoint=False):
        """x = K^{-1} r on the line grid; r: complex128 (R, Wz, Wy, n)."""
        import torch
        r = r.contiguous()
        x = torch.empty_like(r)
        _check(lib().helm_line_solve(self.handle, zg, yg, _ptr(r), _ptr(x), r.shape[0], int(adjoint),
                                     _stream()), "helm_line_solve")
        return x

    def stats(self):
        st = helm_stats()
        _check(lib().helm_get_stats(self.handle, ctypes.byref(st)), "helm_get_stats")
        return {f: getattr(st, f) for f, _ in helm_stats._fields_}

    def reset_stats(self):
        _check(lib().helm_reset_stats(self.handle), "helm_reset_stats")

    def autotune(self, R, cache_path=None):
        """Time a sweep of R right-hand sides with each candidate launch shape and keep the
        fastest (cached in cache_path); returns (variant, ms per sweep)."""
        v, ms = _I(), _D()
        path = cache_path.encode() if cache_path else None
        _check(lib().helm_autotune(self.handle, int(R), path, ctypes.byref(v), ctypes.byref(ms), _stream()),
               "helm_autotune")
        return v.value, ms.value

    def set_line_solver(self, solver):
        """Line problems of the forward complex64 sweeps: "ldu" (block LDU chains) or "nd"
        (nested dissection; factors them on the first switch)."""
        kind = {"ldu": HELM_LINE_LDU, "nd": HELM_LINE_ND}[solver]
        _check(lib().helm_set_line_solver(self.handle, kind, _stream()), "helm_set_line_solver")

    def set_launch(self, variant):
        """Use launch-shape variant k for the sweeps (-1: automatic)."""
        _check(lib().helm_set_launch(self.handle, int(variant)), "helm_set_launch")

    def sweep_shape(self, R):
        """(variant, description) a sweep of R right-hand sides uses now."""
        v = _I()
        buf = ctypes.create_string_buffer(96)
        _check(lib().helm_sweep_shape(self.handle, int(R), ctypes.byref(v), buf, 96), "helm_sweep_shape")
        return v.value, buf.value.decode()

    def set_exchange_test(self, drop_publish, spin_limit=0):
        """Failure injection for tests of the sweep's error path (see helm.h)."""
        _check(lib().helm_set_exchange_test(self.handle, int(drop_publish), int(spin_limit)),
               "helm_set_exchange_test")

    def close(self):
        if self._h is not None:
            lib().helm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
