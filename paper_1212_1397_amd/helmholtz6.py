"""Python binding of the helmholtz6 C ABI (include/helmholtz6.h, include/h6net.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Vectors are torch complex128 tensors on the GPU, contiguous, of
shape (n'z, n'y, n'x) (x fastest); PyTorch supplies device memory and the
current HIP stream.  If the compiled library is missing this module raises at
import time; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhelmholtz6.so")

H6_OK, H6_NOT_CONVERGED, H6_DIVERGED = 0, 1, 2
H6_ERR_ARG, H6_ERR_UNSUPPORTED_BC, H6_ERR_ALLOC, H6_ERR_HIP, H6_ERR_SINGULAR = -1, -2, -3, -4, -5
BC_CODES = {"D": 0, "N": 1, "S": 2}
METHODS = {"gmres": 0, "fgmres": 1, "sks": 2, "chebyshev": 3}
PRECISIONS = {"fp64": 0, "mixed": 1}
KERNEL_CLASSES = ("stencil", "stencil_resid", "xform_x", "xform_y", "tridiag_z", "mgs_dots",
                  "mgs_update", "norm", "axpy", "rhs")

EXPORTED = ("helmholtz6_setup", "helmholtz6_dims", "helmholtz6_apply_A", "helmholtz6_apply_Pinv",
            "helmholtz6_apply_Pinv_noalloc",
            "helmholtz6_rhs_gaussians", "helmholtz6_solve", "helmholtz6_profile",
            "helmholtz6_kernel_time", "helmholtz6_destroy", "helmholtz6_status_string",
            "helmholtz6_last_error", "helmholtz6_spectrum_bounds", "helmholtz6_psi_order",
            "helmholtz6_solve_batch", "helmholtz6_solve_batch_queue", "helmholtz6_queue_create",
            "helmholtz6_queue_solve", "helmholtz6_queue_last_error", "helmholtz6_queue_destroy",
            "helmholtz6_set_graphs", "helmholtz6_autotune",
            "helmholtz6_rhs_separable", "helmholtz6_rhs_dirichlet_z", "helmholtz6_rhs_neumann")
EXPORTED_NET = ("h6net_param_count", "h6net_create", "h6net_set_params", "h6net_get_params",
                "h6net_forward", "h6net_gradients", "h6net_train_step", "h6net_gradients_op",
                "h6net_train_step_op", "h6net_training_pair", "helmholtz6_attach_net",
                "helmholtz6_learned_steps", "h6net_destroy")
# layers of the correction network: (name, Cin, Cout), in parameter order
NET_LAYERS = (("e1a", 3, 16), ("e1b", 16, 16), ("e2a", 16, 32), ("e2b", 32, 32), ("b3a", 32, 64),
              ("b3b", 64, 64), ("d2a", 96, 32), ("d2b", 32, 32), ("d1a", 48, 16), ("d1b", 16, 16),
              ("out", 16, 2))


class H6Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("h", ctypes.c_double), ("k_re", ctypes.c_double),
                ("k_im", ctypes.c_double), ("bc", ctypes.c_int * 6), ("precision", ctypes.c_int)]


class H6SolveInfo(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int), ("restart", ctypes.c_int), ("maxit", ctypes.c_int),
                ("tol", ctypes.c_double), ("iters", ctypes.c_int), ("rel_resid", ctypes.c_double),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_len", ctypes.c_int),
                ("zero_guess", ctypes.c_int)]


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(f"helmholtz6 HIP library not found at {path}; build it with "
                           "`python -m paper_1212_1397_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(path)
    vp, ip = ctypes.c_void_p, ctypes.c_int
    lib.helmholtz6_setup.argtypes = [ctypes.POINTER(H6Params), vp, ctypes.POINTER(vp)]
    lib.helmholtz6_dims.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    lib.helmholtz6_apply_A.argtypes = [vp, vp, vp, vp]
    lib.helmholtz6_apply_Pinv.argtypes = [vp, vp, vp, vp]
    lib.helmholtz6_apply_Pinv_noalloc.argtypes = [vp, vp, vp, vp]
    lib.helmholtz6_rhs_gaussians.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_double), ctypes.c_double, vp, vp]
    lib.helmholtz6_solve.argtypes = [vp, vp, vp, ctypes.POINTER(H6SolveInfo), vp]
    lib.helmholtz6_profile.argtypes = [vp, ip]
    lib.helmholtz6_kernel_time.argtypes = [vp, ctypes.c_char_p, ip, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_longlong),
                                           ctypes.POINTER(ctypes.c_double)]
    lib.helmholtz6_destroy.argtypes = [vp]
    lib.helmholtz6_destroy.restype = None
    lib.helmholtz6_status_string.argtypes = [ip]
    lib.helmholtz6_status_string.restype = ctypes.c_char_p
    lib.helmholtz6_last_error.argtypes = [vp]
    lib.helmholtz6_last_error.restype = ctypes.c_char_p
    lib.helmholtz6_spectrum_bounds.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                               ctypes.POINTER(ctypes.c_double)]
    lib.helmholtz6_spectrum_bounds.restype = ctypes.c_int
    lib.helmholtz6_psi_order.argtypes = [ctypes.c_double] * 5
    lib.helmholtz6_psi_order.restype = ctypes.c_double
    lib.helmholtz6_solve_batch.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                           ctypes.POINTER(H6SolveInfo), ctypes.POINTER(ip), ip, ip]
    lib.helmholtz6_solve_batch.restype = ctypes.c_int
    lib.helmholtz6_solve_batch_queue.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                                 ctypes.POINTER(H6SolveInfo), ctypes.POINTER(ip), ip, ip]
    lib.helmholtz6_solve_batch_queue.restype = ctypes.c_int
    lib.helmholtz6_queue_create.argtypes = [ctypes.POINTER(vp), ip, ip, ip, ctypes.POINTER(vp)]
    lib.helmholtz6_queue_create.restype = ctypes.c_int
    lib.helmholtz6_queue_solve.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                           ctypes.POINTER(H6SolveInfo), ctypes.POINTER(ip)]
    lib.helmholtz6_queue_solve.restype = ctypes.c_int
    lib.helmholtz6_queue_last_error.argtypes = [vp]
    lib.helmholtz6_queue_last_error.restype = ctypes.c_char_p
    lib.helmholtz6_queue_destroy.argtypes = [vp]
    lib.helmholtz6_queue_destroy.restype = None
    lib.helmholtz6_set_graphs.argtypes = [vp, ip]
    lib.helmholtz6_set_graphs.restype = ctypes.c_int
    lib.helmholtz6_autotune.argtypes = [vp, ctypes.c_char_p, vp]
    lib.helmholtz6_autotune.restype = ctypes.c_int
    lib.helmholtz6_rhs_separable.argtypes = [vp, ip] + [ctypes.POINTER(ctypes.c_double)] * 4 + [vp, vp]
    lib.helmholtz6_rhs_separable.restype = ctypes.c_int
    lib.helmholtz6_rhs_dirichlet_z.argtypes = [vp, ip, vp, vp, vp]
    lib.helmholtz6_rhs_dirichlet_z.restype = ctypes.c_int
    lib.helmholtz6_rhs_neumann.argtypes = [vp, ip, ip] + [ctypes.POINTER(ctypes.c_double)] * 3 + [vp, vp]
    lib.helmholtz6_rhs_neumann.restype = ctypes.c_int
    for name in ("helmholtz6_setup", "helmholtz6_dims", "helmholtz6_apply_A", "helmholtz6_apply_Pinv",
                 "helmholtz6_apply_Pinv_noalloc", "helmholtz6_rhs_gaussians", "helmholtz6_solve", "helmholtz6_profile",
                 "helmholtz6_kernel_time"):
        getattr(lib, name).restype = ctypes.c_int
    fp = ctypes.POINTER(ctypes.c_float)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.h6net_param_count.argtypes = []
    lib.h6net_param_count.restype = ctypes.c_longlong
    lib.h6net_create.argtypes = [ctypes.POINTER(ctypes.c_int), vp, ctypes.POINTER(vp)]
    lib.h6net_set_params.argtypes = [vp, fp, ctypes.c_longlong, vp]
    lib.h6net_get_params.argtypes = [vp, fp, ctypes.c_longlong, vp]
    lib.h6net_forward.argtypes = [vp, vp, ctypes.c_double, vp, vp]
    lib.h6net_gradients.argtypes = [vp, vp, ctypes.c_double, vp, fp, dp, vp]
    lib.h6net_train_step.argtypes = [vp, vp, ctypes.c_double, vp, ctypes.c_float, dp, vp]
    lib.h6net_gradients_op.argtypes = [vp, vp, vp, vp, fp, dp, vp]
    lib.h6net_train_step_op.argtypes = [vp, vp, vp, vp, ctypes.c_float, dp, vp]
    lib.h6net_training_pair.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.h6net_training_pair.restype = ctypes.c_int
    lib.helmholtz6_attach_net.argtypes = [vp, vp]
    lib.helmholtz6_learned_steps.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    lib.h6net_destroy.argtypes = [vp]
    lib.h6net_destroy.restype = None
    for name in ("h6net_create", "h6net_set_params", "h6net_get_params", "h6net_forward",
                 "h6net_gradients", "h6net_train_step", "h6net_gradients_op", "h6net_train_step_op",
                 "helmholtz6_attach_net",
                 "helmholtz6_learned_steps"):
        getattr(lib, name).restype = ctypes.c_int
    return lib


_lib = load_library()


class H6Error(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"helmholtz6 status {status}: {msg}")
        self.status = status


def _stream_handle(stream=None):
    if stream is None:
        if not torch.cuda.is_available():
            return ctypes.c_void_p(None)     # legacy default stream (argument checks only)
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """A solver plan for one grid, wavenumber and face pattern (helmholtz6_setup)."""

    def __init__(self, n, h: float, k: complex, bc: str = "DDDDDD", precision: str = "fp64",
                 stream=None):
        if isinstance(n, int):
            n = (n, n, n)
        p = H6Params()
        for a in range(3):
            p.n[a] = int(n[a])
        p.h = float(h)
        k = complex(k)
        p.k_re, p.k_im = k.real, k.imag
        for f, c in enumerate(bc):
            p.bc[f] = BC_CODES[c]
        p.precision = PRECISIONS[precision]
        self._plan = ctypes.c_void_p()
        st = _lib.helmholtz6_setup(ctypes.byref(p), _stream_handle(stream), ctypes.byref(self._plan))
        if st != H6_OK:
            raise H6Error(st, _lib.helmholtz6_last_error(None).decode())
        dims = (ctypes.c_int * 3)()
        _lib.helmholtz6_dims(self._plan, dims)
        self.dims = tuple(dims)
        self.n, self.h, self.k, self.bc, self.precision = tuple(n), float(h), k, bc, precision

    @property
    def shape(self):
        return (self.dims[2], self.dims[1], self.dims[0])

    def _check(self, st):
        if st < 0:
            raise H6Error(st, _lib.helmholtz6_last_error(self._plan).decode())
        return st

    def _vec(self, t, name):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128
                and t.is_contiguous() and tuple(t.shape) == self.shape):
            raise ValueError(f"{name} must be a contiguous complex128 CUDA tensor of shape {self.shape}")
        return ctypes.c_void_p(t.data_ptr())

    def empty(self):
        return torch.empty(self.shape, dtype=torch.complex128, device="cuda")

    def apply_A(self, x, out=None, stream=None):
        out = self.empty() if out is None else out
        self._check(_lib.helmholtz6_apply_A(self._plan, self._vec(x, "x"), self._vec(out, "out"),
                                           _stream_handle(stream)))
        return out

    def apply_Pinv(self, r, out=None, stream=None):
        out = self.empty() if out is None else out
        self._check(_lib.helmholtz6_apply_Pinv(self._plan, self._vec(r, "r"), self._vec(out, "out"),
                                              _stream_handle(stream)))
        return out

    def apply_Pinv_noalloc(self, r, out=None, stream=None):
        """apply_Pinv with the library's fixed device work space (allocates nothing
        in the library; `out` must be given to avoid an allocation here)."""
        out = self.empty() if out is None else out
        self._check(_lib.helmholtz6_apply_Pinv_noalloc(self._plan, self._vec(r, "r"), self._vec(out, "out"),
                                                      _stream_handle(stream)))
        return out

    def rhs_gaussians(self, centres, amps, sigma: float, out=None, stream=None):
        import numpy as np
        c = np.ascontiguousarray(np.asarray(centres, dtype=np.float64).reshape(-1, 3))
        a = np.asarray(amps, dtype=np.complex128).reshape(-1)
        ab = np.ascontiguousarray(np.stack([a.real, a.imag], 1))
        out = self.empty() if out is None else out
        dp = ctypes.POINTER(ctypes.c_double)
        self._check(_lib.helmholtz6_rhs_gaussians(
            self._plan, int(c.shape[0]), c.ctypes.data_as(dp), ab.ctypes.data_as(dp), float(sigma),
            self._vec(out, "out"), _stream_handle(stream)))
        return out

    def rhs_separable(self, coef, tx, ty, tz, out=None, stream=None):
        """F for f = sum_s coef[s] X_s(x) Y_s(y) Z_s(z); tx, ty, tz: arrays of
        shape (nterms, 5, n'_a) holding derivative orders 0..4 of each factor at
        the unknown nodes of its axis (include/helmholtz6.h)."""
        import numpy as np
        c = np.ascontiguousarray(np.asarray(coef, dtype=np.complex128).reshape(-1))
        nt = c.shape[0]
        tabs = []
        for name, t, n in (("tx", tx, self.dims[0]), ("ty", ty, self.dims[1]), ("tz", tz, self.dims[2])):
            a = np.ascontiguousarray(np.asarray(t, dtype=np.complex128))
            if a.shape != (nt, 5, n):
                raise ValueError(f"{name} must have shape {(nt, 5, n)}, got {a.shape}")
            tabs.append(a)
        out = self.empty() if out is None else out
        dp = ctypes.POINTER(ctypes.c_double)
        self._check(_lib.helmholtz6_rhs_separable(
            self._plan, nt, c.ctypes.data_as(dp), *[a.ctypes.data_as(dp) for a in tabs],
            self._vec(out, "out"), _stream_handle(stream)))
        return out

    def rhs_dirichlet_z(self, side: int, g, F, stream=None):
        """F -= G g on the unknown plane next to Dirichlet z face `side` (0 or 1);
        g: contiguous complex128 CUDA tensor of shape (n'y, n'x)."""
        if not (isinstance(g, torch.Tensor) and g.is_cuda and g.dtype == torch.complex128
                and g.is_contiguous() and tuple(g.shape) == (self.dims[1], self.dims[0])):
            raise ValueError(f"g must be a contiguous complex128 CUDA tensor of shape {(self.dims[1], self.dims[0])}")
        self._check(_lib.helmholtz6_rhs_dirichlet_z(self._plan, int(side), ctypes.c_void_p(g.data_ptr()),
                                                   self._vec(F, "F"), _stream_handle(stream)))
        return F

    def rhs_neumann(self, face: int, coef, t1, t2, F, stream=None):
        """F += the eq. (3DN) data term of beta = sum_s coef[s] T1_s T2_s on Neumann
        face `face` (0..5); t1, t2: arrays (nterms, 5, n') of derivative orders
        0..4 along the face's tangential axes (increasing axis order)."""
        import numpy as np
        ax = int(face) // 2
        ta, tb = [a for a in range(3) if a != ax]
        c = np.ascontiguousarray(np.asarray(coef, dtype=np.complex128).reshape(-1))
        nt = c.shape[0]
        tabs = []
        for name, t, n in (("t1", t1, self.dims[ta]), ("t2", t2, self.dims[tb])):
            a = np.ascontiguousarray(np.asarray(t, dtype=np.complex128))
            if a.shape != (nt, 5, n):
                raise ValueError(f"{name} must have shape {(nt, 5, n)}, got {a.shape}")
            tabs.append(a)
        dp = ctypes.POINTER(ctypes.c_double)
        self._check(_lib.helmholtz6_rhs_neumann(self._plan, int(face), nt, c.ctypes.data_as(dp),
                                               tabs[0].ctypes.data_as(dp), tabs[1].ctypes.data_as(dp),
                                               self._vec(F, "F"), _stream_handle(stream)))
        return F

    def solve(self, F, U=None, method="gmres", restart=30, maxit=1000, tol=1e-10, history=512,
              stream=None, zero_guess=None):
        """Solve A U = F (U: initial guess, overwritten).  Returns (U, info dict).
        zero_guess=True starts from U = 0 without reading U (default: when U is None)."""
        if zero_guess is None:
            zero_guess = U is None
        U = torch.empty_like(F) if U is None else U
        hist = (ctypes.c_double * max(history, 1))()
        info = H6SolveInfo(METHODS[method], int(restart), int(maxit), float(tol), 0, 0.0,
                           ctypes.cast(hist, ctypes.POINTER(ctypes.c_double)), int(history),
                           int(bool(zero_guess)))
        st = self._check(_lib.helmholtz6_solve(self._plan, self._vec(F, "F"), self._vec(U, "U"),
                                               ctypes.byref(info), _stream_handle(stream)))
        status = {H6_OK: "ok", H6_NOT_CONVERGED: "not_converged", H6_DIVERGED: "diverged"}[st]
        return U, dict(status=status, iters=info.iters, rel_resid=info.rel_resid,
                       history=list(hist[:info.history_len]))

    def set_graphs(self, mode=True):
        """HIP graphs for GMRES / FGMRES: False / 0 off, True / 1 one graph per
        Arnoldi step, 2 or "cycle" one graph per restart cycle with the Givens
        rotations on the device."""
        m = 2 if mode == "cycle" else int(mode)
        self._check(_lib.helmholtz6_set_graphs(self._plan, m))

    def autotune(self, cache_path=None, stream=None):
        """Time the kernel variants on this grid and keep the fastest (optionally cached)."""
        self._check(_lib.helmholtz6_autotune(self._plan, cache_path.encode() if cache_path else None,
                                             _stream_handle(stream)))

    def spectrum_bounds(self):
        """(lo, hi): exact extreme eigenvalues of A A_p^{-1} (all-Dirichlet, real k)."""
        lo, hi = ctypes.c_double(), ctypes.c_double()
        self._check(_lib.helmholtz6_spectrum_bounds(self._plan, ctypes.byref(lo), ctypes.byref(hi)))
        return lo.value, hi.value

    def training_pair(self, F, Ustar, U, r=None, t=None, stream=None):
        """(r, t): r = F - A U and t = (Ustar - U) - A_p^{-1} r (h6net_training_pair)."""
        r = self.empty() if r is None else r
        t = self.empty() if t is None else t
        st = _lib.h6net_training_pair(self._plan, self._vec(F, "F"), self._vec(Ustar, "Ustar"), self._vec(U, "U"),
                                      self._vec(r, "r"), self._vec(t, "t"), _stream_handle(stream))
        self._check(st)
        return r, t

    def attach_net(self, net):
        """Use the learned correction of `net` in flexible GMRES solves (None detaches)."""
        self._net = net
        self._check(_lib.helmholtz6_attach_net(self._plan, net._net if net is not None else None))

    def learned_steps(self) -> int:
        n = ctypes.c_int()
        self._check(_lib.helmholtz6_learned_steps(self._plan, ctypes.byref(n)))
        return n.value

    def profile(self, enable: bool = True):
        self._check(_lib.helmholtz6_profile(self._plan, int(enable)))

    def kernel_time(self, name: str, reset: bool = False):
        """(total ms, launches, algorithmic bytes) of one kernel class since the last reset."""
        ms = ctypes.c_double()
        n = ctypes.c_longlong()
        b = ctypes.c_double()
        self._check(_lib.helmholtz6_kernel_time(self._plan, name.encode(), int(reset), ctypes.byref(ms),
                                                ctypes.byref(n), ctypes.byref(b)))
        return ms.value, n.value, b.value

    def close(self):
        if getattr(self, "_plan", None) and self._plan.value:
            _lib.helmholtz6_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Net:
    """The learned correction network (include/h6net.h) for grids of `dims`
    (n'x, n'y, n'z).  Parameters are host float32 arrays in the parameter
    layout: per layer of NET_LAYERS, W[co][ci][dz][dy][dx] then b[co]."""

    def __init__(self, dims, stream=None):
        d = (ctypes.c_int * 3)(*[int(x) for x in dims])
        self._net = ctypes.c_void_p()
        st = _lib.h6net_create(d, _stream_handle(stream), ctypes.byref(self._net))
        if st != H6_OK:
            raise H6Error(st, "h6net_create failed")
        self.dims = tuple(int(x) for x in dims)
        self.count = int(_lib.h6net_param_count())

    @property
    def shape(self):
        return (self.dims[2], self.dims[1], self.dims[0])

    def _check(self, st, what):
        if st < 0:
            raise H6Error(st, what)
        return st

    def _vec(self, t, name):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128
                and t.is_contiguous() and tuple(t.shape) == self.shape):
            raise ValueError(f"{name} must be a contiguous complex128 CUDA tensor of shape {self.shape}")
        return ctypes.c_void_p(t.data_ptr())

    def set_params(self, flat, stream=None):
        import numpy as np
        a = np.ascontiguousarray(np.asarray(flat, dtype=np.float32).reshape(-1))
        if a.size != self.count:
            raise ValueError(f"expected {self.count} parameters, got {a.size}")
        self._check(_lib.h6net_set_params(self._net, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                          self.count, _stream_handle(stream)), "set_params")

    def get_params(self, stream=None):
        import numpy as np
        a = np.empty(self.count, dtype=np.float32)
        self._check(_lib.h6net_get_params(self._net, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                          self.count, _stream_handle(stream)), "get_params")
        return a

    def forward(self, r, kh: float, out=None, stream=None):
        out = torch.empty_like(r) if out is None else out
        self._check(_lib.h6net_forward(self._net, self._vec(r, "r"), float(kh), self._vec(out, "out"),
                                       _stream_handle(stream)), "forward")
        return out

    def gradients(self, r, kh: float, t, stream=None):
        """(loss, flat float32 gradients) of the pair (r, t) without an update."""
        import numpy as np
        g = np.empty(self.count, dtype=np.float32)
        loss = ctypes.c_double()
        self._check(_lib.h6net_gradients(self._net, self._vec(r, "r"), float(kh), self._vec(t, "t"),
                                         g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                         ctypes.byref(loss), _stream_handle(stream)), "gradients")
        return loss.value, g

    def train_step(self, r, kh: float, t, lr: float, want_loss: bool = True, stream=None):
        loss = ctypes.c_double()
        self._check(_lib.h6net_train_step(self._net, self._vec(r, "r"), float(kh), self._vec(t, "t"),
                                          float(lr), ctypes.byref(loss) if want_loss else None,
                                          _stream_handle(stream)), "train_step")
        return loss.value if want_loss else None

    def gradients_op(self, plan, r, t, stream=None):
        """(operator-weighted loss |A (c - t)|^2 / |A t|^2, flat float32
        gradients) of the pair (r, t) on plan's grid, without an update."""
        import numpy as np
        g = np.empty(self.count, dtype=np.float32)
        loss = ctypes.c_double()
        self._check(_lib.h6net_gradients_op(self._net, plan._plan, self._vec(r, "r"), self._vec(t, "t"),
                                            g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                            ctypes.byref(loss), _stream_handle(stream)), "gradients_op")
        return loss.value, g

    def train_step_op(self, plan, r, t, lr: float, want_loss: bool = True, stream=None):
        """One Adam step on the operator-weighted loss of (r, t) on plan's grid."""
        loss = ctypes.c_double()
        self._check(_lib.h6net_train_step_op(self._net, plan._plan, self._vec(r, "r"), self._vec(t, "t"),
                                             float(lr), ctypes.byref(loss) if want_loss else None,
                                             _stream_handle(stream)), "train_step_op")
        return loss.value if want_loss else None

    def close(self):
        if getattr(self, "_net", None) and self._net.value:
            _lib.h6net_destroy(self._net)
            self._net = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pack_net_params(params) -> "numpy.ndarray":
    """Flat float32 parameter vector from {name: (W, b)} in NET_LAYERS order."""
    import numpy as np
    parts = []
    for name, cin, cout in NET_LAYERS:
        W, b = params[name]
        parts += [np.asarray(W, dtype=np.float32).reshape(-1), np.asarray(b, dtype=np.float32).reshape(-1)]
    return np.concatenate(parts)


def unpack_net_params(flat) -> dict:
    """{name: (W (Cout, Cin, 3, 3, 3), b (Cout,))} from the flat parameter vector."""
    import numpy as np
    out, o = {}, 0
    for name, cin, cout in NET_LAYERS:
        nw = cout * cin * 27
        W = np.asarray(flat[o:o + nw]).reshape(cout, cin, 3, 3, 3)
        b = np.asarray(flat[o + nw:o + nw + cout])
        out[name] = (W, b)
        o += nw + cout
    return out


def solve_batch(plans, Fs, Us, method="fgmres", restart=30, maxit=1000, tol=1e-8, nstreams=4,
                history=0):
    """Solve plans[i] x = Fs[i] into Us[i] (initial guesses, overwritten) concurrently on
    `nstreams` library streams, longest first.  Returns a list of info dicts."""
    n = len(plans)
    if not (len(Fs) == len(Us) == n):
        raise ValueError("plans, Fs and Us must have the same length")
    P = (ctypes.c_void_p * n)(*[p._plan.value for p in plans])
    Fp = (ctypes.c_void_p * n)(*[p._vec(F, "F").value for p, F in zip(plans, Fs)])
    Up = (ctypes.c_void_p * n)(*[p._vec(U, "U").value for p, U in zip(plans, Us)])
    hists = [(ctypes.c_double * max(history, 1))() for _ in range(n)]
    infos = (H6SolveInfo * n)()
    for i in range(n):
        infos[i] = H6SolveInfo(METHODS[method], int(restart), int(maxit), float(tol), 0, 0.0,
                               ctypes.cast(hists[i], ctypes.POINTER(ctypes.c_double)), int(history))
    sts = (ctypes.c_int * n)()
    torch.cuda.synchronize()              # inputs ready before the library streams start
    st = _lib.helmholtz6_solve_batch(P, Fp, Up, infos, sts, n, int(nstreams))
    if st < 0:
        msgs = [plans[i]._plan and _lib.helmholtz6_last_error(plans[i]._plan).decode()
                for i in range(n) if sts[i] < 0]
        raise H6Error(st, "; ".join(m for m in msgs if m) or "batch solve failed")
    names = {H6_OK: "ok", H6_NOT_CONVERGED: "not_converged", H6_DIVERGED: "diverged"}
    return [dict(status=names[sts[i]], iters=infos[i].iters, rel_resid=infos[i].rel_resid,
                 history=list(hists[i][:infos[i].history_len])) for i in range(n)]


def _queue_arrays(plans, Fs, Us, restart, maxit, tol):
    n = len(plans)
    if not (len(Fs) == len(Us) == n):
        raise ValueError("plans, Fs and Us must have the same length")
    Fp = (ctypes.c_void_p * n)(*[p._vec(F, "F").value for p, F in zip(plans, Fs)])
    Up = (ctypes.c_void_p * n)(*[p._vec(U, "U").value for p, U in zip(plans, Us)])
    infos = (H6SolveInfo * n)()
    for i in range(n):
        infos[i] = H6SolveInfo(METHODS["fgmres"], int(restart), int(maxit), float(tol), 0, 0.0, None, 0, 1)
    return Fp, Up, infos, (ctypes.c_int * n)()


def _queue_results(infos, sts, n):
    names = {H6_OK: "ok", H6_NOT_CONVERGED: "not_converged", H6_DIVERGED: "diverged"}
    return [dict(status=names[sts[i]], iters=infos[i].iters, rel_resid=infos[i].rel_resid, history=[])
            for i in range(n)]


class Queue:
    """Many flexible GMRES(restart) solves as one captured graph fed by a
    device-side queue per grid shape (helmholtz6_queue_create): built once for
    a list of plans, solved any number of times with new right-hand sides."""

    def __init__(self, plans, restart=30, lanes=2):
        n = len(plans)
        P = (ctypes.c_void_p * n)(*[p._plan.value for p in plans])
        self._q = ctypes.c_void_p()
        st = _lib.helmholtz6_queue_create(P, n, int(restart), int(lanes), ctypes.byref(self._q))
        if st != H6_OK:
            raise H6Error(st, _lib.helmholtz6_queue_last_error(None).decode() or "queue creation failed")
        self.plans, self.restart = list(plans), int(restart)

    def solve(self, Fs, Us, tol=1e-8, maxit=1000):
        """U[i] (overwritten; solves start from zero) for every F[i]; list of info dicts."""
        n = len(self.plans)
        Fp, Up, infos, sts = _queue_arrays(self.plans, Fs, Us, self.restart, maxit, tol)
        torch.cuda.synchronize()          # inputs ready before the library's streams start
        st = _lib.helmholtz6_queue_solve(self._q, Fp, Up, infos, sts)
        if st < 0:
            raise H6Error(st, _lib.helmholtz6_queue_last_error(self._q).decode() or "queued solve failed")
        return _queue_results(infos, sts, n)

    def close(self):
        if self._q:
            _lib.helmholtz6_queue_destroy(self._q)
            self._q = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch_queue(plans, Fs, Us, restart=30, maxit=1000, tol=1e-8, lanes=2):
    """Flexible GMRES(restart) solves of plans[i] x = Fs[i] into Us[i] (from zero) as one
    captured graph fed by a device-side queue per grid shape (helmholtz6_solve_batch_queue:
    queue create, solve and destroy in one call), `lanes` lanes per shape."""
    n = len(plans)
    P = (ctypes.c_void_p * n)(*[p._plan.value for p in plans])
    Fp, Up, infos, sts = _queue_arrays(plans, Fs, Us, restart, maxit, tol)
    torch.cuda.synchronize()              # inputs ready before the library's streams start
    st = _lib.helmholtz6_solve_batch_queue(P, Fp, Up, infos, sts, n, int(lanes))
    if st < 0:
        raise H6Error(st, _lib.helmholtz6_last_error(plans[0]._plan).decode() or "queued batch failed")
    return _queue_results(infos, sts, n)


def psi_order(r1_h: float, r2_h: float, r1_gh: float, r2_gh: float, gamma: float) -> float:
    """eq. (PSI) from the first two SKS residual norms on grids h and gamma h."""
    return _lib.helmholtz6_psi_order(float(r1_h), float(r2_h), float(r1_gh), float(r2_gh), float(gamma))


def status_string(status: int) -> str:
    return _lib.helmholtz6_status_string(int(status)).decode()
