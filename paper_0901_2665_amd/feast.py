"""Python binding of libfeast.so (include/feast.h).

Argument marshalling only: every step runs inside the HIP library.  Tensors
are torch.float64 CUDA(HIP) tensors; torch only provides device memory and the
stream.  If the library is not built the binding raises; there is no other
code path.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfeast.so")

_lib = None


class FeastError(RuntimeError):
    def __init__(self, status: int, where: str, lib=None):
        msg = lib.feast_strerror(status).decode() if lib is not None else ""
        super().__init__(f"{where}: status {status} ({msg})")
        self.status = status


class BTMatrix(ctypes.Structure):
    _fields_ = [("nc", ctypes.c_int32), ("b", ctypes.c_int32),
                ("A_diag", ctypes.c_void_p), ("A_up", ctypes.c_void_p),
                ("B_diag", ctypes.c_void_p), ("B_up", ctypes.c_void_p)]


class ZBTMatrix(ctypes.Structure):
    _fields_ = [("nc", ctypes.c_int32), ("b", ctypes.c_int32),
                ("A_diag", ctypes.c_void_p), ("A_up", ctypes.c_void_p),
                ("B_diag", ctypes.c_void_p), ("B_up", ctypes.c_void_p)]


class Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_loops", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("partitions", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("Y0", ctypes.c_void_p),
                ("seed", ctypes.c_uint64), ("verbose", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("loops", ctypes.c_int32), ("M", ctypes.c_int32),
                ("trace", ctypes.c_double), ("trace_rel", ctypes.c_double),
                ("max_res", ctypes.c_double), ("status", ctypes.c_int32),
                ("fallback", ctypes.c_int32),
                ("trace_hist", ctypes.c_double * 64), ("count_hist", ctypes.c_int32 * 64),
                ("rr_sweeps", ctypes.c_int32), ("refine_steps", ctypes.c_int32),
                ("solve_res", ctypes.c_double), ("m0_small", ctypes.c_int32)]


class Problem(ctypes.Structure):
    _fields_ = [("AB", BTMatrix), ("emin", ctypes.c_double), ("emax", ctypes.c_double),
                ("M0", ctypes.c_int32), ("Ne", ctypes.c_int32), ("Y0", ctypes.c_void_p),
                ("lam", ctypes.c_void_p), ("X", ctypes.c_void_p), ("res", ctypes.c_void_p),
                ("info", ctypes.c_void_p), ("status", ctypes.c_int32)]


EXPORTED = ["feast_default_opts", "feast_init", "feast_destroy", "feast_strerror",
            "feast_solve", "feast_contour", "feast_bt_multiply", "feast_shifted_solve",
            "feast_filter", "feast_project", "feast_reduced_eig", "feast_timing",
            "feast_timing_read", "feast_shifted_solve_mixed", "feast_filter_mixed",
            "feast_solve_batched", "feast_autotune_partitions", "feast_random_start",
            "feast_reduced_eig_noalloc", "feast_mlp_create", "feast_mlp_destroy",
            "feast_mlp_params", "feast_mlp_forward", "feast_mlp_gradients",
            "feast_mlp_train_step", "feast_cross_gram", "feast_cross_gram_workspace",
            "feast_tall_gemm", "feast_cell_gram_accumulate", "feast_basis_project",
            "feast_basis_expand", "feast_solve_hermitian", "feast_shifted_solve_hermitian",
            "feast_filter_hermitian"]


def load_library(path: str = LIB_PATH):
    """Load libfeast.so and declare its signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libfeast.so not built ({path}); run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    P, I32, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    lib.feast_default_opts.argtypes = [ctypes.POINTER(Opts)]
    lib.feast_default_opts.restype = None
    lib.feast_init.argtypes = [ctypes.POINTER(P), ctypes.c_int, P]
    lib.feast_destroy.argtypes = [P]
    lib.feast_strerror.argtypes = [ctypes.c_int]
    lib.feast_strerror.restype = ctypes.c_char_p
    lib.feast_solve.argtypes = [P, ctypes.POINTER(BTMatrix), D, D, I32, I32,
                                ctypes.POINTER(Opts), P, P, P, ctypes.POINTER(Info)]
    lib.feast_contour.argtypes = [I32, D, D, P, P, P, P, P, P]
    lib.feast_bt_multiply.argtypes = [P, ctypes.POINTER(BTMatrix), I32, I32, P, P]
    lib.feast_shifted_solve.argtypes = [P, ctypes.POINTER(BTMatrix), D, D, I32, P, P, P, I32]
    lib.feast_filter.argtypes = [P, ctypes.POINTER(BTMatrix), D, D, I32, I32, P, P]
    lib.feast_shifted_solve_mixed.argtypes = [P, ctypes.POINTER(BTMatrix), D, D, I32, P, P, P,
                                              I32, ctypes.POINTER(I32), ctypes.POINTER(D)]
    lib.feast_filter_mixed.argtypes = [P, ctypes.POINTER(BTMatrix), D, D, I32, I32, P, P,
                                       ctypes.POINTER(I32), ctypes.POINTER(D)]
    lib.feast_project.argtypes = [P, ctypes.POINTER(BTMatrix), I32, P, P, P]
    lib.feast_reduced_eig.argtypes = [P, I32, P, P, P, P, ctypes.POINTER(I32)]
    lib.feast_solve_batched.argtypes = [P, ctypes.POINTER(Problem), I32, ctypes.POINTER(Opts),
                                        I32]
    lib.feast_autotune_partitions.argtypes = [P, ctypes.POINTER(BTMatrix), D, D, I32, I32,
                                              ctypes.c_char_p, ctypes.POINTER(I32)]
    lib.feast_reduced_eig_noalloc.argtypes = [P, I32, P, P, P, P, ctypes.POINTER(I32)]
    lib.feast_solve_hermitian.argtypes = [P, ctypes.POINTER(ZBTMatrix), D, D, I32, I32,
                                          ctypes.POINTER(Opts), P, P, P, ctypes.POINTER(Info)]
    lib.feast_shifted_solve_hermitian.argtypes = [P, ctypes.POINTER(ZBTMatrix), D, D, I32, P,
                                                  I32, P, I32]
    lib.feast_filter_hermitian.argtypes = [P, ctypes.POINTER(ZBTMatrix), D, D, I32, I32, P, P]
    F32P = ctypes.c_void_p
    lib.feast_mlp_create.argtypes = [P, ctypes.POINTER(I32), I32, P, ctypes.POINTER(P)]
    lib.feast_mlp_destroy.argtypes = [P]
    lib.feast_mlp_params.argtypes = [P, P]
    lib.feast_mlp_forward.argtypes = [P, I32, P, P]
    lib.feast_mlp_gradients.argtypes = [P, I32, P, P, P, ctypes.POINTER(D)]
    lib.feast_mlp_train_step.argtypes = [P, I32, P, P, ctypes.c_float, ctypes.POINTER(D)]
    lib.feast_cross_gram.argtypes = [P, ctypes.c_int64, I32, I32, P, I32, P, I32, P, P]
    lib.feast_cross_gram_workspace.argtypes = [ctypes.c_int64, I32, I32]
    lib.feast_tall_gemm.argtypes = [P, ctypes.c_int64, I32, I32, P, I32, P, P]
    lib.feast_cell_gram_accumulate.argtypes = [P, I32, I32, I32, P, P]
    lib.feast_basis_project.argtypes = [P, I32, I32, I32, I32, P, P, D, F32P]
    lib.feast_basis_expand.argtypes = [P, I32, I32, I32, I32, P, F32P, D, P, D, P]
    lib.feast_random_start.argtypes = [P, ctypes.c_uint64, ctypes.c_int64, I32, P]
    lib.feast_timing.argtypes = [P, I32]
    lib.feast_timing_read.argtypes = [P, I32, ctypes.POINTER(ctypes.c_char_p),
                                      ctypes.POINTER(D), ctypes.POINTER(ctypes.c_int64)]
    for name in EXPORTED:
        if name not in ("feast_default_opts", "feast_strerror"):
            getattr(lib, name).restype = ctypes.c_int
    lib.feast_cross_gram_workspace.restype = ctypes.c_int64
    _lib = lib
    return lib


def _fptr(t, dtype_name="float32"):
    import torch
    want = {"float32": torch.float32, "float64": torch.float64}[dtype_name]
    if not (t.is_cuda and t.dtype == want and t.is_contiguous()):
        raise ValueError(f"expected a contiguous {dtype_name} device tensor")
    return t.data_ptr()


class Mlp:
    """The warm-start network of feast.h (feast_mlp_*): every product on the
    matrix cores in bfloat16 with float32 sums, Adam in float32."""

    def __init__(self, ctx: "Context", dims, params, max_batch: int = 64):
        self.ctx = ctx
        self.lib = ctx.lib
        self.dims = tuple(int(d) for d in dims)
        self.max_batch = int(max_batch)
        arr = (ctypes.c_int32 * 4)(*self.dims)
        h = ctypes.c_void_p()
        st = self.lib.feast_mlp_create(ctx.handle, arr, self.max_batch, _fptr(params),
                                       ctypes.byref(h))
        if st != 0:
            raise FeastError(st, "feast_mlp_create", self.lib)
        self.handle = h
        self.nparam = params.numel()

    def close(self):
        if getattr(self, "handle", None):
            self.lib.feast_mlp_destroy(self.handle)
            self.handle = None

    def params(self):
        import torch
        out = torch.empty(self.nparam, dtype=torch.float32, device=f"cuda:{self.ctx.device}")
        st = self.lib.feast_mlp_params(self.handle, _fptr(out))
        if st:
            raise FeastError(st, "feast_mlp_params", self.lib)
        return out

    def forward(self, x, out=None):
        import torch
        if out is None:
            out = torch.empty((x.shape[0], self.dims[3]), dtype=torch.float32, device=x.device)
        st = self.lib.feast_mlp_forward(self.handle, x.shape[0], _fptr(x), _fptr(out))
        if st:
            raise FeastError(st, "feast_mlp_forward", self.lib)
        return out

    def gradients(self, x, t):
        import torch
        g = torch.empty(self.nparam, dtype=torch.float32, device=x.device)
        loss = ctypes.c_double(0.0)
        st = self.lib.feast_mlp_gradients(self.handle, x.shape[0], _fptr(x), _fptr(t), _fptr(g),
                                          ctypes.byref(loss))
        if st:
            raise FeastError(st, "feast_mlp_gradients", self.lib)
        return g, loss.value

    def train_step(self, x, t, lr: float, want_loss: bool = True):
        loss = ctypes.c_double(0.0)
        st = self.lib.feast_mlp_train_step(self.handle, x.shape[0], _fptr(x), _fptr(t),
                                           ctypes.c_float(lr),
                                           ctypes.byref(loss) if want_loss else None)
        if st:
            raise FeastError(st, "feast_mlp_train_step", self.lib)
        return loss.value if want_loss else None


def contour(ne: int, emin: float, emax: float):
    """Host-side Gauss-Legendre rule and contour (eqs. 13-15)."""
    lib = load_library()
    out = [np.zeros(ne) for _ in range(6)]
    st = lib.feast_contour(ne, emin, emax, *[o.ctypes.data for o in out])
    if st != 0:
        raise FeastError(st, "feast_contour", lib)
    x, w, zr, zi, kr, ki = out
    return x, w, zr + 1j * zi, kr + 1j * ki


@dataclasses.dataclass
class SolveResult:
    lam: "object"          # torch tensor [M0] (device)
    X: "object"            # torch tensor [N][M0] (device)
    res: "object"          # torch tensor [M0] (device)
    M: int
    loops: int
    trace: float
    trace_rel: float
    max_res: float
    status: int
    fallback: int
    traces: list
    counts: list
    rr_sweeps: int = 0
    refine_steps: int = 0  # precision 1: float32 correction solves; 2: float32 loops
    solve_res: float = 0.0  # precision 1: worst final relative residual of a shifted solve
    m0_small: int = 0       # 1 if M0 < 1.5 M (below the paper's subspace-size guidance)


def _ptr(t):
    import torch
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 device tensor")
    return t.data_ptr()


class Pencil:
    """Device copy of a block-tridiagonal pencil (torch float64 tensors)."""

    def __init__(self, Ad, Au, Bd, Bu, device="cuda"):
        import torch
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64,
                                      device=device).contiguous()
        self.Ad, self.Au, self.Bd, self.Bu = f(Ad), f(Au), f(Bd), f(Bu)
        self.nc, self.b = int(self.Ad.shape[0]), int(self.Ad.shape[1])
        self.n = self.nc * self.b

    @classmethod
    def from_tensors(cls, Ad, Au, Bd, Bu):
        """Wrap float64 device tensors without copying."""
        p = cls.__new__(cls)
        for t in (Ad, Au, Bd, Bu):
            _ptr(t) if t.numel() else None
        p.Ad, p.Au, p.Bd, p.Bu = Ad, Au, Bd, Bu
        p.nc, p.b = int(Ad.shape[0]), int(Ad.shape[1])
        p.n = p.nc * p.b
        return p

    def struct(self) -> BTMatrix:
        up_a = self.Au.data_ptr() if self.Au.numel() else None
        up_b = self.Bu.data_ptr() if self.Bu.numel() else None
        return BTMatrix(self.nc, self.b, self.Ad.data_ptr(), up_a, self.Bd.data_ptr(), up_b)


def _zptr(t):
    import torch
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()):
        raise ValueError("expected a contiguous complex128 device tensor")
    return t.data_ptr()


class HermitianPencil:
    """Device copy of a Hermitian pencil: A complex (complex128), B real."""

    def __init__(self, Ad, Au, Bd, Bu, device="cuda"):
        import torch
        c = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.complex128,
                                      device=device).contiguous()
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64,
                                      device=device).contiguous()
        self.Ad, self.Au, self.Bd, self.Bu = c(Ad), c(Au), f(Bd), f(Bu)
        self.nc, self.b = int(self.Ad.shape[0]), int(self.Ad.shape[1])
        self.n = self.nc * self.b

    def struct(self) -> ZBTMatrix:
        up_a = self.Au.data_ptr() if self.Au.numel() else None
        up_b = self.Bu.data_ptr() if self.Bu.numel() else None
        return ZBTMatrix(self.nc, self.b, self.Ad.data_ptr(), up_a, self.Bd.data_ptr(), up_b)


class Context:
    """A feast_ctx bound to a device and to torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.lib = load_library()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        h = ctypes.c_void_p()
        st = self.lib.feast_init(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream))
        if st != 0:
            raise FeastError(st, "feast_init", self.lib)
        self.handle = h
        self.device = device

    def close(self):
        if getattr(self, "handle", None):
            self.lib.feast_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, where, warn_ok=False):
        if st < 0 or (st > 0 and not warn_ok):
            raise FeastError(st, where, self.lib)
        return st

    def solve(self, p: Pencil, emin: float, emax: float, M0: int, Ne: int, Y0,
              tol: float = 1e-12, max_loops: int = 20, out=None,
              partitions: int = 0, precision: int = 0, graph: int = 0,
              seed: int = 0, verbose: int = 0) -> SolveResult:
        """Y0: device tensor [N][M0], or None for the library's seeded random
        start (Philox4x64-10 + Box-Muller from ``seed``)."""
        import torch
        dev = p.Ad.device
        if out is None:
            lam = torch.empty(M0, dtype=torch.float64, device=dev)
            X = torch.empty((p.n, M0), dtype=torch.float64, device=dev)
            res = torch.empty(M0, dtype=torch.float64, device=dev)
        else:
            lam, X, res = out
        opts = Opts(tol=tol, max_loops=max_loops, precision=precision, partitions=partitions,
                    graph=graph, Y0=_ptr(Y0) if Y0 is not None else None, seed=seed,
                    verbose=verbose)
        info = Info()
        ab = p.struct()
        st = self.lib.feast_solve(self.handle, ctypes.byref(ab), emin, emax, M0, Ne,
                                  ctypes.byref(opts), _ptr(lam), _ptr(X), _ptr(res),
                                  ctypes.byref(info))
        self._check(st, "feast_solve", warn_ok=True)
        n = min(info.loops, 64)
        return SolveResult(lam, X, res, info.M, info.loops, info.trace, info.trace_rel,
                           info.max_res, st, info.fallback, list(info.trace_hist[:n]),
                           list(info.count_hist[:n]), info.rr_sweeps, info.refine_steps,
                           info.solve_res, info.m0_small)

    def solve_batched(self, problems, tol: float = 1e-12, max_loops: int = 20,
                      partitions: int = 0, precision: int = 0, workers: int = 0,
                      graph: int = 0, seed: int = 0):
        """Solve independent problems together.  problems: list of
        (Pencil, emin, emax, M0, Ne, Y0) with Y0 a device tensor.  Returns
        (status, [SolveResult]); a problem's own error is in its result's
        status, an error of the call raises."""
        import torch
        keep, res_list = [], []
        arr = (Problem * len(problems))()
        for i, (p, emin, emax, M0, Ne, Y0) in enumerate(problems):
            dev = p.Ad.device
            lam = torch.empty(M0, dtype=torch.float64, device=dev)
            X = torch.empty((p.n, M0), dtype=torch.float64, device=dev)
            res = torch.empty(M0, dtype=torch.float64, device=dev)
            info = Info()
            keep.append((p, Y0, lam, X, res, info))
            arr[i] = Problem(p.struct(), emin, emax, M0, Ne,
                             _ptr(Y0) if Y0 is not None else None, _ptr(lam), _ptr(X),
                             _ptr(res), ctypes.cast(ctypes.pointer(info), ctypes.c_void_p), 0)
        opts = Opts(tol=tol, max_loops=max_loops, precision=precision, partitions=partitions,
                    graph=graph, Y0=None, seed=seed)
        st = self.lib.feast_solve_batched(self.handle, arr, len(problems), ctypes.byref(opts),
                                          workers)
        if st < 0 and all(arr[i].status != st for i in range(len(problems))):
            raise FeastError(st, "feast_solve_batched", self.lib)  # the call itself failed
        for i, (p, Y0, lam, X, res, info) in enumerate(keep):
            n = min(info.loops, 64)
            res_list.append(SolveResult(lam, X, res, info.M, info.loops, info.trace,
                                        info.trace_rel, info.max_res, arr[i].status,
                                        info.fallback, list(info.trace_hist[:n]),
                                        list(info.count_hist[:n]), info.rr_sweeps,
                                        info.refine_steps, info.solve_res, info.m0_small))
        return st, res_list

    def autotune_partitions(self, p: Pencil, emin: float, emax: float, M0: int, Ne: int,
                            cache_path: str | None = None) -> int:
        """Fastest partition count of the factorisation for this shape (measured)."""
        out = ctypes.c_int32(0)
        ab = p.struct()
        path = cache_path.encode() if cache_path else None
        st = self.lib.feast_autotune_partitions(self.handle, ctypes.byref(ab), emin, emax, M0,
                                                Ne, path, ctypes.byref(out))
        self._check(st, "feast_autotune_partitions")
        return out.value

    def timing(self, enable: bool):
        """Start (clear) or stop hipEvent timing of the kernel classes."""
        self._check(self.lib.feast_timing(self.handle, 1 if enable else 0), "feast_timing")

    def timing_read(self) -> dict:
        """{class name: (total ms, launches)} of the events recorded so far."""
        n = self.lib.feast_timing_read(self.handle, -1, None, None, None)
        out = {}
        for k in range(n):
            name = ctypes.c_char_p()
            ms = ctypes.c_double()
            cnt = ctypes.c_int64()
            st = self.lib.feast_timing_read(self.handle, k, ctypes.byref(name), ctypes.byref(ms),
                                            ctypes.byref(cnt))
            self._check(st, "feast_timing_read")
            out[name.value.decode()] = (ms.value, cnt.value)
        return out

    def bt_multiply(self, p: Pencil, which: int, V):
        import torch
        out = torch.empty_like(V)
        ab = p.struct()
        st = self.lib.feast_bt_multiply(self.handle, ctypes.byref(ab), which, V.shape[1],
                                        _ptr(V), _ptr(out))
        self._check(st, "feast_bt_multiply")
        return out

    # ---- float64 data kernels of the learned warm start ----

    def cross_gram(self, X, V, m: int | None = None, m2: int | None = None):
        """X[:, :m]^T V[:, :m2] (float64, device)."""
        import torch
        N = X.shape[0]
        m = X.shape[1] if m is None else m
        m2 = V.shape[1] if m2 is None else m2
        ws = torch.empty(max(1, int(self.lib.feast_cross_gram_workspace(N, m, m2))),
                         dtype=torch.float64, device=X.device)
        G = torch.empty((m, m2), dtype=torch.float64, device=X.device)
        st = self.lib.feast_cross_gram(self.handle, N, m, m2, _ptr(X), X.shape[1], _ptr(V),
                                       V.shape[1], _ptr(ws), _ptr(G))
        self._check(st, "feast_cross_gram")
        return G

    def tall_gemm(self, X, G, m: int | None = None, out=None):
        import torch
        N = X.shape[0]
        m = X.shape[1] if m is None else m
        if out is None:
            out = torch.empty((N, G.shape[1]), dtype=torch.float64, device=X.device)
        st = self.lib.feast_tall_gemm(self.handle, N, m, G.shape[1], _ptr(X), X.shape[1],
                                      _ptr(G), _ptr(out))
        self._check(st, "feast_tall_gemm")
        return out

    def cell_gram_accumulate(self, nc: int, b: int, T, Gc):
        st = self.lib.feast_cell_gram_accumulate(self.handle, nc, b, T.shape[1], _ptr(T), _ptr(Gc))
        self._check(st, "feast_cell_gram_accumulate")

    def basis_project(self, nc: int, b: int, U, T, scale: float = 1.0, out=None):
        import torch
        r, m = U.shape[2], T.shape[1]
        if out is None:
            out = torch.empty(nc * r * m, dtype=torch.float32, device=T.device)
        st = self.lib.feast_basis_project(self.handle, nc, b, r, m, _ptr(U), _ptr(T), scale,
                                          _fptr(out))
        self._check(st, "feast_basis_project")
        return out

    def basis_expand(self, nc: int, b: int, U, C, m: int, scale: float = 1.0, R=None,
                     rscale: float = 0.0, out=None):
        import torch
        r = U.shape[2]
        if out is None:
            out = torch.empty((nc * b, m), dtype=torch.float64, device=U.device)
        st = self.lib.feast_basis_expand(self.handle, nc, b, r, m, _ptr(U), _fptr(C), scale,
                                         _ptr(R) if R is not None else None, rscale, _ptr(out))
        self._check(st, "feast_basis_expand")
        return out

    # ---- Hermitian A (eq. 12) ----

    def solve_hermitian(self, p: "HermitianPencil", emin: float, emax: float, M0: int, Ne: int,
                        Y0=None, tol: float = 1e-12, max_loops: int = 20, seed: int = 0,
                        verbose: int = 0, partitions: int = 0) -> SolveResult:
        import torch
        dev = p.Ad.device
        lam = torch.empty(M0, dtype=torch.float64, device=dev)
        X = torch.empty((p.n, M0), dtype=torch.complex128, device=dev)
        res = torch.empty(M0, dtype=torch.float64, device=dev)
        opts = Opts(tol=tol, max_loops=max_loops, precision=0, partitions=partitions, graph=0,
                    Y0=_zptr(Y0) if Y0 is not None else None, seed=seed, verbose=verbose)
        info = Info()
        ab = p.struct()
        st = self.lib.feast_solve_hermitian(self.handle, ctypes.byref(ab), emin, emax, M0, Ne,
                                            ctypes.byref(opts), _ptr(lam), _zptr(X), _ptr(res),
                                            ctypes.byref(info))
        self._check(st, "feast_solve_hermitian", warn_ok=True)
        n = min(info.loops, 64)
        return SolveResult(lam, X, res, info.M, info.loops, info.trace, info.trace_rel,
                           info.max_res, st, info.fallback, list(info.trace_hist[:n]),
                           list(info.count_hist[:n]), info.rr_sweeps, 0, 0.0, info.m0_small)

    def shifted_solve_hermitian(self, p: "HermitianPencil", z: complex, R, adjoint: bool = False,
                                partitions: int = 0):
        import torch
        X = torch.empty_like(R)
        ab = p.struct()
        st = self.lib.feast_shifted_solve_hermitian(self.handle, ctypes.byref(ab), z.real, z.imag,
                                                    R.shape[1], _zptr(R), int(adjoint), _zptr(X),
                                                    int(partitions))
        self._check(st, "feast_shifted_solve_hermitian")
        return X

    def filter_hermitian(self, p: "HermitianPencil", emin: float, emax: float, Ne: int, Y):
        import torch
        Q = torch.empty_like(Y)
        ab = p.struct()
        st = self.lib.feast_filter_hermitian(self.handle, ctypes.byref(ab), emin, emax,
                                             Y.shape[1], Ne, _zptr(Y), _zptr(Q))
        self._check(st, "feast_filter_hermitian")
        return Q

    def random_start(self, seed: int, N: int, M0: int):
        """The start block feast_solve draws when Y0 is None (device tensor)."""
        import torch
        Y = torch.empty((N, M0), dtype=torch.float64, device=f"cuda:{self.device}")
        st = self.lib.feast_random_start(self.handle, seed, N, M0, _ptr(Y))
        self._check(st, "feast_random_start")
        return Y

    def shifted_solve(self, p: Pencil, z: complex, R, partitions: int = 0):
        import torch
        xr, xi = torch.empty_like(R), torch.empty_like(R)
        ab = p.struct()
        st = self.lib.feast_shifted_solve(self.handle, ctypes.byref(ab), z.real, z.imag,
                                          R.shape[1], _ptr(R), _ptr(xr), _ptr(xi), partitions)
        self._check(st, "feast_shifted_solve")
        return xr, xi

    def shifted_solve_mixed(self, p: Pencil, z: complex, R, partitions: int = 0):
        """(X_re, X_im, corrections, worst relative residual, status 0 or 5)."""
        import torch
        xr, xi = torch.empty_like(R), torch.empty_like(R)
        steps, rel = ctypes.c_int32(0), ctypes.c_double(0.0)
        ab = p.struct()
        st = self.lib.feast_shifted_solve_mixed(self.handle, ctypes.byref(ab), z.real, z.imag,
                                                R.shape[1], _ptr(R), _ptr(xr), _ptr(xi),
                                                partitions, ctypes.byref(steps),
                                                ctypes.byref(rel))
        self._check(st, "feast_shifted_solve_mixed", warn_ok=True)
        return xr, xi, steps.value, rel.value, st

    def filter_mixed(self, p: Pencil, emin: float, emax: float, Ne: int, Y):
        """(Q, corrections, worst relative residual, status 0 or 5)."""
        import torch
        Q = torch.empty_like(Y)
        steps, rel = ctypes.c_int32(0), ctypes.c_double(0.0)
        ab = p.struct()
        st = self.lib.feast_filter_mixed(self.handle, ctypes.byref(ab), emin, emax, Y.shape[1],
                                         Ne, _ptr(Y), _ptr(Q), ctypes.byref(steps),
                                         ctypes.byref(rel))
        self._check(st, "feast_filter_mixed", warn_ok=True)
        return Q, steps.value, rel.value, st

    def filter(self, p: Pencil, emin: float, emax: float, Ne: int, Y):
        import torch
        Q = torch.empty_like(Y)
        ab = p.struct()
        st = self.lib.feast_filter(self.handle, ctypes.byref(ab), emin, emax, Y.shape[1], Ne,
                                   _ptr(Y), _ptr(Q))
        self._check(st, "feast_filter")
        return Q

    def project(self, p: Pencil, Q):
        import torch
        m0 = Q.shape[1]
        AQ = torch.empty((m0, m0), dtype=torch.float64, device=Q.device)
        BQ = torch.empty_like(AQ)
        ab = p.struct()
        st = self.lib.feast_project(self.handle, ctypes.byref(ab), m0, _ptr(Q), _ptr(AQ),
                                    _ptr(BQ))
        self._check(st, "feast_project")
        return AQ, BQ

    def reduced_eig(self, AQ, BQ):
        import torch
        m0 = AQ.shape[0]
        eps = torch.empty(m0, dtype=torch.float64, device=AQ.device)
        Phi = torch.empty((m0, m0), dtype=torch.float64, device=AQ.device)
        fb = ctypes.c_int32(0)
        st = self.lib.feast_reduced_eig(self.handle, m0, _ptr(AQ.contiguous()),
                                        _ptr(BQ.contiguous()), _ptr(eps), _ptr(Phi),
                                        ctypes.byref(fb))
        self._check(st, "feast_reduced_eig")
        return eps, Phi, bool(fb.value)

    def reduced_eig_noalloc(self, AQ, BQ, eps, Phi):
        """feast_reduced_eig_noalloc into the caller's eps [M0] and Phi [M0][M0]
        (the library allocates nothing); returns the fallback flag."""
        m0 = AQ.shape[0]
        fb = ctypes.c_int32(0)
        st = self.lib.feast_reduced_eig_noalloc(self.handle, m0, _ptr(AQ), _ptr(BQ), _ptr(eps),
                                                _ptr(Phi), ctypes.byref(fb))
        self._check(st, "feast_reduced_eig_noalloc")
        return bool(fb.value)
