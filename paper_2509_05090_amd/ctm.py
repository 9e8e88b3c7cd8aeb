"""Python binding of libctm (ctypes).

Argument marshalling only: every step of the CTMRG runs in the HIP library.
Device memory comes from torch tensors on the GPU and work is enqueued on
torch's current stream.  The names mirror the C interface in include/ctm.h
and include/ctm_kernels.h.  Importing this module loads libctm.so and raises
if it has not been built.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libctm.so")

CTM_OK = 0
CTM_EINVAL = -1
CTM_ENOTSYM = -2
CTM_ENOMEM = -3
CTM_EDEVICE = -4
CTM_ENOTCONV = -5
CTM_ENONFINITE = -6
CTM_ESTATE = -7

PROJ = {"qr": 0, "evd": 1, "qr_chol": 2}
PREC = {"fp64": 0, "fp32": 1, "bf16": 2, "ladder": 3}
DTYPE_CODE = {"float64": 0, "float32": 1, "bfloat16": 2}

EXPORTS = ("ctm_symmetrize", "ctm_init", "ctm_step", "ctm_converge", "ctm_energy",
           "ctm_grad", "ctm_spectrum", "ctm_query", "ctm_get_env", "ctm_set_env",
           "ctm_update_tensor", "ctm_set_precision", "ctm_free", "ctm_last_error", "ctm_gemm",
           "ctm_qr", "ctm_cholesky", "ctm_eigh", "ctm_profile", "ctm_profile_read")
STAGES = ("corner", "projector", "renorm_c", "renorm_t", "big_gemm")


class CtmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libctm error {code}: {msg}")
        self.code = code


class _Config(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("D", ctypes.c_int), ("chi", ctypes.c_int),
                ("proj", ctypes.c_int), ("prec", ctypes.c_int)]


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"libctm.so not built at {path}; run `python -m paper_2509_05090_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i, d, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int64
    pd, pi = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    sig = {
        "ctm_symmetrize": (i, [vp, vp, i, i, vp]),
        "ctm_init": (i, [ctypes.POINTER(vp), ctypes.POINTER(_Config), vp, vp, vp]),
        "ctm_step": (i, [vp, i, pd]),
        "ctm_converge": (i, [vp, d, i, i, pi, pd]),
        "ctm_energy": (i, [vp, pd, pd, pd]),
        "ctm_grad": (i, [vp, pd, i, d, i, vp, pd, pi]),
        "ctm_spectrum": (i, [vp, pd, pi]),
        "ctm_query": (i, [vp, pi, pi, pi]),
        "ctm_get_env": (i, [vp, vp, vp, vp]),
        "ctm_set_env": (i, [vp, i, vp, vp, i, vp]),
        "ctm_update_tensor": (i, [vp, vp]),
        "ctm_set_precision": (i, [vp, i]),
        "ctm_free": (None, [vp]),
        "ctm_last_error": (ctypes.c_char_p, [vp]),
        "ctm_gemm": (i, [i, i, i, i, vp, i64, i, i64, i64, vp, i64, i, i64, i64,
                         vp, i64, i, i64, i64, i, i, d, d, i, vp]),
        "ctm_qr": (i, [vp, i, i, vp, vp, vp]),
        "ctm_cholesky": (i, [vp, i, i, vp, vp, pi, vp]),
        "ctm_eigh": (i, [vp, i, i, vp, vp, pd, vp]),
        "ctm_profile": (i, [vp, i]),
        "ctm_profile_read": (i, [vp, pd, ctypes.POINTER(i64), pd]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = load_library()


def last_error(ctx=None) -> str:
    msg = _lib.ctm_last_error(ctx)
    return msg.decode() if msg else ""


def _check(code: int, ctx=None, allow=()):
    if code != CTM_OK and code not in allow:
        raise CtmError(code, last_error(ctx))
    return code


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "expected a contiguous GPU tensor"
    return ctypes.c_void_p(t.data_ptr())


def symmetrize(raw, out=None):
    """C3v projection + unit-norm normalization of a (d, D, D, D) float64 GPU tensor."""
    import torch
    assert raw.dtype == torch.float64 and raw.dim() == 4
    out = torch.empty_like(raw) if out is None else out
    _check(_lib.ctm_symmetrize(_ptr(raw), _ptr(out), raw.shape[0], raw.shape[1], _stream()))
    return out


def gemm(A, B, C, M, N, K, lda, ldb, ldc, transA=False, transB=False, alpha=1.0, beta=0.0,
         prec=None, batch=(1, 1), sA=(0, 0), sB=(0, 0), sC=(0, 0), ksplit=0):
    """ctm_gemm on torch GPU tensors (see include/ctm_kernels.h)."""
    pa = DTYPE_CODE[str(A.dtype).replace("torch.", "")] if prec is None else prec
    pc = DTYPE_CODE[str(C.dtype).replace("torch.", "")]
    _check(_lib.ctm_gemm(pa, M, N, K, _ptr(A), lda, int(transA), sA[0], sA[1],
                         _ptr(B), ldb, int(transB), sB[0], sB[1],
                         _ptr(C), ldc, pc, sC[0], sC[1], batch[0], batch[1],
                         float(alpha), float(beta), ksplit, _stream()))
    return C


def qr(M):
    """Thin QR of an (n, k) float64 GPU tensor: (Q, R)."""
    import torch
    n, k = M.shape
    Q = torch.empty((n, k), dtype=torch.float64, device=M.device)
    R = torch.empty((k, k), dtype=torch.float64, device=M.device)
    _check(_lib.ctm_qr(_ptr(M.contiguous()), n, k, _ptr(Q), _ptr(R), _stream()))
    return Q, R


def cholesky(G, m):
    """ctm_cholesky on a (k, k) float64 GPU tensor taken as the Gram matrix of
    an m-row matrix: (R, R^{-1}, status bits)."""
    import torch
    k = G.shape[0]
    R = torch.empty((k, k), dtype=torch.float64, device=G.device)
    Ri = torch.empty((k, k), dtype=torch.float64, device=G.device)
    st = ctypes.c_int(0)
    _check(_lib.ctm_cholesky(_ptr(G.contiguous()), k, m, _ptr(R), _ptr(Ri), ctypes.byref(st),
                             _stream()))
    return R, Ri, st.value


def eigh_top(A, k, P=None):
    """ctm_eigh on an (n, n) float64 GPU tensor: (U (n, k) tensor, eigenvalues)."""
    import torch
    n = A.shape[0]
    U = torch.empty((n, k), dtype=torch.float64, device=A.device)
    lam = np.zeros(k)
    _check(_lib.ctm_eigh(_ptr(A.contiguous()), n, k, _ptr(None if P is None else P.contiguous()),
                         _ptr(U), lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream()))
    return U, lam


class Context:
    """One CTMRG run (ctm_init ... ctm_free)."""

    def __init__(self, A, G, chi: int, proj: str = "qr", prec: str = "fp64"):
        import torch
        assert A.dtype == torch.float64 and A.dim() == 4 and A.is_cuda
        d, D = A.shape[0], A.shape[1]
        assert tuple(G.shape) == (chi * D * D, chi) and G.dtype == torch.float64 and G.is_cuda
        self.d, self.D, self.chi = d, D, chi
        cfg = _Config(d, D, chi, PROJ[proj], PREC[prec])
        h = ctypes.c_void_p()
        _check(_lib.ctm_init(ctypes.byref(h), ctypes.byref(cfg), _ptr(A.contiguous()),
                             _ptr(G.contiguous()), _stream()))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.ctm_free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def step(self, n: int = 1, delta: bool = False):
        out = ctypes.c_double(math.nan)
        _check(_lib.ctm_step(self._h, n, ctypes.byref(out) if delta else None), self._h)
        return out.value if delta else None

    def converge(self, tol: float, max_steps: int, n_check: int = 1):
        steps, delta = ctypes.c_int(0), ctypes.c_double(math.nan)
        code = _check(_lib.ctm_converge(self._h, tol, max_steps, n_check, ctypes.byref(steps),
                                        ctypes.byref(delta)), self._h, allow=(CTM_ENOTCONV,))
        return steps.value, delta.value, code == CTM_OK

    def energy(self, h: np.ndarray):
        dd = self.d * self.d
        h = np.ascontiguousarray(h, dtype=np.float64).reshape(dd, dd)
        e = ctypes.c_double(math.nan)
        rho = np.zeros((dd, dd))
        _check(_lib.ctm_energy(self._h, h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               ctypes.byref(e), rho.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               self._h)
        return e.value, rho

    def grad(self, h: np.ndarray, mode: int = 0, tol: float = 1e-12, max_iter: int = 100000):
        """ctm_grad: (g, E, adjoint steps, converged); g is a (d, D, D, D)
        float64 GPU tensor, the symmetric projection of dE/dA."""
        import torch
        dd = self.d * self.d
        h = np.ascontiguousarray(h, dtype=np.float64).reshape(dd, dd)
        g = torch.empty((self.d, self.D, self.D, self.D), dtype=torch.float64, device="cuda")
        e = ctypes.c_double(math.nan)
        it = ctypes.c_int(0)
        code = _check(_lib.ctm_grad(self._h, h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    int(mode), float(tol), int(max_iter), _ptr(g), ctypes.byref(e),
                                    ctypes.byref(it)), self._h, allow=(CTM_ENOTCONV,))
        return g, e.value, it.value, code == CTM_OK

    def spectrum(self) -> np.ndarray:
        s = np.zeros(self.chi)
        n = ctypes.c_int(0)
        _check(_lib.ctm_spectrum(self._h, s.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 ctypes.byref(n)), self._h)
        return s[: n.value].copy()

    def query(self):
        x, st, pr = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(_lib.ctm_query(self._h, ctypes.byref(x), ctypes.byref(st), ctypes.byref(pr)), self._h)
        return x.value, st.value, pr.value

    def get_env(self):
        """(C, T, P) as float64 GPU tensors (P is None before the first truncation)."""
        import torch
        x, _, pr = self.query()
        D2 = self.D * self.D
        dev = torch.device("cuda")
        C = torch.empty((x, x), dtype=torch.float64, device=dev)
        T = torch.empty((x, D2, x), dtype=torch.float64, device=dev)
        P = torch.empty((pr, self.chi), dtype=torch.float64, device=dev) if pr else None
        _check(_lib.ctm_get_env(self._h, _ptr(C), _ptr(T), _ptr(P)), self._h)
        return C, T, P

    def set_env(self, C, T, P=None):
        x = C.shape[0]
        pr = 0 if P is None else P.shape[0]
        _check(_lib.ctm_set_env(self._h, x, _ptr(C.contiguous()), _ptr(T.contiguous()), pr,
                                _ptr(None if P is None else P.contiguous())), self._h)

    def update_tensor(self, A):
        """ctm_update_tensor: a new C3v-symmetric site tensor (same d, D),
        keeping the environment."""
        assert tuple(A.shape) == (self.d, self.D, self.D, self.D)
        _check(_lib.ctm_update_tensor(self._h, _ptr(A.contiguous())), self._h)

    def profile(self, enable: bool = True):
        _check(_lib.ctm_profile(self._h, int(enable)), self._h)

    def profile_read(self):
        """{stage: (ms, intervals)} and the big-product flop count."""
        ms = (ctypes.c_double * len(STAGES))()
        cnt = (ctypes.c_int64 * len(STAGES))()
        fl = ctypes.c_double(0.0)
        _check(_lib.ctm_profile_read(self._h, ms, cnt, ctypes.byref(fl)), self._h)
        return {name: (ms[i], cnt[i]) for i, name in enumerate(STAGES)}, fl.value

    def set_precision(self, prec: str):
        _check(_lib.ctm_set_precision(self._h, PREC[prec]), self._h)


def _energy_function():
    import torch

    class CtmEnergy(torch.autograd.Function):
        """E(A) = Tr(rho h) on the converged QR-CTMRG environment of the
        C3v-symmetric site tensor A; backward multiplies the incoming
        gradient by ctm_grad's fixed-point gradient (symmetric projection of
        dE/dA).  forward(A, G, chi, h, tol, max_steps)."""

        @staticmethod
        def forward(ctx, A, G, chi, h, tol=1e-12, max_steps=20000):
            with Context(A.detach().contiguous(), G, chi) as c:
                c.converge(tol, max_steps, n_check=10)
                g, e, _, _ = c.grad(h, mode=0, tol=tol)
            ctx.save_for_backward(g)
            return torch.tensor(e, dtype=A.dtype, device=A.device)

        @staticmethod
        def backward(ctx, gE):
            (g,) = ctx.saved_tensors
            return gE * g, None, None, None, None, None

    return CtmEnergy


def energy(A, G, chi, h, tol=1e-12, max_steps=20000):
    """Differentiable converged CTMRG energy (torch.autograd.Function)."""
    return _energy_function().apply(A, G, chi, h, tol, max_steps)
