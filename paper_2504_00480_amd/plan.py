"""Python face of the C ABI (include/nfftgp.h): one class per plan.

Device memory and streams come from PyTorch; every numerical step runs in
libnfftgp's HIP kernels.  Names follow the paper: sigma_f, ell, sigma_eps,
bandwidth N, window cutoff m, feature windows W_s.
"""
from __future__ import annotations

import ctypes
from typing import Sequence

import numpy as np
import torch

from . import _lib

GAUSS = 0
MATERN12 = 1
MATERN32 = 2
MQ = 3          # multiquadric (r^2 + c^2)^(1/2), c passed as ell
IMQ = 4         # inverse multiquadric (r^2 + c^2)^(-1/2)
SINC = 5        # sin(c r) / r
SCALE_AUTO = 0
SCALE_NONE = 1
_KERNELS = {"gauss": GAUSS, "gaussian": GAUSS, "matern12": MATERN12, "matern": MATERN12,
            "matern32": MATERN32, "mq": MQ, "multiquadric": MQ, "imq": IMQ,
            "inverse_multiquadric": IMQ, "sinc": SINC}


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class AdditiveKernelPlan:
    """Fast summation plan for fixed points X (n x p) and feature windows.

    Parameters
    ----------
    X : torch.Tensor on a ROCm device, float32 or float64, n x p (row-major).
    windows : list of feature-index lists (disjoint, 1..3 features each).
    kernel : per-window kernel ("gauss" / "matern12" / "matern32" / "mq" / "imq" / "sinc" or
             0 .. 5), or one for all; for mq, imq and sinc the shape parameter c takes the
             place of ell.
    N : per-window bandwidth (power of two), or one for all.
    m : window cutoff (2, 4, 6 or 8).
    scale_mode : SCALE_AUTO (scale each window into [-1/4, 1/4)^d) or SCALE_NONE.
    max_nrhs : largest number of vectors per apply / CG call (<= 64).
    scale : optional (c0, c) -- per window the centre (d_s values) and factor of
        the map x -> c (x - c0) into the box, e.g. taken from another plan's
        ``window_info`` so that both plans share one kernel (scale_mode is then
        ignored).
    """

    def __init__(self, X: torch.Tensor, windows: Sequence[Sequence[int]], kernel, N, m: int,
                 scale_mode: int = SCALE_AUTO, max_nrhs: int = 1, scale=None):
        lib = _lib.load()
        if not X.is_cuda:
            raise ValueError("X must be a device tensor")
        if X.dtype not in (torch.float32, torch.float64):
            raise ValueError("X must be float32 or float64")
        if X.dim() != 2 or X.stride(1) != 1:
            raise ValueError("X must be a row-major n x p matrix")
        self.dtype = X.dtype
        self.device = X.device
        self.prec = 0 if X.dtype == torch.float32 else 1
        self.n, self.p = X.shape
        self.windows = [list(map(int, w)) for w in windows]
        P = len(self.windows)
        self.P = P
        ks = kernel if isinstance(kernel, (list, tuple)) else [kernel] * P
        self.kernel = [(_KERNELS[k.lower()] if isinstance(k, str) else int(k)) for k in ks]
        self.N = [int(x) for x in (N if isinstance(N, (list, tuple)) else [N] * P)]
        self.m = int(m)
        self.max_nrhs = int(max_nrhs)
        ptr = np.zeros(P + 1, dtype=np.int32)
        for s, w in enumerate(self.windows):
            ptr[s + 1] = ptr[s] + len(w)
        idx = np.array([f for w in self.windows for f in w] or [0], dtype=np.int32)
        kt = np.array(self.kernel, dtype=np.int32)
        Ns = np.array(self.N, dtype=np.int32)
        self._stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            if scale is None:
                st = lib.nfftgp_plan_create(ctypes.byref(h), _ptr(X), self.n, self.p, X.stride(0), P,
                                            _np_ptr(ptr), _np_ptr(idx), _np_ptr(kt), _np_ptr(Ns), self.m,
                                            self.prec, int(scale_mode), self.max_nrhs,
                                            ctypes.c_void_p(self._stream.cuda_stream))
            else:
                c0 = np.array([float(v) for s_ in range(P) for v in np.ravel(scale[0][s_])] or [0.0])
                cf = np.array([float(v) for v in scale[1]], dtype=np.float64)
                if c0.shape[0] != max(1, int(ptr[-1])) or cf.shape[0] != P:
                    raise ValueError("scale needs d_s centres and one factor per window")
                st = lib.nfftgp_plan_create_scaled(ctypes.byref(h), _ptr(X), self.n, self.p, X.stride(0), P,
                                                   _np_ptr(ptr), _np_ptr(idx), _np_ptr(kt), _np_ptr(Ns),
                                                   self.m, self.prec, _np_ptr(c0), _np_ptr(cf), self.max_nrhs,
                                                   ctypes.c_void_p(self._stream.cuda_stream))
        _lib.check(st, "nfftgp_plan_create")
        self._h = h
        self.sigma_f = None
        self.ell = None
        self.sigma_eps = None

    # ------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().nfftgp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------
    def set_hyper(self, sigma_f: float, ell, sigma_eps: float):
        """theta = (sigma_f, ell, sigma_eps); ell is one value or one per window."""
        ells = np.array([float(e) for e in (ell if np.ndim(ell) else [ell] * self.P)], dtype=np.float64)
        if ells.shape[0] != self.P:
            raise ValueError("need one ell per window")
        st = _lib.load().nfftgp_set_hyper(self._h, float(sigma_f), _np_ptr(ells), float(sigma_eps))
        _lib.check(st, "nfftgp_set_hyper")
        self.sigma_f, self.ell, self.sigma_eps = float(sigma_f), ells.copy(), float(sigma_eps)

    def window_info(self, s: int) -> dict:
        c0 = np.zeros(3)
        c = ctypes.c_double()
        d = ctypes.c_int32()
        N = ctypes.c_int32()
        mb = ctypes.c_double()
        mbd = ctypes.c_double()
        st = _lib.load().nfftgp_get_window_info(self._h, s, _np_ptr(c0), ctypes.byref(c), ctypes.byref(d),
                                               ctypes.byref(N), ctypes.byref(mb), ctypes.byref(mbd))
        _lib.check(st, "nfftgp_get_window_info")
        return {"c0": c0[: d.value].copy(), "c": c.value, "d": d.value, "N": N.value,
                "min_b": mb.value, "min_bder": mbd.value}

    def profile(self, enable=True):
        """Start (or stop) kernel timing with HIP events: True / False for every
        category or none, or an iterable of category names to time only those
        (each timed launch adds an event pair to the stream)."""
        if isinstance(enable, bool):
            mask = (1 << len(_lib.PROF_NAMES)) - 1 if enable else 0
        else:
            mask = 0
            for name in enable:
                mask |= 1 << _lib.PROF_NAMES.index(name)
        _lib.check(_lib.load().nfftgp_profile(self._h, mask), "nfftgp_profile")

    def profile_read(self) -> dict:
        """{category: (total ms, launches)} since profiling was enabled."""
        ms = np.zeros(len(_lib.PROF_NAMES))
        cnt = np.zeros(len(_lib.PROF_NAMES), dtype=np.int32)
        _lib.check(_lib.load().nfftgp_profile_read(self._h, _np_ptr(ms), _np_ptr(cnt)), "nfftgp_profile_read")
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(_lib.PROF_NAMES)}

    def autotune(self, nrhs: int, derivs: bool = True, reps: int = 3) -> str:
        """Choose spreading subproblem size, vectors per spreading group and the
        interpolation variant per window group by timing applies; returns the report."""
        buf = ctypes.create_string_buffer(4096)
        _lib.check(_lib.load().nfftgp_autotune(self._h, int(nrhs), 1 if derivs else 0, int(reps), buf, 4096),
                   "nfftgp_autotune")
        return buf.value.decode()

    def workspace_bytes(self) -> int:
        b = ctypes.c_size_t()
        _lib.check(_lib.load().nfftgp_get_workspace_bytes(self._h, ctypes.byref(b)), "workspace")
        return int(b.value)

    def describe(self, nrhs: int = 1) -> str:
        """The kernel forms an apply of nrhs vectors takes, one line per window group."""
        buf = ctypes.create_string_buffer(4096)
        _lib.check(_lib.load().nfftgp_describe(self._h, int(nrhs), buf, len(buf)), "nfftgp_describe")
        return buf.value.decode()

    # ------------------------------------------------------------------
    def _check_vec(self, V: torch.Tensor):
        if V.dim() == 1:
            V = V[:, None]
        if V.dtype != self.dtype or V.device != self.device:
            raise ValueError("vectors must match the plan's dtype and device")
        if V.shape[0] != self.n:
            raise ValueError("vectors must have n rows")
        if V.stride(1) != 1:
            V = V.contiguous()
        return V

    def apply(self, V: torch.Tensor, derivs: bool = False, out: torch.Tensor | None = None) -> dict:
        """Khat V; with derivs also dKhat/d ell_s V (P blocks), dKhat/d sigma_f V, dKhat/d sigma_eps V."""
        V = self._check_vec(V)
        nrhs = V.shape[1]
        KV = out if out is not None else torch.empty((self.n, nrhs), dtype=self.dtype, device=self.device)
        dl = dsf = dse = None
        if derivs:
            dl = torch.empty((self.P, self.n, nrhs), dtype=self.dtype, device=self.device)
            dsf = torch.empty((self.n, nrhs), dtype=self.dtype, device=self.device)
            dse = torch.empty((self.n, nrhs), dtype=self.dtype, device=self.device)
        st = _lib.load().nfftgp_apply(self._h, _ptr(V), V.stride(0), nrhs, _ptr(KV), _ptr(dl),
                                      _ptr(dsf), _ptr(dse))
        _lib.check(st, "nfftgp_apply")
        res = {"KV": KV}
        if derivs:
            res.update({"dKV_dell": dl, "dKV_dsf": dsf, "dKV_dse": dse})
        return res

    def col_dots(self, A: torch.Tensor, B: torch.Tensor) -> np.ndarray:
        """FP64 column dot products sum_i A[i, c] B[i, c] on the device."""
        A = self._check_vec(A)
        B = self._check_vec(B)
        out = np.zeros(A.shape[1])
        st = _lib.load().nfftgp_col_dots(self._h, _ptr(A), A.stride(0), _ptr(B), B.stride(0), A.shape[0],
                                         A.shape[1], _np_ptr(out))
        _lib.check(st, "nfftgp_col_dots")
        return out

    # ------------------------------------------------------------------ AAFN
    def attach_precond(self, X: torch.Tensor, per_window: int = 10, max_rank: int = 300, block: int = 100):
        """Attach the additive AFN preconditioner (Sec. 2.3): per_window landmarks
        per window by farthest point sampling, merged up to max_rank; Schur
        complement kept in diagonal blocks of at most `block` points.  X: the
        points the plan was created from."""
        if X.dtype != self.dtype or X.device != self.device or X.shape != (self.n, self.p) or X.stride(1) != 1:
            raise ValueError("X must be the plan's n x p points (same dtype and device)")
        st = _lib.load().nfftgp_precond_attach(self._h, _ptr(X), X.stride(0), int(per_window), int(max_rank),
                                               int(block))
        _lib.check(st, "nfftgp_precond_attach")

    def precond_info(self) -> dict:
        """{'k', 'nblocks', 'logdet' (log det M), 'dlogdet' (tr(M^-1 dM/dtheta_j), theta =
        sigma_f, ell_1..ell_P, sigma_eps)} at the current theta."""
        k = ctypes.c_int32()
        nb = ctypes.c_int32()
        ld = ctypes.c_double()
        dl = np.zeros(self.P + 2)
        st = _lib.load().nfftgp_precond_info(self._h, ctypes.byref(k), ctypes.byref(nb), ctypes.byref(ld),
                                             _np_ptr(dl))
        _lib.check(st, "nfftgp_precond_info")
        return {"k": k.value, "nblocks": nb.value, "logdet": ld.value, "dlogdet": dl}

    def precond_landmarks(self) -> np.ndarray:
        k = ctypes.c_int32()
        _lib.check(_lib.load().nfftgp_precond_info(self._h, ctypes.byref(k), None, None, None), "nfftgp_precond_info")
        idx = np.zeros(max(1, k.value), dtype=np.int32)
        _lib.check(_lib.load().nfftgp_precond_landmarks(self._h, _np_ptr(idx)), "nfftgp_precond_landmarks")
        return idx[: k.value]

    def precond_apply(self, V: torch.Tensor, op: str = "minv") -> torch.Tensor:
        """op = 'minv' (M^-1 V), 'finvt' (F^-T V) or 'f' (F V), M = F F^T."""
        V = self._check_vec(V).contiguous()
        out = torch.empty_like(V)
        code = {"minv": _lib.PC_MINV, "finvt": _lib.PC_FINVT, "f": _lib.PC_F}[op]
        st = _lib.load().nfftgp_precond_apply(self._h, code, _ptr(V), V.shape[1], _ptr(out))
        _lib.check(st, "nfftgp_precond_apply")
        return out

    def precond_dquad(self, W: torch.Tensor) -> np.ndarray:
        """w_c^T dM/dtheta_j w_c, shape (P + 2, columns)."""
        W = self._check_vec(W).contiguous()
        out = np.zeros((self.P + 2, W.shape[1]))
        st = _lib.load().nfftgp_precond_dquad(self._h, _ptr(W), W.shape[1], _np_ptr(out))
        _lib.check(st, "nfftgp_precond_dquad")
        return out

    def cg(self, B: torch.Tensor, tol: float, maxit: int, check_every: int = 8, raise_on=("notpd",),
           out: torch.Tensor | None = None, history: bool = True, precond: bool = False):
        """CG on Khat X = B from zero; returns (X, iters, (alpha, beta) history, rel. residuals, status).
        Passing the same `out` again lets the library replay its captured iteration.  The
        Lanczos history (needs maxit <= MAX_CG_HISTORY) is None with history=False.
        precond=True: CG preconditioned with the attached AAFN preconditioner."""
        B = self._check_vec(B).contiguous()
        nrhs = B.shape[1]
        X = out if out is not None else torch.empty_like(B)
        if X.shape != B.shape or X.dtype != B.dtype or X.device != B.device or not X.is_contiguous():
            raise ValueError("out must be a contiguous tensor like B")
        iters = np.zeros(nrhs, dtype=np.int32)
        if history and maxit > _lib.MAX_CG_HISTORY:
            raise ValueError(f"the Lanczos history holds at most {_lib.MAX_CG_HISTORY} iterations; "
                             "pass history=False for longer solves")
        ab = np.zeros((max(maxit, 1), nrhs, 2)) if history else None
        res = np.zeros(nrhs)
        fn = _lib.load().nfftgp_pcg if precond else _lib.load().nfftgp_cg
        st = fn(self._h, _ptr(B), nrhs, _ptr(X), float(tol), int(maxit), int(check_every),
                _np_ptr(iters), _np_ptr(ab) if history else None, _np_ptr(res))
        if st not in (_lib.OK, _lib.E_NOCONV, _lib.E_NOTPD) or \
                (st == _lib.E_NOTPD and "notpd" in raise_on) or (st == _lib.E_NOCONV and "noconv" in raise_on):
            _lib.check(st, "nfftgp_pcg" if precond else "nfftgp_cg")
        return X, iters, ab, res, st


def slq_logquad(ab: np.ndarray, iters: np.ndarray, znorm2: np.ndarray) -> np.ndarray:
    """z^T logm(Khat) z for each column from its CG coefficients (stochastic Lanczos quadrature)."""
    ab = np.ascontiguousarray(ab, dtype=np.float64)
    maxit, ncol = ab.shape[0], ab.shape[1]
    iters = np.ascontiguousarray(iters, dtype=np.int32)
    zn = np.ascontiguousarray(znorm2, dtype=np.float64)
    out = np.zeros(ncol)
    st = _lib.load().nfftgp_slq_logquad(_np_ptr(ab), _np_ptr(iters), ncol, maxit, _np_ptr(zn), _np_ptr(out))
    _lib.check(st, "nfftgp_slq_logquad")
    return out
